// The sequential chain of cyclic coordinate descent over one block of coordinates, run by one
// wavefront in the covariance form: lane l holds the gradient g_l = x~_l' r / n and coefficient beta_l
// of coordinate l of the block, col(t) returns G[t][lane] (the Gram entry between coordinates t and l).
// A coordinate step t sets beta_t <- S(g_t + beta_t, lambda), d = change, and g <- g - d G[t][.].
//
// chain_fast runs a block on the assumption that every coordinate keeps its status: a nonzero
// coefficient keeps its sign (then d_t = g_t - lambda sign(beta_t)) and a zero coefficient stays zero
// (|g_t| <= lambda at its step, d_t = 0, and the step is skipped).  Each taken step is then one FMA on a
// vector of pending changes plus a lane read and a select, instead of the full soft threshold.  The
// assumptions are checked after the block (conservatively for the zero coefficients); if one may fail
// the block is not changed and the caller runs chain_exact, the plain sequential chain, from the same
// state.  Both produce the coordinate-descent iterate: skipped steps are exact no-ops, and a kept-sign
// step differs from the written-out soft threshold only in rounding.  chain_fast_next, the form of the
// multi-workgroup solve, checks the zero coefficients exactly (on their gradients at their own steps) and
// also forms the next block's first update in its step loop.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace blk {

__device__ __forceinline__ double chain_readlane(double v, int lane) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, lane);
    const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint64_t chain_below(int t) { return t >= 64 ? ~0ull : ((1ull << t) - 1ull); }

// Plain chain over steps t < bl: soft threshold written out, one coordinate after the other.  lam is
// this lane's threshold (the same in every lane unless the penalty weights differ); step t uses lane t's.
template <int NB, typename Col>
__device__ __forceinline__ void chain_exact(double& gl, double& bv, Col col, double lam, int bl, double& dl,
                                            double& wmax) {
    const int lane = threadIdx.x & 63;
    const double bv0 = bv;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        if (t < bl) {
            const double gt = chain_readlane(gl, t);
            const double bt = chain_readlane(bv0, t);
            const double lt = chain_readlane(lam, t);
            const double u = gt + bt;
            const double bn = u - fmin(fmax(u, -lt), lt);  // S(u, lambda_t)
            const double d = bn - bt;
            gl = fma(-d, col(t), gl);
            bv = lane == t ? bn : bv;
            dl = lane == t ? d : dl;
            wmax = fmax(wmax, fabs(d));
        }
    }
}

// Status-keeping chain; returns false (and changes nothing) if a coordinate might change status.  lam is
// this lane's threshold, as in chain_exact.
// The loop carries the pending changes dv_l = g_l - lambda sign(beta_l) (sign -1 for beta_l = 0): a taken
// step reads d_t = dv_t and subtracts d_t G[t][.]; the gradient is dv + lambda sign(beta).  The step's lane
// read comes from a masked copy dm that is held at zero on the lanes of zero coefficients (their Gram
// entries are zeroed in its update), so a zero coefficient's step reads d = 0 without a scalar select on
// the dependency chain; the full vector dv, the bound sums and the per-lane changes are updated beside it
// with the same operations in the same order.  A zero coefficient l is certain to stay zero if |g_l| at
// the end of the block plus sum_t |d_t G[t][l]| (a bound on how far the block moved g_l) is at most lambda.
template <int NB, typename Col>
__device__ __forceinline__ bool chain_fast(double& gl, double& bv, Col col, double lam, int bl, double& dl,
                                           double& wmax) {
    const int lane = threadIdx.x & 63;
    const uint64_t lanes = chain_below(bl);
    const uint64_t amask = __ballot(bv != 0.0) & lanes;
    const bool act = (amask >> lane) & 1ull;
    const double ls = bv > 0.0 ? lam : -lam;
    double dv = gl - ls;
    double dm = act ? dv : 0.0;
    double b0 = 0.0, b1 = 0.0, w0 = 0.0, w1 = 0.0, ds = 0.0;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        const double d = chain_readlane(dm, t);   // +0 for a zero coefficient: its lane of dm stays +0
        const double c = col(t);
        dm = fma(-d, act ? c : 0.0, dm);
        dv = fma(-d, c, dv);
        const double ad = fabs(d);
        if (t & 1) {
            b1 = fma(ad, fabs(c), b1);
            w1 = fmax(w1, ad);
        } else {
            b0 = fma(ad, fabs(c), b0);
            w0 = fmax(w0, ad);
        }
        ds = lane == t ? d : ds;
    }
    const double g2 = dv + ls;
    uint64_t viol = __ballot(fabs(g2) + (b0 + b1) > lam) & ~amask & lanes;
    const double bn = bv + ds;
    // nonzero coefficients must keep their sign
    viol |= __ballot(bv > 0.0 ? !(bn > 0.0) : (bv < 0.0 ? !(bn < 0.0) : false)) & lanes;
    if (viol) return false;
    gl = g2;
    bv = bn;
    dl = ds;
    wmax = fmax(wmax, fmax(w0, w1));
    return true;
}

// sum_t gn(t) dsh[t] over a block's changes dsh (NB doubles of LDS read as broadcasts), even and odd t
// summed separately, then added: the next block's first update in the order chain_fast_next sums it in its
// step loop, for blocks that chain_exact ran
template <int NB, typename ColN>
__device__ __forceinline__ double chain_next_update(ColN gn, const double* dsh) {
    double u0 = 0.0, u1 = 0.0;
#pragma unroll
    for (int t = 0; t < NB; t += 2) {
        const double2 d2 = *reinterpret_cast<const double2*>(dsh + t);
        u0 = fma(gn(t), d2.x, u0);
        u1 = fma(gn(t + 1), d2.y, u1);
    }
    return u0 + u1;
}

// The status-keeping chain for a wave that runs the blocks one after the other, everything in the step loop:
// only the lane read of the masked pending changes dm and one FMA are on the dependency chain (dm is held
// at +0 on the lanes of zero coefficients, whose Gram entries are multiplied by 0, so their steps read
// d = +0).  Beside them the full vector dv takes the same updates, lane t's dv before step t is kept in ds
// (for a nonzero coefficient the change taken, for a zero one its gradient at its own step less lambda sign,
// so the check that it stays zero is exact), and the next block's first update grows by gn(t) d_t (gn(t):
// the Gram entry between coordinate t of this block and this lane's coordinate of the next block; even and
// odd t summed separately, then added, the order of chain_next_update).  wmax receives max(wmax, |change|)
// of this lane alone: the caller takes the maximum over the wave when it needs the largest change.
template <int NB, typename Col, typename ColN>
__device__ __forceinline__ bool chain_fast_next(double& gl, double& bv, Col col, ColN gn, double lam, int bl,
                                                double& dl, double& wmax, double& un) {
    const int lane = threadIdx.x & 63;
    const uint64_t lanes = chain_below(bl);
    const uint64_t amask = __ballot(bv != 0.0) & lanes;
    const bool act = (amask >> lane) & 1ull;
    const double ls = bv > 0.0 ? lam : -lam;
    const double af = act ? 1.0 : 0.0;
    double dv = gl - ls;
    double dm = act ? dv : 0.0;
    double ds = 0.0, u0 = 0.0, u1 = 0.0;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        ds = lane == t ? dv : ds;
        const double d = chain_readlane(dm, t);   // +0 for a zero coefficient
        const double c = col(t);
        dm = fma(-d, c * af, dm);
        dv = fma(-d, c, dv);
        // the update is taken at its step (an empty asm keeps the scheduler from holding every step's d in
        // scalar registers until the end of the loop)
        if (t & 1) {
            u1 = fma(gn(t), d, u1);
            asm volatile("" : "+v"(u1));
        } else {
            u0 = fma(gn(t), d, u0);
            asm volatile("" : "+v"(u0));
        }
    }
    uint64_t viol = __ballot(!act && fabs(ds + ls) > lam) & lanes;
    ds = act ? ds : 0.0;
    const double bn = bv + ds;
    viol |= __ballot(bv > 0.0 ? !(bn > 0.0) : (bv < 0.0 ? !(bn < 0.0) : false)) & lanes;
    if (viol) return false;
    un = u0 + u1;
    gl = dv + ls;
    bv = bn;
    dl = ds;
    wmax = fmax(wmax, fabs(ds));
    return true;
}

}  // namespace blk
