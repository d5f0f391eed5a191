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
// step differs from the written-out soft threshold only in rounding.
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

// The status-keeping chain for a wave that runs the blocks one after the other.  Only the dependency chain
// is inside the step loop: the lane read of the masked pending changes and one FMA, plus a select that
// keeps step t's change in lane t of ds.  The full pending-change vector, the bound sums and the largest
// change are formed after the loop from ds, stored to dsh (NB doubles of LDS, 16-byte aligned, written and
// read by this wave only) and read back as broadcasts, with the same operations in the same order as the
// step-by-step form, so the results are identical.  The next block's first update is folded into that
// post-pass: gn(t) returns the Gram entry between coordinate t of this block and this
// lane's coordinate of the next block, and un receives sum_t gn(t) d_t (even and odd t summed separately,
// then added).
template <int NB, typename Col, typename ColN>
__device__ __forceinline__ bool chain_fast_next(double& gl, double& bv, Col col, ColN gn, double lam, int bl,
                                                double& dl, double& wmax, double* dsh, double& un) {
    const int lane = threadIdx.x & 63;
    const uint64_t lanes = chain_below(bl);
    const uint64_t amask = __ballot(bv != 0.0) & lanes;
    const bool act = (amask >> lane) & 1ull;
    const double ls = bv > 0.0 ? lam : -lam;
    const double dv0 = gl - ls;
    double dm = act ? dv0 : 0.0;
    double ds = 0.0;
    // the Gram entries of the masked copy: zero on the lanes of zero coefficients, so those lanes stay +0
    // (every lane runs the loop: a lane read of a lane outside the running set would be undefined)
    double cm[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) cm[t] = act ? col(t) : 0.0;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        // step t's change is lane t of dm before the step: keep it there, then broadcast it
        ds = lane == t ? dm : ds;
        const double d = chain_readlane(dm, t);   // +0 for a zero coefficient: its lane of dm stays +0
        dm = fma(-d, cm[t], dm);
    }
    if (lane < NB) dsh[lane] = ds;
    double dv = dv0, b0 = 0.0, b1 = 0.0, w0 = 0.0, w1 = 0.0, u0 = 0.0, u1 = 0.0;
#pragma unroll
    for (int t = 0; t < NB; t += 2) {
        const double2 d2 = *reinterpret_cast<const double2*>(dsh + t);
        const double c0 = col(t), c1 = col(t + 1);
        dv = fma(-d2.x, c0, dv);
        dv = fma(-d2.y, c1, dv);
        b0 = fma(fabs(d2.x), fabs(c0), b0);
        w0 = fmax(w0, fabs(d2.x));
        b1 = fma(fabs(d2.y), fabs(c1), b1);
        w1 = fmax(w1, fabs(d2.y));
        u0 = fma(gn(t), d2.x, u0);
        u1 = fma(gn(t + 1), d2.y, u1);
    }
    un = u0 + u1;
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
// summed separately, then added: the update chain_fast_next folds into its post-pass
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

}  // namespace blk
