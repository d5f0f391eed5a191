// The sequential chain of cyclic coordinate descent over one block of coordinates, run by one
// wavefront in the covariance form: lane l holds the gradient g_l = x~_l' r / n and coefficient beta_l
// of coordinate l of the block, col(t) returns G[t][lane] (the Gram entry between coordinates t and l).
// A coordinate step t sets beta_t <- S(g_t + beta_t, lambda), d = change, and g <- g - d G[t][.].
//
// chain_fast runs a block on the assumption that every coordinate keeps its status: a nonzero
// coefficient keeps its sign (then d_t = g_t - lambda sign(beta_t)) and a zero coefficient stays zero
// (|g_t| <= lambda at its step, d_t = 0, and the step changes nothing).  Each step is then one FMA on a
// vector of pending changes plus a lane read and a scalar select, instead of the full soft threshold.  The
// assumptions are checked after the block from the values each coordinate had at its own step; if one
// fails the block is not changed and the caller runs chain_exact, the plain sequential chain, from the same
// state.  Both produce the coordinate-descent iterate: a zero coefficient's step is an exact no-op, and a
// kept-sign step differs from the written-out soft threshold only in rounding.
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

// Status-keeping chain; returns false (and changes nothing) if a coordinate would change status.  lam is
// this lane's threshold, as in chain_exact.
// The loop carries the pending changes dv_l = g_l - lambda sign(beta_l) (sign -1 for beta_l = 0) of every
// lane: step t reads d_t = dv_t, or +0 when coefficient t is zero (a scalar select on the wave-uniform set of
// nonzero coefficients), and subtracts d_t G[t][.]; the gradient is dv + lambda sign(beta).  Lane t's dv
// before step t is kept in ds: for a nonzero coefficient it is the change taken, for a zero one its gradient
// at its own step less lambda sign, so the check that the coefficient stays zero, |g_t| <= lambda there, is
// exact.
template <int NB, typename Col>
__device__ __forceinline__ bool chain_fast(double& gl, double& bv, Col col, double lam, int bl, double& dl,
                                           double& wmax) {
    const int lane = threadIdx.x & 63;
    const uint64_t lanes = chain_below(bl);
    const uint64_t amask = __ballot(bv != 0.0) & lanes;
    const bool act = (amask >> lane) & 1ull;
    const double ls = bv > 0.0 ? lam : -lam;
    double dv = gl - ls;
    double w0 = 0.0, w1 = 0.0, ds = 0.0;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        ds = lane == t ? dv : ds;
        const double dr = chain_readlane(dv, t);
        const double d = ((amask >> t) & 1ull) ? dr : 0.0;
        dv = fma(-d, col(t), dv);
        if (t & 1) w1 = fmax(w1, fabs(d));
        else w0 = fmax(w0, fabs(d));
    }
    // a zero coefficient whose gradient at its step exceeds its threshold would move
    uint64_t viol = __ballot(!act && fabs(ds + ls) > lam) & lanes;
    ds = act ? ds : 0.0;
    const double bn = bv + ds;
    // nonzero coefficients must keep their sign
    viol |= __ballot(bv > 0.0 ? !(bn > 0.0) : (bv < 0.0 ? !(bn < 0.0) : false)) & lanes;
    if (viol) return false;
    gl = dv + ls;
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

// The status-keeping chain for a wave that runs the blocks one after the other: chain_fast's step loop, whose
// checks need no sums over the steps, followed only by the next block's first update: the block's changes are
// stored to dsh (NB doubles of LDS, 16-byte aligned, written and read by this wave only) and read back as
// broadcasts, gn(t) returns the Gram entry between coordinate t of this block and this lane's coordinate of
// the next block, and un receives sum_t gn(t) d_t (even and odd t summed separately, then added).  wmax
// receives max(wmax, |change|) of this lane alone: the caller takes the maximum over the wave when it needs
// the largest change.
template <int NB, typename Col, typename ColN>
__device__ __forceinline__ bool chain_fast_next(double& gl, double& bv, Col col, ColN gn, double lam, int bl,
                                                double& dl, double& wmax, double* dsh, double& un) {
    const int lane = threadIdx.x & 63;
    const uint64_t lanes = chain_below(bl);
    const uint64_t amask = __ballot(bv != 0.0) & lanes;
    const bool act = (amask >> lane) & 1ull;
    const double ls = bv > 0.0 ? lam : -lam;
    double dv = gl - ls;
    double ds = 0.0;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        ds = lane == t ? dv : ds;
        const double dr = chain_readlane(dv, t);
        const double d = ((amask >> t) & 1ull) ? dr : 0.0;
        dv = fma(-d, col(t), dv);
    }
    uint64_t viol = __ballot(!act && fabs(ds + ls) > lam) & lanes;
    ds = act ? ds : 0.0;
    const double bn = bv + ds;
    viol |= __ballot(bv > 0.0 ? !(bn > 0.0) : (bv < 0.0 ? !(bn < 0.0) : false)) & lanes;
    if (viol) return false;
    if (lane < NB) dsh[lane] = ds;
    un = chain_next_update<NB>(gn, dsh);
    gl = dv + ls;
    bv = bn;
    dl = ds;
    wmax = fmax(wmax, fabs(ds));
    return true;
}

}  // namespace blk
