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

// Plain chain over steps t < bl: soft threshold written out, one coordinate after the other.
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
            const double u = gt + bt;
            const double bn = u - fmin(fmax(u, -lam), lam);  // S(u, lambda)
            const double d = bn - bt;
            gl = fma(-d, col(t), gl);
            bv = lane == t ? bn : bv;
            dl = lane == t ? d : dl;
            wmax = fmax(wmax, fabs(d));
        }
    }
}

// Status-keeping chain; returns false (and changes nothing) if a coordinate might change status.
// The loop carries only the pending changes dv_l = g_l - lambda sign(beta_l) (sign -1 for beta_l = 0):
// a taken step reads d_t = dv_t and subtracts d_t G[t][.]; the gradient is dv + lambda sign(beta).
// A zero coefficient l is stepped over; it is certain to stay zero if |g_l| at the end of the block
// plus sum_t |d_t G[t][l]| (a bound on how far the block moved g_l) is at most lambda.
template <int NB, typename Col>
__device__ __forceinline__ bool chain_fast(double& gl, double& bv, Col col, double lam, int bl, double& dl,
                                           double& wmax) {
    const int lane = threadIdx.x & 63;
    const uint64_t lanes = chain_below(bl);
    const uint64_t amask = __ballot(bv != 0.0) & lanes;
    const double ls = bv > 0.0 ? lam : -lam;
    double dv = gl - ls;
    double dsv[NB];   // the changes, wave-uniform
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        // a zero coefficient's step is the exact no-op d = 0 (selected, not branched around)
        const double r = chain_readlane(dv, t);
        const double d = ((amask >> t) & 1ull) ? r : 0.0;
        dv = fma(-d, col(t), dv);
        dsv[t] = d;
    }
    // checks and per-lane results: no step depends on another here
    double b0 = 0.0, b1 = 0.0, w0 = 0.0, w1 = 0.0, ds = 0.0;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        const double d = fabs(dsv[t]);
        if (t & 1) {
            b1 = fma(d, fabs(col(t)), b1);
            w1 = fmax(w1, d);
        } else {
            b0 = fma(d, fabs(col(t)), b0);
            w0 = fmax(w0, d);
        }
        ds = lane == t ? dsv[t] : ds;
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

}  // namespace blk
