// Coordinate descent with covariance updates on the working set.
//
// For the working set E (m features, ascending) the solve keeps the gradient
// g_e = x~_{E[e]}' r / n instead of the residual.  A coordinate step
//   u = g_e + beta_e,  beta_e' = S(u, lambda),  d = beta_e' - beta_e,
//   g_k -= d * G[k, e]  for every k in E,   G = X~_E' X~_E / n,
// is the same cyclic coordinate descent as the residual form (the same
// iterates up to rounding), but a step touches m numbers instead of n.
//
// G comes from a Gram "pool": every feature that has ever been in a working
// set along the path keeps its row of Gram entries, computed once with the
// simplified identity  x~_j' x~_k = (sum_i x_ij x_ik - n c_j c_k)/(s_j s_k)
// (type (1) of the paper's Section 3.1.1).  New members of E get their
// entries against the whole pool by a tiled FP64 GEMM; G_E is then gathered.
//
// The sequential part runs in blocks of GCD_B coordinates: one wavefront
// carries the chain of a block with the block's own Gram entries in LDS
// (lane l holds g of coordinate b0+l; each step broadcasts g_t, computes d,
// updates every lane).  Then the whole workgroup pushes the block's changes
// into the gradient of every other coordinate.  After the solve the residual
// is brought up to date in one pass, r -= X~_E (beta_E - beta_E(start)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <stdint.h>

#include "chain.h"
#include "internal.h"

namespace blk {

namespace {

constexpr int WAVE = 64;


template <typename XT>
__device__ __forceinline__ double ld_x(const XT* p) { return (double)*p; }

// ---- pool membership ---------------------------------------------------------------------------------
// Features of set[0..len) without a pool slot get slots pool_size, pool_size+1, ... in set order.
__global__ __launch_bounds__(1024) void k_pool_add(const int32_t* __restrict__ set, const int64_t* __restrict__ len_dev,
                                                   int64_t len_host, int32_t* __restrict__ pool_pos,
                                                   int32_t* __restrict__ pool_list, int64_t pool_size,
                                                   int64_t* __restrict__ n_new_out) {
    __shared__ int32_t sh[1024];
    __shared__ int64_t carry;
    const int64_t len = len_dev ? *len_dev : len_host;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < len; b0 += blockDim.x) {
        const int64_t t = b0 + threadIdx.x;
        int32_t j = -1;
        int flag = 0;
        if (t < len) {
            j = set[t];
            flag = pool_pos[j] < 0 ? 1 : 0;
        }
        sh[threadIdx.x] = flag;
        __syncthreads();
        for (int off = 1; off < (int)blockDim.x; off <<= 1) {
            int add = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (flag) {
            const int64_t pos = pool_size + carry + sh[threadIdx.x] - 1;
            pool_pos[j] = (int32_t)pos;
            pool_list[pos] = j;
        }
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry += sh[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_new_out = carry;
}

// ---- Gram entries of new pool members ----------------------------------------------------------------
// C[k, t] = x~_{pool[k]}' x~_{pool[P0 + t]} / n for k < P, t < N, written to G[k, P0+t] and G[P0+t, k].
// The raw products sum_i x_{pool[k], i} x_{pool[P0+t], i} (over the fitted rows) are formed on FP64 matrix
// cores (v_mfma_f64_16x16x4f64).  A workgroup holds a 32 x 16 tile of C; its four waves take a quarter of
// the rows each (64 rows a step, the next step's values loaded while the current one is multiplied) and
// their partial tiles are added in wave order through LDS.  Lane (m, kq) feeds rows i0 + 16 kq ..
// i0 + 16 kq + 15 of pool columns kb + m and kb + 16 + m and of new column tb + m, read straight from X;
// register q of its result holds C[kb + kq + 4q (+ 16), tb + m].  The standardization
// (C - n c_k c_t) / (n s_k s_t) is applied on the way out.  A pair of two new columns appears in two tiles;
// only the one with k - P0 <= t writes it (both triangles), so G stays exactly symmetric.
typedef double f64x4 __attribute__((ext_vector_type(4)));
constexpr int GM_W = 4;    // waves per workgroup (row quarters)
constexpr int GM_K = 32;   // pool columns per workgroup
constexpr int GM_N = 16;   // new columns per workgroup
constexpr int GM_R = 64;   // rows per step

// keeps the loads above it issued before the work below it: neither the IR passes (memory clobber) nor the
// machine scheduler (sched_barrier) move them down to their first use
__device__ __forceinline__ void issue_fence_g() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

// 16 consecutive elements of a column, read as 16-byte words (p 16-byte aligned)
template <typename XT>
__device__ __forceinline__ void load16(const XT* p, XT (&dst)[16]) {
    typedef int v4w __attribute__((ext_vector_type(4)));
    constexpr int NV = 16 * (int)sizeof(XT) / 16;
    v4w t[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) t[i] = reinterpret_cast<const v4w*>(p)[i];
    __builtin_memcpy(dst, t, sizeof(t));
}

// VEC: columns and the row mask are 16-byte aligned; every step whose 64 rows lie below n_total then reads
// each lane's 16 values with plain 16-byte loads (no per-element test), the next step's loads in flight during
// the current step's matrix-core work; only a final partial step takes the element-wise guarded path.  The
// operands and the matrix-core sequence are the same either way.
template <typename XT, bool MASK, bool VEC>
__global__ __launch_bounds__(64 * GM_W) void k_gram_update(const XT* __restrict__ X, int64_t ldx, int64_t n_total,
                                                          const uint8_t* __restrict__ mask,
                                                          const int32_t* __restrict__ pool_list, int64_t P,
                                                          int64_t P0, int64_t N, const double* __restrict__ c,
                                                          const double* __restrict__ s, double n_rows,
                                                          double* __restrict__ G, int64_t ldg) {
    __shared__ f64x4 red[GM_W - 1][2][WAVE];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int m = lane & 15, kq = lane >> 4;
    const int64_t kb = (int64_t)blockIdx.x * GM_K, tb = (int64_t)blockIdx.y * GM_N;
    const XT* ac[2];
    bool aok[2];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        const int64_t k = kb + 16 * f + m;
        aok[f] = k < P;
        ac[f] = X + (int64_t)(aok[f] ? pool_list[k] : 0) * ldx;
    }
    const bool bok = tb + m < N;
    const XT* bc = X + (int64_t)(bok ? pool_list[P0 + tb + m] : 0) * ldx;
    // this wave's steps
    const int64_t ns = (n_total + GM_R - 1) / GM_R;
    const int64_t s0 = ns * w / GM_W, s1 = ns * (w + 1) / GM_W;
    XT ra[2][16], rb[16];
    bool rm[16];
    auto load = [&](int64_t step) {
        const int64_t r0 = step * GM_R + 16 * kq;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const bool in = r0 + q < n_total;
            ra[0][q] = (aok[0] && in) ? ac[0][r0 + q] : (XT)0;
            ra[1][q] = (aok[1] && in) ? ac[1][r0 + q] : (XT)0;
            rb[q] = (bok && in) ? bc[r0 + q] : (XT)0;
            rm[q] = MASK ? (in && mask[r0 + q] != 0) : true;
        }
    };
    f64x4 acc[2] = {(f64x4){0.0, 0.0, 0.0, 0.0}, (f64x4){0.0, 0.0, 0.0, 0.0}};
    auto step_mfma = [&]() {
        double av[2][16], bv[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            av[0][q] = (double)ra[0][q];
            av[1][q] = (double)ra[1][q];
            bv[q] = rm[q] ? (double)rb[q] : 0.0;
        }
        return [=, &acc]() {
#pragma unroll
            for (int st = 0; st < 16; ++st) {
                acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[0][st], bv[st], acc[0], 0, 0, 0);
                acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[1][st], bv[st], acc[1], 0, 0, 0);
            }
        };
    };
    int64_t sg = s0;   // first step of the guarded path
    if constexpr (VEC) {
        // full steps: whole 16-row segments for every lane
        auto load_full = [&](int64_t step) {
            const int64_t r0 = step * GM_R + 16 * kq;
            load16<XT>(ac[0] + r0, ra[0]);
            load16<XT>(ac[1] + r0, ra[1]);
            load16<XT>(bc + r0, rb);
            if constexpr (MASK) {
                typedef int v4w __attribute__((ext_vector_type(4)));
                const v4w mw = *reinterpret_cast<const v4w*>(mask + r0);
#pragma unroll
                for (int q = 0; q < 16; ++q) rm[q] = ((mw[q >> 2] >> (8 * (q & 3))) & 0xff) != 0;
            } else {
#pragma unroll
                for (int q = 0; q < 16; ++q) rm[q] = true;
            }
        };
        const int64_t nfs = n_total / GM_R;
        const int64_t f1 = s1 < nfs ? s1 : nfs;
        if (s0 < f1) load_full(s0);
        for (int64_t step = s0; step < f1; ++step) {
            auto run = step_mfma();                          // the current step's operands, converted
            load_full(step + 1 < f1 ? step + 1 : f1 - 1);   // unconditional (the last full step reloads)
            issue_fence_g();
            run();
        }
        sg = s0 > f1 ? s0 : f1;
    }
    if (sg < s1) load(sg);
    for (int64_t step = sg; step < s1; ++step) {
        auto run = step_mfma();
        if (step + 1 < s1) load(step + 1);
        run();
    }
    if (w > 0) {
        red[w - 1][0][lane] = acc[0];
        red[w - 1][1][lane] = acc[1];
    }
    __syncthreads();
    if (w > 0) return;
#pragma unroll
    for (int v = 0; v < GM_W - 1; ++v) {
        acc[0] += red[v][0][lane];
        acc[1] += red[v][1][lane];
    }
    const int64_t t = tb + m;
    if (t >= N) return;
    const int jt = pool_list[P0 + t];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t k = kb + 16 * f + kq + 4 * q;
            if (k >= P) continue;
            if (k >= P0 && k - P0 > t) continue;   // written by the tile of its mirror
            const int jk = pool_list[k];
            const double gv = (acc[f][q] - n_rows * (c[jk] * c[jt])) / (n_rows * (s[jk] * s[jt]));
            G[k * ldg + (P0 + t)] = gv;
            G[(P0 + t) * ldg + k] = gv;
        }
    }
}

// The same update for int8 codes on the int8 matrix cores.  The raw cross-products sum_i x_ik x_it over the
// fitted rows are integers: the int32 sums of v_mfma_i32_16x16x64_i8 (moved to FP64 after every 128 rows) are
// exact, as are the FP64 kernel's sums (every partial sum is an integer below 2^53), so both kernels produce
// the same Gram entries bit for bit.  Lane (m, kq) loads 16 consecutive codes of its column (rows 16 kq .. of a
// 64-row step) and hands the word to the matrix cores as it is.  Columns, ldx and the row mask are 16-byte
// aligned; the word holding the last row is read whole (it lies within the column's padded length; a row mask
// is taken here only when n_total is a multiple of 16, so its words end at row n_total), and its rows past
// n_total, like the rows outside the fit, are cleared in the B operand.  The output layout of this
// instruction is row 4 kq + q (the FP64 one above is kq + 4 q).
typedef int i32x4 __attribute__((ext_vector_type(4)));
constexpr int GI_R = 64;   // rows per int8 step

// 0xFF in each nonzero byte of v, 0x00 elsewhere
__device__ __forceinline__ uint32_t bytes_nonzero(uint32_t v) {
    const uint32_t h = (((v & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | v) & 0x80808080u;
    return (h >> 7) * 0xFFu;
}
// 0xFF in the first nv bytes (nv clamped to 0..4)
__device__ __forceinline__ uint32_t bytes_below(int64_t nv) {
    return nv >= 4 ? 0xFFFFFFFFu : (nv <= 0 ? 0u : ((1u << (8 * (int)nv)) - 1u));
}

template <bool MASK>
__global__ __launch_bounds__(64 * GM_W) void k_gram_update_i8(const int8_t* __restrict__ X, int64_t ldx,
                                                             int64_t n_total, const uint8_t* __restrict__ mask,
                                                             const int32_t* __restrict__ pool_list, int64_t P,
                                                             int64_t P0, int64_t N, const double* __restrict__ c,
                                                             const double* __restrict__ s, double n_rows,
                                                             double* __restrict__ G, int64_t ldg) {
    __shared__ f64x4 red[GM_W - 1][2][WAVE];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int m = lane & 15, kq = lane >> 4;
    const int64_t kb = (int64_t)blockIdx.x * GM_K, tb = (int64_t)blockIdx.y * GM_N;
    const int8_t* ac[2];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        const int64_t k = kb + 16 * f + m;
        ac[f] = X + (int64_t)(k < P ? pool_list[k] : 0) * ldx;
    }
    const bool bok = tb + m < N;
    const int8_t* bc = X + (int64_t)(bok ? pool_list[P0 + tb + m] : 0) * ldx;
    const int64_t ns = (n_total + GI_R - 1) / GI_R;
    const int64_t s0 = ns * w / GM_W, s1 = ns * (w + 1) / GM_W;
    const int64_t last_word = (n_total - 1) & ~(int64_t)15;
    // raw words of a step (an in-bounds word where the step's rows end before this lane's 16)
    auto load = [&](int64_t step, i32x4& a0, i32x4& a1, i32x4& bw, i32x4& mw) {
        const int64_t r0 = step * GI_R + 16 * kq;
        const int64_t rl = r0 < n_total ? r0 : last_word;
        a0 = *reinterpret_cast<const i32x4*>(ac[0] + rl);
        a1 = *reinterpret_cast<const i32x4*>(ac[1] + rl);
        bw = *reinterpret_cast<const i32x4*>(bc + rl);
        if constexpr (MASK) mw = *reinterpret_cast<const i32x4*>(mask + rl);
    };
    i32x4 acc[2] = {(i32x4){0, 0, 0, 0}, (i32x4){0, 0, 0, 0}};
    f64x4 a64[2] = {(f64x4){0.0, 0.0, 0.0, 0.0}, (f64x4){0.0, 0.0, 0.0, 0.0}};
    // B's bytes of rows past n_total or outside the fit are cleared as the step is consumed (clearing them at
    // the load would wait for the load)
    auto mma = [&](int64_t step, const i32x4& a0, const i32x4& a1, const i32x4& braw, const i32x4& mw) {
        const int64_t r0 = step * GI_R + 16 * kq;
        i32x4 bw;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
            uint32_t keep = bytes_below(n_total - r0 - 4 * d);
            if constexpr (MASK) keep &= bytes_nonzero((uint32_t)mw[d]);
            bw[d] = (int)((uint32_t)braw[d] & keep);
        }
        acc[0] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a0, bw, acc[0], 0, 0, 0);
        acc[1] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a1, bw, acc[1], 0, 0, 0);
    };
    auto flush = [&]() {
#pragma unroll
        for (int f = 0; f < 2; ++f) {
#pragma unroll
            for (int q = 0; q < 4; ++q) a64[f][q] += (double)acc[f][q];
            acc[f] = (i32x4){0, 0, 0, 0};
        }
    };
    // pairs of steps, two register sets taking turns (no branch between a prefetch and its use)
    i32x4 xa0, xa1, xb, xm = {-1, -1, -1, -1}, ya0, ya1, yb, ym = {-1, -1, -1, -1};
    if (s0 < s1) load(s0, xa0, xa1, xb, xm);
    int64_t step = s0;
    for (; step + 1 < s1; step += 2) {
        load(step + 1, ya0, ya1, yb, ym);
        issue_fence_g();
        mma(step, xa0, xa1, xb, xm);
        load(step + 2 < s1 ? step + 2 : s1 - 1, xa0, xa1, xb, xm);
        issue_fence_g();
        mma(step + 1, ya0, ya1, yb, ym);
        flush();
    }
    if (step < s1) mma(step, xa0, xa1, xb, xm);
    flush();
    if (w > 0) {
        red[w - 1][0][lane] = a64[0];
        red[w - 1][1][lane] = a64[1];
    }
    __syncthreads();
    if (w > 0) return;
#pragma unroll
    for (int v = 0; v < GM_W - 1; ++v) {
        a64[0] += red[v][0][lane];
        a64[1] += red[v][1][lane];
    }
    const int64_t t = tb + m;
    if (t >= N) return;
    const int jt = pool_list[P0 + t];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t k = kb + 16 * f + 4 * kq + q;
            if (k >= P) continue;
            if (k >= P0 && k - P0 > t) continue;   // written by the tile of its mirror
            const int jk = pool_list[k];
            const double gv = (a64[f][q] - n_rows * (c[jk] * c[jt])) / (n_rows * (s[jk] * s[jt]));
            G[k * ldg + (P0 + t)] = gv;
            G[(P0 + t) * ldg + k] = gv;
        }
    }
}

// G_E[e, f] = G_pool[pos(set[e]), pos(set[f])] (symmetric, m x m)
__global__ void k_gather_gram(const int32_t* __restrict__ set, int64_t m, const int32_t* __restrict__ pool_pos,
                              const double* __restrict__ Gp, int64_t ldg, double* __restrict__ GE) {
    const int64_t total = m * m;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = idx / m, f = idx - e * m;
        GE[idx] = Gp[(int64_t)pool_pos[set[e]] * ldg + pool_pos[set[f]]];
    }
}

// gradient and coefficients of the set at the start of a solve
__global__ void k_gather_start(const int32_t* __restrict__ set, int64_t m, const double* __restrict__ z,
                               const double* __restrict__ beta, double* __restrict__ g0,
                               double* __restrict__ b0) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int j = set[e];
        g0[e] = z[j];
        b0[e] = beta[j];
    }
}

// ---- the solve -----------------------------------------------------------------------------------------
constexpr int GCD_THREADS = 512;

__global__ __launch_bounds__(GCD_THREADS) void k_gcd(GcdArgs a) {
    __shared__ double g[GCD_MAX];
    __shared__ double bE[GCD_MAX];
    __shared__ double Gbb[GCD_B * GCD_B];
    __shared__ double dlt[GCD_B];
    __shared__ int nz[GCD_B];
    __shared__ int nnz_sh;
    __shared__ double maxd_sh;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
    const int64_t m = a.m;
    const double lam = a.lam;
    const double* __restrict__ G = a.G;
    for (int64_t e = tid; e < m; e += GCD_THREADS) {
        g[e] = a.g0[e];
        bE[e] = a.b0[e];
    }
    int sweeps = 0, status = 0;
    if (tid == 0) maxd_sh = 0.0;
    __syncthreads();
    if (m > 0) {
        for (;;) {
            for (int64_t b0 = 0; b0 < m; b0 += GCD_B) {
                const int bl = (int)((m - b0) < GCD_B ? (m - b0) : GCD_B);
                for (int idx = tid; idx < GCD_B * GCD_B; idx += GCD_THREADS) {
                    const int t = idx / GCD_B, l = idx % GCD_B;
                    Gbb[idx] = (t < bl && l < bl) ? G[(b0 + t) * m + b0 + l] : 0.0;
                }
                __syncthreads();
                if (wv == 0) {
                    // the sequential chain of this block, one coordinate per step
                    double gl = lane < bl ? g[b0 + lane] : 0.0;
                    double bv = lane < bl ? bE[b0 + lane] : 0.0;
                    const double ll = (a.lamv && lane < bl) ? a.lamv[b0 + lane] : lam;   // this lane's threshold
                    double dl = 0.0, wmax = 0.0;
                    auto col = [&](int t) { return Gbb[t * GCD_B + lane]; };
                    if (!chain_fast<GCD_B>(gl, bv, col, ll, bl, dl, wmax))
                        chain_exact<GCD_B>(gl, bv, col, ll, bl, dl, wmax);
                    if (lane < bl) {
                        g[b0 + lane] = gl;
                        bE[b0 + lane] = bv;
                        dlt[lane] = dl;
                    }
                    const uint64_t ball = __ballot(lane < bl && dl != 0.0);
                    const int before = __popcll(ball & ((1ull << lane) - 1ull));
                    if (lane < bl && dl != 0.0) nz[before] = lane;
                    if (lane == 0) {
                        nnz_sh = __popcll(ball);
                        maxd_sh = fmax(maxd_sh, wmax);
                    }
                }
                __syncthreads();
                const int nnz = nnz_sh;
                if (nnz > 0) {
                    // push the block's changes into every other coordinate's gradient
                    for (int64_t k = tid; k < m; k += GCD_THREADS) {
                        if (k >= b0 && k < b0 + bl) continue;
                        double acc = g[k];
                        for (int q = 0; q < nnz; ++q) {
                            const int t = nz[q];
                            acc = fma(-dlt[t], G[(b0 + t) * m + k], acc);
                        }
                        g[k] = acc;
                    }
                }
                __syncthreads();
            }
            ++sweeps;
            const double md = maxd_sh;
            __syncthreads();
            if (tid == 0) maxd_sh = 0.0;
            if (md < a.tol) break;
            if (sweeps >= a.max_sweeps) {
                status = 1;
                break;
            }
            __syncthreads();
        }
    } else {
        sweeps = 1;
    }
    __syncthreads();
    for (int64_t e = tid; e < m; e += GCD_THREADS) {
        a.b1[e] = bE[e];
        a.beta[a.set[e]] = bE[e];
    }
    if (tid == 0) {
        a.sc->round.sweeps = sweeps;
        a.sc->round.status = status;
        a.sc->round.cd_len = (int32_t)m;
    }
}

// ---- the solve across workgroups ----------------------------------------------------------------------
//
// Workgroup 0 (the leader) runs the sequential chain, block after block, in a
// global sequence q = sweep * nb + b (block b = q mod nb).  After the chain of
// q it publishes the block's coefficient changes d_q.  Every other workgroup
// (a helper) owns some blocks of the gradient g and applies each published d_q
// to them, in sequence order, except for the blocks b_q, b_q+1, ..., b_q+SLACK
// (mod nb): block b_q took its own changes inside the chain, and the leader
// itself applies the SLACK most recent changes to the block it is about to run.
// So before running block b at sequence q the leader needs the owner of b to
// have applied every sequence below q - SLACK; that is what it waits for.
// Every gradient entry receives the changes in sequence order, so the result
// does not depend on timing.  Changes are kept for two sweeps (slot q mod 2nb):
// the leader waits for every helper at least once per sweep, so a slot is never
// rewritten before its last reader has taken it.
//
// Shared data (gradient, changes, coefficients) is written and read with
// device-coherent (relaxed, device-scope) atomic accesses, and a writer waits
// for its stores to complete before it raises the counter that publishes them.
// Every wait is bounded: on time-out the waiter raises an error flag that all
// others see, and the host reports a device error.
constexpr int MB = 32;      // coordinates per block
constexpr int SLACK = 4;    // most recent blocks whose changes the leader applies itself
constexpr int MT = 256;     // threads per workgroup
constexpr int HBATCH = 4;   // sequences a helper applies per round trip at most
constexpr int HOWN = 2;     // blocks a helper owns at most

__device__ __forceinline__ double ld_coh(const double* p) {
    return __builtin_bit_cast(double, __hip_atomic_load((const uint64_t*)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_coh(double* p, double v) {
    __hip_atomic_store((uint64_t*)p, __builtin_bit_cast(uint64_t, v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_flag(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_flag(uint32_t* p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// wait until every memory access this wave issued has completed
__device__ __forceinline__ void wait_mem() { __builtin_amdgcn_s_waitcnt(0); }

// sync word layout (uint32): [0] published sequences, [1] stop, [2] error,
// [SYNC_APPLIED + 16 h] sequences helper h has applied (one 64-byte line each)
constexpr int SYNC_PUB = 0, SYNC_STOP = 1, SYNC_ERR = 2, SYNC_APPLIED = 64;

__device__ __forceinline__ int blk_len(int64_t m, int b) {
    const int64_t r = m - (int64_t)b * MB;
    return (int)(r < MB ? r : MB);
}

// load G[rows of block rb, columns of block cb] into dst[t * MB + l] (t column, l row), zero padded;
// the caller's STEP threads (numbered t0 = 0..STEP-1) each issue all their loads before storing any
template <int STEP>
__device__ __forceinline__ void load_gblock(const double* __restrict__ G, int64_t m, int rb, int cb, double* dst,
                                            int t0) {
    constexpr int PER = MB * MB / STEP;
    const int rl = blk_len(m, rb), cl = blk_len(m, cb);
    const int64_t r0 = (int64_t)rb * MB, c0 = (int64_t)cb * MB;
    double v[PER];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
        const int idx = t0 + k * STEP;
        const int t = idx / MB, l = idx % MB;
        v[k] = (t < cl && l < rl) ? G[(c0 + t) * m + r0 + l] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < PER; ++k) dst[t0 + k * STEP] = v[k];
}

// LDS arena shared by the two roles (a workgroup is either the leader or a helper)
// leader rings: Gram sets (GR), changes (DR, at least SLACK + 2), chain results awaiting publication (OR)
constexpr int GR = 3, DR = 8, OR = 4;
// leader counters in LDS: chains run, blocks prepared, blocks published, Gram sets loaded (each a count of
// sequences), the sequence count at which the chain stopped (INT_MAX while running), an error flag, and
// the solve's results
enum { LC_CHAIN, LC_PREP, LC_PUB, LC_GRAM, LC_STOP, LC_ERR, LC_SWEEPS, LC_STATUS, LC_N };
constexpr int LEAD_LDS = GR * (SLACK + 1) * MB * MB + 2 * 2 * MB + DR * MB + 2 * OR * MB + 8;
constexpr int HELP_LDS = HBATCH * HOWN * MB * MB + HBATCH * MB + HOWN * MB + (MT / MB) * HOWN * MB + 8;
constexpr int ARENA = LEAD_LDS > HELP_LDS ? LEAD_LDS : HELP_LDS;

// The working-set Gram matrix G (m x m, m <= 16,320, so byte offsets fit 32 bits) is read through a
// buffer resource: an offset past its end reads 0, which pads partial blocks without branches.
constexpr uint32_t GOFF_NONE = 0xFFFFFFF8u;
__device__ __forceinline__ __amdgpu_buffer_rsrc_t gram_rsrc(const double* G, int64_t m) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(G), (short)0, (int)(m * m * 8), 0x00020000);
}
__device__ __forceinline__ double gram_ld(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    const u2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)off, 0, 0);
    return __builtin_bit_cast(double, v);
}
// byte offset of G[(cb*MB + t) * m + rb*MB + l], or GOFF_NONE outside the blocks' lengths
__device__ __forceinline__ uint32_t gram_off(int64_t m, int cb, int cl, int rb, int rl, int t, int l) {
    return (t < cl && l < rl) ? (uint32_t)((((uint32_t)(cb * MB + t)) * (uint32_t)m + (uint32_t)(rb * MB + l)) * 8u)
                              : GOFF_NONE;
}

// The leader loads Gram sets with 16-byte loads: lane l covers rows 2 (l % 16) and 2 (l % 16) + 1 of
// columns l / 16 + 4k, k < GPER.  A set is (SLACK + 1) GPER = 40 loads per lane: under the 63 memory
// operations a wave can keep in flight, so issuing a set never waits for the first of its own loads to
// return (the next set's loads wait for the oldest ones of the set before).  The set size is what paces the
// loader: with SLACK = 5 (48 loads) the chain waited for it, and loading the next set block by block between
// the stores of the current one was slower still.
constexpr int GPER = MB * MB / (2 * WAVE);   // 16-byte loads per lane for one Gram block
constexpr int GSET = (SLACK + 1) * GPER;      // for one set of SLACK + 1 blocks
constexpr uint32_t GOFF_NONE2 = 0xFFFFFFF0u;  // out of range for a 16-byte load

__device__ __forceinline__ double2 gram_ld2(__amdgpu_buffer_rsrc_t rs, uint32_t off) {
    typedef unsigned int u4 __attribute__((ext_vector_type(4)));
    const u4 v = __builtin_amdgcn_raw_buffer_load_b128(rs, (int)off, 0, 0);
    return __builtin_bit_cast(double2, v);
}

// issue the loads of the Gram blocks of block rb against its own block and the SLACK blocks run before
// it (sequence qb and the SLACK sequences before it) into v; store_gset writes them to dst[s][t * MB + l].
// Rows past the block's length are zeroed: by the range check when both rows are out, by a select when
// only the second one is.
__device__ __forceinline__ void load_gset(__amdgpu_buffer_rsrc_t rs, int64_t m, int nb, int64_t qb, int rb,
                                          double2 (&v)[GSET], int lane) {
    const int rl = blk_len(m, rb);
    const int t0 = lane >> 4, l = 2 * (lane & 15);
    const uint32_t step = 4u * (uint32_t)m * 8u;
#pragma unroll
    for (int s = 0; s <= SLACK; ++s) {
        int cbk = rb - s;
        if (cbk < 0) cbk += nb;
        const int cl = qb - s >= 0 ? blk_len(m, cbk) : 0;
        const uint32_t base = (((uint32_t)(cbk * MB + t0)) * (uint32_t)m + (uint32_t)(rb * MB + l)) * 8u;
        const bool row_ok = l < rl;
#pragma unroll
        for (int k = 0; k < GPER; ++k) {
            const bool ok = row_ok && t0 + 4 * k < cl;
            v[s * GPER + k] = gram_ld2(rs, ok ? base + (uint32_t)k * step : GOFF_NONE2);
        }
    }
    if (l + 1 >= rl) {
#pragma unroll
        for (int k = 0; k < GSET; ++k) v[k].y = 0.0;
    }
}
__device__ __forceinline__ void store_gset(const double2 (&v)[GSET], double* dst, int lane) {
    const int t0 = lane >> 4, l = 2 * (lane & 15);
#pragma unroll
    for (int s = 0; s <= SLACK; ++s)
#pragma unroll
        for (int k = 0; k < GPER; ++k)
            *reinterpret_cast<double2*>(dst + s * MB * MB + (t0 + 4 * k) * MB + l) = v[s * GPER + k];
}

__device__ __forceinline__ int lc_get(const int* c, int i) {
    return __hip_atomic_load(c + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// raise a counter after this wave's stores to LDS: a wave's LDS operations complete in order, and the
// compiler fence keeps the stores before it
__device__ __forceinline__ void lc_set(int* c, int i, int v) {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    if ((threadIdx.x & (WAVE - 1)) == 0) __hip_atomic_store(c + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// wait until ready() holds; false if the solve failed, if the wait outlasts `limit` wall-clock ticks (then
// it fails the solve), or (exit_on_stop) once the chain has stopped
template <typename Ready>
__device__ __forceinline__ bool lead_wait(int* ctr, Ready ready, uint64_t limit, bool exit_on_stop) {
    uint64_t t0 = 0;
    for (uint32_t n = 0;; ++n) {
        if (__builtin_amdgcn_readfirstlane((int)ready())) break;
        if (__builtin_amdgcn_readfirstlane(lc_get(ctr, LC_ERR))) return false;
        if (exit_on_stop && __builtin_amdgcn_readfirstlane(lc_get(ctr, LC_STOP)) != INT_MAX) return false;
        if ((n & 63u) == 63u) {
            const uint64_t t = wall_clock64();
            if (t0 == 0) {
                t0 = t;
            } else if (t - t0 > limit) {
                lc_set(ctr, LC_ERR, 1);
                return false;
            }
        }
        if (exit_on_stop) __builtin_amdgcn_s_sleep(1);
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    return true;
}
// store Gram set j (registers v) into ring slot j mod GR once the chain that last used the slot is done
__device__ __forceinline__ bool lead_gram_store(int* ctr, const double2 (&v)[GSET], double* Gm, int64_t j,
                                                uint64_t limit, int lane) {
    if (!lead_wait(ctr, [&] { return (int64_t)lc_get(ctr, LC_CHAIN) > j - GR; }, limit, true)) return false;
    store_gset(v, Gm + (int)(j % GR) * (SLACK + 1) * MB * MB, lane);
    lc_set(ctr, LC_GRAM, (int)(j + 1));
    return true;
}

// OWN: blocks each helper owns at most (1 when there are helpers for every block, else 2)
template <int OWN>
__global__ __launch_bounds__(MT) void k_gcd_multi(GcdMultiArgs a) {
    // the wave index is uniform across the wave: taken through a scalar register, the per-wave branches
    // below compile to scalar jumps instead of execution-masked code that every wave walks through
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = __builtin_amdgcn_readfirstlane(tid / WAVE);
    const int64_t m = a.m;
    const int nb = (int)((m + MB - 1) / MB);
    const int H = a.H;
    uint32_t* sync = a.sync;
    const uint32_t spin_limit = a.spin_limit;
    __shared__ __attribute__((aligned(16))) double arena[ARENA];

    if (blockIdx.x == 0) {
        // ---------------- leader ----------------
        // Four waves, each running its own loop; they hand work to each other through counters in LDS
        // (no workgroup barrier inside the solve), so a wave waiting on memory holds up only the waves
        // that need its result.  For the block b_q run at sequence q:
        //   wave 3 loads the Gram set of q into ring slot q mod GR: [0] = G(b_q, b_q), [s] = G(b_q, b_{q-s});
        //   wave 2 prepares the block: once the owner has applied every change below q - SLACK it takes
        //          the block's gradient and coefficients and applies the changes of q - SLACK .. q - 2;
        //   wave 0 applies the change of q - 1 and runs the chain;
        //   wave 1 publishes the change, gradient and coefficients of the block for the helpers.
        double* Gm = arena;                               // [GR][SLACK + 1][MB * MB]
        double* gp = Gm + GR * (SLACK + 1) * MB * MB;     // [2][MB] prepared gradient, slot q mod 2
        double* bp = gp + 2 * MB;                         // [2][MB] prepared coefficients
        double* dh = bp + 2 * MB;                         // [DR][MB] changes, slot q mod DR
        double* go = dh + DR * MB;                        // [OR][MB] chain results (gradient), slot q mod OR
        double* bo = go + OR * MB;                        // [OR][MB] chain results (coefficients)
        int* ctr = reinterpret_cast<int*>(bo + OR * MB);  // counters, see LC_*
        if (tid < LC_N) ctr[tid] = tid == LC_STOP ? INT_MAX : 0;
        __syncthreads();
        const __amdgpu_buffer_rsrc_t grs = gram_rsrc(a.G, m);
        const uint64_t limit = (uint64_t)spin_limit * 100u;   // wall-clock ticks (100 MHz) of any one wait
        if (wv == 0) {
            // ---- the chain ----
            const int l32 = lane & (MB - 1);
            const double lam = a.lam;
            // gc: Gram columns of the block to run; gn: its entries against the block after it, which takes
            // un = sum_t gn[t] d_t from this block's changes, formed in the chain's post-pass
            double gc[MB], gn[MB], un = 0.0, maxd = 0.0;
            int sweeps = 0, status = 0, b = 0;
            int64_t q = 0;
            bool ok = lead_wait(ctr, [&] { return lc_get(ctr, LC_GRAM) > 0; }, limit, false);
            if (ok) {
#pragma unroll
                for (int t = 0; t < MB; ++t) gc[t] = Gm[t * MB + l32];
            }
            while (ok) {
                // the prepared block, free result slots (their publication is done) and the next block's
                // entries against this one (its Gram set is loaded whether or not the chain stops after this
                // block), the three counters read together: the other waves run ahead, so one read usually
                // finds all of them ready
                ok = lead_wait(ctr, [&] {
                    const int pr = lc_get(ctr, LC_PREP), pu = lc_get(ctr, LC_PUB), gr = lc_get(ctr, LC_GRAM);
                    return (pr > q) & (pu > q - OR) & (gr > q + 1);
                }, limit, false);
                if (!ok) break;
                const int cur = (int)(q & 1), bl = blk_len(m, b);
                // every lane reads (the slots hold MB values), so that no branch holds up the reads after these
                const double gpl = gp[cur * MB + l32], bpl = bp[cur * MB + l32];
                const double* Gn1 = Gm + (int)((q + 1) % GR) * (SLACK + 1) * MB * MB;
#pragma unroll
                for (int t = 0; t < MB; ++t) gn[t] = Gn1[MB * MB + t * MB + l32];
                __builtin_amdgcn_sched_barrier(0);   // all of these reads issue before the first use of one
                // the previous block's changes
                double gl = lane < bl ? (q >= 1 ? gpl - un : gpl) : 0.0;
                const double bv0 = lane < bl ? bpl : 0.0;
                double bv = bv0, dl = 0.0, wmax = 0.0;
                auto col = [&](int t) { return gc[t]; };
                auto coln = [&](int t) { return gn[t]; };
                double* dq = dh + (int)(q & (DR - 1)) * MB;   // this block's change slot
                if (!chain_fast_next<MB>(gl, bv, col, coln, lam, bl, dl, wmax, un)) {
                    chain_exact<MB>(gl, bv, col, lam, bl, dl, wmax);
                    if (lane < MB) dq[lane] = lane < bl ? dl : 0.0;
                    un = chain_next_update<MB>(coln, dq);
                }
                if (lane < MB) {
                    dq[lane] = lane < bl ? dl : 0.0;
                    go[(int)(q & (OR - 1)) * MB + lane] = gl;
                    bo[(int)(q & (OR - 1)) * MB + lane] = bv;
                }
                maxd = fmax(maxd, wmax);   // this lane's largest change in the sweep so far
                bool stop = false;
                if (b == nb - 1) {
                    ++sweeps;
#pragma unroll
                    for (int o = WAVE / 2; o > 0; o >>= 1) maxd = fmax(maxd, __shfl_xor(maxd, o, WAVE));
                    if (maxd < a.tol) stop = true;
                    else if (sweeps >= a.max_sweeps) {
                        status = 1;
                        stop = true;
                    }
                    maxd = 0.0;
                }
                ++q;
                if (stop) lc_set(ctr, LC_STOP, (int)q);
                lc_set(ctr, LC_CHAIN, (int)q);
                if (stop) break;
                b = b + 1 == nb ? 0 : b + 1;
                // the Gram columns of the next block (its set was waited for above)
                const double* Gn = Gm + (int)(q % GR) * (SLACK + 1) * MB * MB;
#pragma unroll
                for (int t = 0; t < MB; ++t) gc[t] = Gn[t * MB + l32];
            }
            if (!ok) {
                status = 2;
                lc_set(ctr, LC_ERR, 1);
                lc_set(ctr, LC_STOP, (int)q);
            }
            if (lane == 0) {
                ctr[LC_SWEEPS] = sweeps;
                ctr[LC_STATUS] = status;
            }
        } else if (wv == 1) {
            // ---- publishing: every chain result, in sequence order ----
            // (the wait ends on the stop only once every result up to it is published: the chain raises the
            // stop count before the chain count, so leaving on the stop flag alone could drop the last block)
            int bq = 0, slot = 0;
            for (int64_t q = 0;; ++q) {
                const bool ok = lead_wait(
                    ctr, [&] { return lc_get(ctr, LC_CHAIN) > q || lc_get(ctr, LC_STOP) <= q; }, limit, false);
                if (!ok || lc_get(ctr, LC_CHAIN) <= q) break;
                const int pl = blk_len(m, bq), rs = (int)(q & (OR - 1));
                const int64_t e0 = (int64_t)bq * MB;
                if (lane < pl) {
                    st_coh(a.delta + (int64_t)slot * MB + lane, dh[(int)(q & (DR - 1)) * MB + lane]);
                    st_coh(a.g + e0 + lane, go[rs * MB + lane]);
                    st_coh(a.b + e0 + lane, bo[rs * MB + lane]);
                }
                wait_mem();
                if (lane == 0) st_flag(sync + SYNC_PUB, (uint32_t)(q + 1));
                lc_set(ctr, LC_PUB, (int)(q + 1));
                bq = bq + 1 == nb ? 0 : bq + 1;
                slot = slot + 1 == 2 * nb ? 0 : slot + 1;
            }
        } else if (wv == 2) {
            // ---- preparing the block of sequence q ----
            // Pipelined by one block so that the global-memory round trips overlap the work in LDS: the owner's
            // count for the next block is read before this block's sums, and the next block's gradient and
            // coefficients are read (once that count and the publication allow) after this block is handed on,
            // to arrive while the next block's sums are formed.
            const int l32 = lane & (MB - 1), half = lane >> 5;
            // block bb at sequence qq: its owner must have applied every change below qq - SLACK (fl: a value
            // of the owner's count read earlier, polled again only if it is not yet enough), and its
            // coefficients, last set at sequence qq - nb, must be published; then its reads go out
            auto fetch = [&](int64_t qq, int bb, uint32_t fl, double& gq, double& bq_) -> bool {
                const int64_t need = qq - SLACK;
                bool ok = true;
                if (need > 0 && (int64_t)fl < need) {
                    const int owner = bb % H;
                    ok = lead_wait(ctr, [&] { return (int64_t)ld_flag(sync + SYNC_APPLIED + 16 * owner) >= need; },
                                   limit, true);
                }
                if (ok && qq >= nb) ok = lead_wait(ctr, [&] { return lc_get(ctr, LC_PUB) > qq - nb; }, limit, true);
                if (!ok) return false;
                const int nl = blk_len(m, bb);
                const int64_t e0 = (int64_t)bb * MB;
                gq = l32 < nl ? ld_coh(a.g + e0 + l32) : 0.0;
                bq_ = l32 < nl ? ld_coh(a.b + e0 + l32) : 0.0;
                return true;
            };
            int bq = 0;
            double gcur = 0.0, bcur = 0.0;
            bool ok = lc_get(ctr, LC_STOP) == INT_MAX && fetch(0, 0, 0u, gcur, bcur);
            for (int64_t q = 0; ok; ++q) {
                if (lc_get(ctr, LC_STOP) != INT_MAX) break;
                const int bn1 = bq + 1 == nb ? 0 : bq + 1;
                const uint32_t fl1 = ld_flag(sync + SYNC_APPLIED + 16 * (bn1 % H));   // used after the sums
                // the changes up to q - 2, the Gram set of q, and a free slot (the chain of q - 2 is done)
                ok = lead_wait(ctr, [&] { return lc_get(ctr, LC_CHAIN) >= q - 1 && lc_get(ctr, LC_GRAM) > q; },
                               limit, true);
                if (!ok) break;
                const double* Gn = Gm + (int)(q % GR) * (SLACK + 1) * MB * MB;
                double u = 0.0;
#pragma unroll
                for (int o = SLACK; o >= 2; --o) {
                    const int64_t sq = q - o;
                    if (sq < 0) continue;
                    const double* Gs = Gn + o * MB * MB;
                    const double* ds = dh + (int)(sq & (DR - 1)) * MB;
                    double gs[MB / 2], dd[MB / 2];
#pragma unroll
                    for (int t = 0; t < MB / 2; ++t) {
                        const int tt = half * (MB / 2) + t;
                        gs[t] = Gs[tt * MB + l32];
                        dd[t] = ds[tt];
                    }
#pragma unroll
                    for (int t = 0; t < MB / 2; ++t) u = fma(gs[t], dd[t], u);
                }
                u += __shfl_xor(u, 32, WAVE);
                if (lane < MB) {
                    gp[(int)(q & 1) * MB + lane] = gcur - u;
                    bp[(int)(q & 1) * MB + lane] = bcur;
                }
                lc_set(ctr, LC_PREP, (int)(q + 1));
                ok = fetch(q + 1, bn1, fl1, gcur, bcur);
                bq = bn1;
            }
            // the reads still in flight complete before the wave ends
            wait_mem();
        } else {
            // ---- Gram sets, two in flight: set j + 1 is loading while set j is stored ----
            double2 va[GSET], vb[GSET];
            int bj = 0;
            load_gset(grs, m, nb, 0, 0, va, lane);
            for (int64_t j = 0;; j += 2) {
                int b1 = bj + 1 == nb ? 0 : bj + 1;
                load_gset(grs, m, nb, j + 1, b1, vb, lane);
                if (!lead_gram_store(ctr, va, Gm, j, limit, lane)) break;
                int b2 = b1 + 1 == nb ? 0 : b1 + 1;
                load_gset(grs, m, nb, j + 2, b2, va, lane);
                if (!lead_gram_store(ctr, vb, Gm, j + 1, limit, lane)) break;
                bj = b2;
            }
            // the loads still in flight complete before the wave ends
            wait_mem();
        }
        __syncthreads();
        if (tid == 0) {
            const int status = ctr[LC_STATUS];
            st_flag(sync + SYNC_STOP, 1u);
            if (status == 2) st_flag(sync + SYNC_ERR, 1u);
            a.sc->round.sweeps = ctr[LC_SWEEPS];
            a.sc->round.status = status;
            a.sc->round.cd_len = (int32_t)m;
        }
        return;
    }

    // ---------------- helper ----------------
    auto Gh = reinterpret_cast<double(*)[OWN][MB * MB]>(arena);                         // [HBATCH][OWN][MB*MB]
    auto dlt = reinterpret_cast<double(*)[MB]>(arena + HBATCH * OWN * MB * MB);           // [HBATCH][MB]
    auto gh = reinterpret_cast<double(*)[MB]>(arena + HBATCH * OWN * MB * MB + HBATCH * MB);  // [OWN][MB]
    auto hp = reinterpret_cast<double(*)[OWN][MB]>(arena + HBATCH * OWN * MB * MB + HBATCH * MB + OWN * MB);
    int64_t& pub_sh = *reinterpret_cast<int64_t*>(arena + HELP_LDS - 8);
    int& quit_sh = *reinterpret_cast<int*>(arena + HELP_LDS - 7);
    const int h = blockIdx.x - 1;
    int own[OWN];
    int nown = 0;
    for (int c = h; c < nb && nown < OWN; c += H) own[nown++] = c;
    const __amdgpu_buffer_rsrc_t grs = gram_rsrc(a.G, m);
    int64_t s0 = 0;  // next sequence to apply
    int hb = 0;      // s0 mod nb
    int hslot = 0;   // s0 mod 2nb
    for (;;) {
        if (tid == 0) {
            uint32_t spins = 0;
            int quit = 0;
            int64_t pub;
            for (;;) {
                pub = (int64_t)ld_flag(sync + SYNC_PUB);
                if (pub > s0) break;
                if (ld_flag(sync + SYNC_STOP) || ld_flag(sync + SYNC_ERR)) {
                    quit = 1;
                    break;
                }
                if (++spins > spin_limit) {
                    st_flag(sync + SYNC_ERR, 1u);
                    quit = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            pub_sh = pub;
            quit_sh = quit;
        }
        __syncthreads();
        if (quit_sh) break;
        const int nbat = (int)((pub_sh - s0) < HBATCH ? (pub_sh - s0) : HBATCH);
        // changes and Gram blocks of this batch, and the owned gradient blocks: every load is
        // issued before the first one is waited for
        {
            constexpr int PER = MB * MB / MT;
            double gv[HBATCH][OWN][PER];
            double dv[HBATCH];
            double hv[OWN];
#pragma unroll
            for (int k = 0; k < HBATCH; ++k) {
                int bq = hb + k;
                if (bq >= nb) bq -= nb;
                int sl = hslot + k;
                if (sl >= 2 * nb) sl -= 2 * nb;
                const bool kin = k < nbat;
                dv[k] = (kin && tid < blk_len(m, bq)) ? ld_coh(a.delta + (int64_t)sl * MB + tid) : 0.0;
#pragma unroll
                for (int o = 0; o < OWN; ++o) {
                    int dist = own[o] - bq;
                    if (dist < 0) dist += nb;
                    const bool use = kin && o < nown && dist > SLACK;
                    const int ob = o < nown ? own[o] : 0;
                    const int rl = use ? blk_len(m, ob) : 0, cl = use ? blk_len(m, bq) : 0;
#pragma unroll
                    for (int q2 = 0; q2 < PER; ++q2) {
                        const int idx = tid + q2 * MT;
                        gv[k][o][q2] = gram_ld(grs, gram_off(m, bq, cl, ob, rl, idx / MB, idx % MB));
                    }
                }
            }
#pragma unroll
            for (int o = 0; o < OWN; ++o)
                hv[o] = (o < nown && tid < blk_len(m, own[o])) ? ld_coh(a.g + (int64_t)own[o] * MB + tid) : 0.0;
#pragma unroll
            for (int k = 0; k < HBATCH; ++k) {
                if (tid < MB) dlt[k][tid] = dv[k];
#pragma unroll
                for (int o = 0; o < OWN; ++o)
#pragma unroll
                    for (int q2 = 0; q2 < PER; ++q2) Gh[k][o][tid + q2 * MT] = gv[k][o][q2];
            }
#pragma unroll
            for (int o = 0; o < OWN; ++o)
                if (tid < MB) gh[o][tid] = hv[o];
        }
        __syncthreads();
        bool touched[OWN] = {};
        for (int k = 0; k < nbat; ++k) {
            int bq = hb + k;
            if (bq >= nb) bq -= nb;
            for (int o = 0; o < nown; ++o) {
                int dist = own[o] - bq;
                if (dist < 0) dist += nb;
                if (dist <= SLACK) continue;  // uniform
                touched[o] = true;
                const int l = tid % MB, pp = tid / MB;
                double acc = 0.0;
#pragma unroll
                for (int t = pp * 4; t < pp * 4 + 4; ++t) acc = fma(Gh[k][o][t * MB + l], dlt[k][t], acc);
                hp[pp][o][l] = acc;
                __syncthreads();
                if (tid < MB) {
                    double tot = 0.0;
#pragma unroll
                    for (int q2 = 0; q2 < MT / MB; ++q2) tot += hp[q2][o][tid];
                    gh[o][tid] -= tot;
                }
                __syncthreads();
            }
        }
        // a block is written back only when this batch changed it: a batch that only skips a block
        // may overlap the leader's own update of it
        for (int o = 0; o < nown; ++o)
            if (touched[o] && tid < blk_len(m, own[o])) st_coh(a.g + (int64_t)own[o] * MB + tid, gh[o][tid]);
        wait_mem();
        __syncthreads();
        s0 += nbat;
        hb += nbat;
        if (hb >= nb) hb -= nb;
        hslot += nbat;
        if (hslot >= 2 * nb) hslot -= 2 * nb;
        if (tid == 0) st_flag(sync + SYNC_APPLIED + 16 * h, (uint32_t)s0);
    }
}

// ---- residual update after a solve -----------------------------------------------------------------------
// partial[c][i] = sum over set positions e in chunk c of x~_{i,set[e]} (b1[e] - b0[e]) on fitted rows
constexpr int RU_CHUNK = 64;

template <typename XT, bool MASK>
__global__ __launch_bounds__(256) void k_r_update_part(const XT* __restrict__ X, int64_t ldx, int64_t n_total,
                                                       const uint8_t* __restrict__ mask,
                                                       const int32_t* __restrict__ set, int64_t m,
                                                       const double* __restrict__ b0, const double* __restrict__ b1,
                                                       const double* __restrict__ c, const double* __restrict__ s,
                                                       double* __restrict__ part) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.y * RU_CHUNK;
    const int64_t e1 = e0 + RU_CHUNK < m ? e0 + RU_CHUNK : m;
    double acc = 0.0;
    if (i < n_total && (!MASK || mask[i])) {
        for (int64_t e = e0; e < e1; ++e) {
            const double d = b1[e] - b0[e];
            if (d == 0.0) continue;
            const int j = set[e];
            acc = fma(d / s[j], ld_x(X + (int64_t)j * ldx + i) - c[j], acc);
        }
    }
    if (i < n_total) part[blockIdx.y * n_total + i] = acc;
}

__global__ void k_r_update_reduce(int64_t n_total, int nchunks, const double* __restrict__ part,
                                  double* __restrict__ r) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_total; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int q = 0; q < nchunks; ++q) acc += part[(int64_t)q * n_total + i];
        r[i] -= acc;
    }
}

int grid_for(int64_t work, int per_block, int max_blocks) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > max_blocks) g = max_blocks;
    return (int)g;
}

}  // namespace

hipError_t launch_pool_add(const int32_t* set, const int64_t* len_dev, int64_t len_host, int32_t* pool_pos,
                           int32_t* pool_list, int64_t pool_size, int64_t* n_new_out, hipStream_t st) {
    k_pool_add<<<1, 1024, 0, st>>>(set, len_dev, len_host, pool_pos, pool_list, pool_size, n_new_out);
    return hipGetLastError();
}

template <typename XT>
static hipError_t gram_typed(const Mat& m, const int32_t* pool_list, int64_t P, int64_t P0, int64_t N,
                             const double* c, const double* s, double n_rows, double* G, int64_t ldg,
                             hipStream_t st) {
    dim3 grid((unsigned)((P + GM_K - 1) / GM_K), (unsigned)((N + GM_N - 1) / GM_N));
    if constexpr (sizeof(XT) == 1) {
        // int8 matrix cores when every column (and the row mask) is 16-byte aligned; with a row mask also only
        // when n_total is a multiple of 16, so that the mask's last 16-byte word lies within its n_total bytes
        // (otherwise the FP64 kernel below, whose integer sums are the same bits)
        const bool al = (uintptr_t)m.X % 16 == 0 && m.ldx % 16 == 0 && (uintptr_t)m.mask % 16 == 0 &&
                        (m.mask == nullptr || m.n_total % 16 == 0);
        if (al && m.n_total > 0) {
            if (m.mask)
                k_gram_update_i8<true><<<grid, 64 * GM_W, 0, st>>>((const int8_t*)m.X, m.ldx, m.n_total, m.mask,
                                                                    pool_list, P, P0, N, c, s, n_rows, G, ldg);
            else
                k_gram_update_i8<false><<<grid, 64 * GM_W, 0, st>>>((const int8_t*)m.X, m.ldx, m.n_total, m.mask,
                                                                     pool_list, P, P0, N, c, s, n_rows, G, ldg);
            return hipGetLastError();
        }
    }
    const bool vec = (uintptr_t)m.X % 16 == 0 && (m.ldx * (int64_t)sizeof(XT)) % 16 == 0 && (uintptr_t)m.mask % 16 == 0;
    if (m.mask && vec)
        k_gram_update<XT, true, true><<<grid, 64 * GM_W, 0, st>>>((const XT*)m.X, m.ldx, m.n_total, m.mask,
                                                                   pool_list, P, P0, N, c, s, n_rows, G, ldg);
    else if (m.mask)
        k_gram_update<XT, true, false><<<grid, 64 * GM_W, 0, st>>>((const XT*)m.X, m.ldx, m.n_total, m.mask,
                                                                    pool_list, P, P0, N, c, s, n_rows, G, ldg);
    else if (vec)
        k_gram_update<XT, false, true><<<grid, 64 * GM_W, 0, st>>>((const XT*)m.X, m.ldx, m.n_total, m.mask,
                                                                    pool_list, P, P0, N, c, s, n_rows, G, ldg);
    else
        k_gram_update<XT, false, false><<<grid, 64 * GM_W, 0, st>>>((const XT*)m.X, m.ldx, m.n_total, m.mask,
                                                                     pool_list, P, P0, N, c, s, n_rows, G, ldg);
    return hipGetLastError();
}

hipError_t launch_gram_update(const Mat& m, const int32_t* pool_list, int64_t P, int64_t P0, int64_t N,
                              const double* c, const double* s, double n_rows, double* G, int64_t ldg,
                              hipStream_t st) {
    if (N <= 0) return hipSuccess;
    switch (m.xtype) {
        case 0: return gram_typed<double>(m, pool_list, P, P0, N, c, s, n_rows, G, ldg, st);
        case 1: return gram_typed<float>(m, pool_list, P, P0, N, c, s, n_rows, G, ldg, st);
        default: return gram_typed<int8_t>(m, pool_list, P, P0, N, c, s, n_rows, G, ldg, st);
    }
}

hipError_t launch_gather_gram(const int32_t* set, int64_t m, const int32_t* pool_pos, const double* Gp, int64_t ldg,
                              double* GE, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    k_gather_gram<<<grid_for(m * m, 256, 8192), 256, 0, st>>>(set, m, pool_pos, Gp, ldg, GE);
    return hipGetLastError();
}

hipError_t launch_gather_start(const int32_t* set, int64_t m, const double* z, const double* beta, double* g0,
                               double* b0, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    k_gather_start<<<grid_for(m, 256, 1024), 256, 0, st>>>(set, m, z, beta, g0, b0);
    return hipGetLastError();
}

hipError_t launch_gcd(const GcdArgs& a, hipStream_t st) {
    k_gcd<<<1, GCD_THREADS, 0, st>>>(a);
    return hipGetLastError();
}

int64_t gram_cd_max() { return (int64_t)255 * HOWN * MB; }  // one workgroup per compute unit at most

int gcd_multi_helpers(int64_t m, int cap) {
    const int nb = (int)((m + MB - 1) / MB);
    if (nb < 2 * (SLACK + 2)) return 0;  // small sets: the single-workgroup solve
    if (nb <= cap) return nb;            // a helper per block: each change reaches every block sooner
    return (nb + HOWN - 1) / HOWN;
}

// ---- elastic net in the covariance solve ----------------------------------------------------------------
__device__ __forceinline__ double enet_q(const double* w, int j, double lr) { return sqrt(1.0 + lr * (w ? w[j] : 1.0)); }

__global__ void k_enet_scale_vec(const int32_t* __restrict__ set, int64_t m, const double* __restrict__ w, double lam,
                                 double alpha, double* __restrict__ g0, double* __restrict__ b0,
                                 double* __restrict__ lamv) {
    const double lr = lam * (1.0 - alpha);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int j = set[e];
        const double wj = w ? w[j] : 1.0;
        const double q = enet_q(w, j, lr);
        g0[e] = (g0[e] - lr * wj * b0[e]) / q;
        b0[e] = b0[e] * q;
        if (lamv) lamv[e] = lam * alpha * wj / q;
    }
}

// G~[e][f] = G[e][f] / (q_e q_f), G~[e][e] = (G[e][e] + lam (1 - alpha) w_e) / q_e^2
__global__ void k_enet_scale_gram(const int32_t* __restrict__ set, int64_t m, const double* __restrict__ w, double lam,
                                  double alpha, double* __restrict__ GE) {
    const double lr = lam * (1.0 - alpha);
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < m * m;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = idx / m, f = idx % m;
        const int je = set[e], jf = set[f];
        const double qe = enet_q(w, je, lr), qf = enet_q(w, jf, lr);
        GE[idx] = e == f ? (GE[idx] + lr * (w ? w[je] : 1.0)) / (qe * qe) : GE[idx] / (qe * qf);
    }
}

__global__ void k_enet_unscale(const int32_t* __restrict__ set, int64_t m, const double* __restrict__ w, double lam,
                               double alpha, double* __restrict__ b0, double* __restrict__ b1,
                               double* __restrict__ beta) {
    const double lr = lam * (1.0 - alpha);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int j = set[e];
        const double q = enet_q(w, j, lr);
        b0[e] = b0[e] / q;
        const double b = b1[e] / q;
        b1[e] = b;
        beta[j] = b;
    }
}

__global__ void k_map_pos(const int32_t* __restrict__ set, int64_t m, const int32_t* __restrict__ pos,
                          int32_t* __restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = pos[set[e]];
}

hipError_t launch_map_pos(const int32_t* set, int64_t m, const int32_t* pool_pos, int32_t* out, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    k_map_pos<<<grid_for(m, 256, 1024), 256, 0, st>>>(set, m, pool_pos, out);
    return hipGetLastError();
}

hipError_t launch_enet_scale(const int32_t* set, int64_t m, const double* w, double lam, double alpha, double* GE,
                             double* g0, double* b0, double* lamv, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    k_enet_scale_vec<<<grid_for(m, 256, 1024), 256, 0, st>>>(set, m, w, lam, alpha, g0, b0, lamv);
    k_enet_scale_gram<<<grid_for(m * m, 256, 8192), 256, 0, st>>>(set, m, w, lam, alpha, GE);
    return hipGetLastError();
}

hipError_t launch_enet_unscale(const int32_t* set, int64_t m, const double* w, double lam, double alpha, double* b0,
                               double* b1, double* beta, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    k_enet_unscale<<<grid_for(m, 256, 1024), 256, 0, st>>>(set, m, w, lam, alpha, b0, b1, beta);
    return hipGetLastError();
}

int gcd_multi_resident() {
    int per_cu1 = 0, per_cu2 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu1, k_gcd_multi<1>, MT, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu2, k_gcd_multi<HOWN>, MT, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return std::min(per_cu1, per_cu2) * device_cu_count();
}

size_t gcd_multi_sync_words(int H) { return (size_t)(SYNC_APPLIED + 16 * (H + 1)); }

hipError_t launch_gcd_multi(const GcdMultiArgs& a, hipStream_t st) {
    const int nb = (int)((a.m + MB - 1) / MB);
    if (a.H >= nb) k_gcd_multi<1><<<1 + a.H, MT, 0, st>>>(a);
    else k_gcd_multi<HOWN><<<1 + a.H, MT, 0, st>>>(a);
    return hipGetLastError();
}

__global__ void k_copy_f64(const double* __restrict__ src, double* __restrict__ dst, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// write the final coefficients back to beta[set[e]]
__global__ void k_scatter_beta(const int32_t* __restrict__ set, int64_t m, const double* __restrict__ b1,
                               double* __restrict__ beta) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        beta[set[e]] = b1[e];
}

hipError_t launch_copy_f64(const double* src, double* dst, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    k_copy_f64<<<grid_for(n, 256, 1024), 256, 0, st>>>(src, dst, n);
    return hipGetLastError();
}

hipError_t launch_scatter_beta(const int32_t* set, int64_t m, const double* b1, double* beta, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    k_scatter_beta<<<grid_for(m, 256, 1024), 256, 0, st>>>(set, m, b1, beta);
    return hipGetLastError();
}

size_t r_update_scratch_bytes(int64_t n_total, int64_t m) {
    const int64_t nch = (m + RU_CHUNK - 1) / RU_CHUNK;
    return (size_t)(nch < 1 ? 1 : nch) * (size_t)n_total * sizeof(double);
}

template <typename XT>
static hipError_t ru_typed(const Mat& mt, const int32_t* set, int64_t m, const double* b0, const double* b1,
                           const double* c, const double* s, double* part, double* r, hipStream_t st) {
    const int nch = (int)((m + RU_CHUNK - 1) / RU_CHUNK);
    dim3 grid((unsigned)((mt.n_total + 255) / 256), (unsigned)nch);
    if (mt.mask)
        k_r_update_part<XT, true><<<grid, 256, 0, st>>>((const XT*)mt.X, mt.ldx, mt.n_total, mt.mask, set, m, b0, b1,
                                                        c, s, part);
    else
        k_r_update_part<XT, false><<<grid, 256, 0, st>>>((const XT*)mt.X, mt.ldx, mt.n_total, mt.mask, set, m, b0,
                                                         b1, c, s, part);
    k_r_update_reduce<<<grid_for(mt.n_total, 256, 1024), 256, 0, st>>>(mt.n_total, nch, part, r);
    return hipGetLastError();
}

hipError_t launch_r_update(const Mat& mt, const int32_t* set, int64_t m, const double* b0, const double* b1,
                           const double* c, const double* s, double* part, double* r, hipStream_t st) {
    if (m <= 0) return hipSuccess;
    switch (mt.xtype) {
        case 0: return ru_typed<double>(mt, set, m, b0, b1, c, s, part, r, st);
        case 1: return ru_typed<float>(mt, set, m, b0, b1, c, s, part, r, st);
        default: return ru_typed<int8_t>(mt, set, m, b0, b1, c, s, part, r, st);
    }
}

}  // namespace blk
