// Precision forms of the scan: int8 design codes on BF16 matrix cores, or on int8 dot products.
//
// BF16 form:
// z_j = (x_j' r - c_j sum(r)) / (n s_j) is computed as Z = X_T' [r1 r2 r3] with
//   r1 = bf16(r), r2 = bf16(r - r1), r3 = bf16(r - r1 - r2)   (residual pieces, FP64 differences)
// on v_mfma_f32_16x16x32_bf16.  Int8 codes convert to BF16 exactly (|x| <= 256),
// each product x * r_c is exact in FP32, the FP32 accumulator is promoted to FP64
// after every 64 rows (two chained MFMA steps), and the three pieces are added in FP64.  The error of z_j is
// bounded column by column (lowp_bound); a decision whose value lies within that
// bound of its threshold is taken again on the exact FP64 scan.
//
// Tile: a wavefront owns 16 columns of the scan list; lane (m = l%16, g = l/16)
// loads 32 consecutive codes of column m (rows i0 + 32g ..) per 128-row batch, so
// a wavefront load covers 16 full 128-byte segments.  The MFMA reduction order
// over rows is free, so step s of a batch feeds rows i0 + 32g + 8s .. +7 of lane
// group g to both operands.  The residual pieces sit in LDS.
//
// int8 form: the residual is split into four int8 pieces with power-of-two scales,
//   r = s_1 q_1 + s_2 q_2 + s_3 q_3 + s_4 q_4 + t,   s_{k+1} = s_k / 128,
// each s_k q_k and the remainder t exact in FP64.  D_jk = x_j' q_k runs on v_dot4_i32_i8 over coalesced
// column streams with exact integer sums, and x_j' r = sum_k s_k D_jk + x_j' t.  The only errors are x_j' t
// (bounded by ||x_j||_2 ||t||_2) and the FP64 sum of the four scaled integers; the codes are used as loaded.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace blk {

namespace {

constexpr int WAVE = 64;
constexpr int SCAN_KC = 128;    // rows per load batch (4 MFMA steps of 32 rows)
constexpr int SCAN_U = 4;       // batches whose loads are in flight together

// Rows of a 128-row batch fed by lane group g (lanes 16g..16g+15) at MFMA step st: 8 consecutive rows,
// arranged so that each 16-byte load instruction of the wave covers whole 64-byte spans of a column
// (steps 0, 1: rows 16g .. 16g+15; steps 2, 3: rows 64+16g .. 64+16g+15).
__device__ __forceinline__ int lane_row(int g, int st) { return st < 2 ? 16 * g + 8 * st : 64 + 16 * g + 8 * (st - 2); }
constexpr int SCAN_PROMOTE = 64; // rows per FP32 chunk: the accumulator goes to FP64 after every two MFMA steps
constexpr int NPIECE = LOWP_PIECES;

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef int v4i32 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __bf16 to_bf16_rn(float f) { return (__bf16)f; }

// residual pieces, zero past n_total (rows outside the fit hold r = 0 already)
__global__ void k_r_pieces(const double* __restrict__ r, int64_t n_total, int64_t n_pad, __bf16* __restrict__ pc) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad; i += (int64_t)gridDim.x * blockDim.x) {
        double rem = i < n_total ? r[i] : 0.0;
#pragma unroll
        for (int c = 0; c < NPIECE; ++c) {
            const __bf16 b = to_bf16_rn((float)rem);
            pc[c * n_pad + i] = b;
            rem -= (double)(float)b;
        }
    }
}

// 8 int8 codes -> 8 bf16 (exact)
__device__ __forceinline__ bf16x8 codes_to_bf16(uint32_t lo, uint32_t hi) {
    f32x8 f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        f[b] = (float)(int)(int8_t)((lo >> (8 * b)) & 0xff);
        f[4 + b] = (float)(int)(int8_t)((hi >> (8 * b)) & 0xff);
    }
    return __builtin_convertvector(f, bf16x8);
}

template <bool PLDS>
__global__ __launch_bounds__(256) void k_scan_bf16(const int8_t* __restrict__ X, int64_t ldx, int64_t n_total,
                                                   int64_t n_pad, const __bf16* __restrict__ pieces,
                                                   const int32_t* __restrict__ cols, const int64_t* __restrict__ len_dev,
                                                   int64_t len_host, const DevScalars* __restrict__ sc,
                                                   const double* __restrict__ c, const double* __restrict__ s,
                                                   const uint8_t* __restrict__ keep, double* __restrict__ z) {
    extern __shared__ __bf16 pl[];
    const int64_t len = len_dev ? *len_dev : len_host;
    const int wpb = blockDim.x / WAVE;
    const int64_t ngroups = (len + 15) / 16;
    const int64_t gw0 = (int64_t)blockIdx.x * wpb;
    if (gw0 >= ngroups) return;
    const __bf16* P = pieces;
    if constexpr (PLDS) {
        const v4i32* src = reinterpret_cast<const v4i32*>(pieces);
        v4i32* dst = reinterpret_cast<v4i32*>(pl);
        const int64_t nv = (int64_t)NPIECE * n_pad / 8;
        for (int64_t k = threadIdx.x; k < nv; k += blockDim.x) dst[k] = src[k];
        __syncthreads();
        P = pl;
    }
    const int lane = threadIdx.x & (WAVE - 1);
    const int m = lane & 15, g = lane >> 4;
    const double sum_r = sc->sum_r;
    const double inv_n = 1.0 / (double)sc->n_rows;
    const int64_t nfull = (n_total / SCAN_KC) * SCAN_KC;
    for (int64_t grp = gw0 + threadIdx.x / WAVE; grp < ngroups; grp += (int64_t)gridDim.x * wpb) {
        const int64_t t = grp * 16 + m;
        const bool valid = t < len;
        const int64_t j = valid ? (cols ? (int64_t)cols[t] : t) : 0;
        const int8_t* xc = X + j * ldx;
        double acc64[4] = {0.0, 0.0, 0.0, 0.0};
        // lanes past the pieces (m >= 3) read piece 0: their matrix-core outputs are never used
        const __bf16* pr = P + (int64_t)(m < NPIECE ? m : 0) * n_pad;
        // one batch of SCAN_KC rows: 4 MFMA steps of 32 rows, FP32 sums of 64 rows promoted to FP64
        auto batch = [&](const v4i32& w0, const v4i32& w1, int64_t ib) {
            // residual pieces of the 4 steps first (one wait for all)
            bf16x8 bq[4];
#pragma unroll
            for (int st = 0; st < 4; ++st) bq[st] = *reinterpret_cast<const bf16x8*>(pr + ib + lane_row(g, st));
            const uint32_t wd[8] = {(uint32_t)w0.x, (uint32_t)w0.y, (uint32_t)w0.z, (uint32_t)w0.w,
                                    (uint32_t)w1.x, (uint32_t)w1.y, (uint32_t)w1.z, (uint32_t)w1.w};
            // the 4 steps go to the matrix cores back to back as two chains of two (steps 0, 2 and 1, 3); each
            // chain's 64-row FP32 sum is then promoted
            f32x4 r[2];
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const bf16x8 a = codes_to_bf16(wd[2 * st], wd[2 * st + 1]);
                const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
                r[st & 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bq[st], st < 2 ? zero : r[st & 1], 0, 0, 0);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc64[q] += (double)r[h][q];
        };
        // SCAN_U batches' loads are issued before the first is used (memory parallelism per wave)
        int64_t i0 = 0;
        for (; i0 + SCAN_U * SCAN_KC <= nfull; i0 += SCAN_U * SCAN_KC) {
            v4i32 w[SCAN_U][2];   // lanes past the end of the list read column 0 (their sums are not written)
#pragma unroll
            for (int u = 0; u < SCAN_U; ++u) {
                const v4i32* xp = reinterpret_cast<const v4i32*>(xc + i0 + u * SCAN_KC + 16 * g);
                w[u][0] = xp[0];
                w[u][1] = xp[4];
            }
#pragma unroll
            for (int u = 0; u < SCAN_U; ++u) batch(w[u][0], w[u][1], i0 + u * SCAN_KC);
        }
        for (; i0 < nfull; i0 += SCAN_KC) {
            const v4i32* xp = reinterpret_cast<const v4i32*>(xc + i0 + 16 * g);
            batch(xp[0], xp[4], i0);
        }
        if (i0 < n_total) {
            // ragged tail: codes past n_total meet zero residual pieces, but are not read
            uint32_t wd[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                uint32_t w = 0;
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    const int64_t i = i0 + (k < 4 ? 16 * g + 4 * k : 64 + 16 * g + 4 * (k - 4)) + b;
                    const uint32_t v = (valid && i < n_total) ? (uint32_t)(uint8_t)xc[i] : 0u;
                    w |= v << (8 * b);
                }
                wd[k] = w;
            }
            f32x4 r[2];
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const bf16x8 a = codes_to_bf16(wd[2 * st], wd[2 * st + 1]);
                const bf16x8 b = *reinterpret_cast<const bf16x8*>(pr + i0 + lane_row(g, st));
                const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
                r[st & 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, st < 2 ? zero : r[st & 1], 0, 0, 0);
            }
#pragma unroll
            for (int h = 0; h < 2; ++h)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc64[q] += (double)r[h][q];
        }
        // lane (piece m, group g) holds columns 4g..4g+3 of this group for piece m; add the pieces
        double tot[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const double p1 = __shfl(acc64[q], lane + 1, WAVE);
            const double p2 = __shfl(acc64[q], lane + 2, WAVE);
            tot[q] = (p2 + p1) + acc64[q];
        }
        if (m == 0) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t tt = grp * 16 + 4 * g + q;
                if (tt < len) {
                    const int64_t jj = cols ? (int64_t)cols[tt] : tt;
                    const bool kept = keep == nullptr || keep[jj] != 0;
                    z[jj] = kept ? (tot[q] - c[jj] * sum_r) * inv_n / s[jj] : 0.0;
                }
            }
        }
    }
}

// ---- int8 form ----
// keeps the loads above it issued before the work below it: neither the IR passes (memory clobber) nor the
// machine scheduler (sched_barrier) move them down to their first use
__device__ __forceinline__ void issue_fence() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
}

constexpr int I8P = LOWP_I8_PIECES;
constexpr int I8_SHIFT = 7;             // s_{k+1} = s_k 2^-7: the remainder after piece k is at most s_k / 2 = 64 s_{k+1}
constexpr int PIECE_THREADS = 1024;

// the same value in every thread of the workgroup (wave partials combined in wave order)
__device__ double block_reduce(double v, bool take_max, double* red) {
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        const double w = __shfl_xor(v, o, WAVE);
        v = take_max ? fmax(v, w) : v + w;
    }
    __syncthreads();
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < (int)(blockDim.x / WAVE); ++k) t = take_max ? fmax(t, red[k]) : t + red[k];
    return t;
}

// r -> pieces q_1..q_4 (rows n_total..n_pad-1 zero), scales s_k = 2^(E - 7(k-1)) with s_1 = 2^E the
// smallest such power where max|r| <= 127 s_1 (E >= -1000, so every s_k q_k stays a normal FP64 number),
// and the bound numerator (||t||_2 + gamma_3 ||w||_2)(1 + 2^-20), w_i = sum_k s_k |q_ik| (the FP64 sum of
// the four scaled integer dot products errs by at most gamma_3 sum_i |x_i| w_i).  One workgroup.
__global__ __launch_bounds__(PIECE_THREADS) void k_r_pieces_i8(const double* __restrict__ r, int64_t n_total,
                                                             int64_t n_pad, int8_t* __restrict__ pc,
                                                             DevScalars* __restrict__ sc) {
    __shared__ double red[PIECE_THREADS / WAVE];
    double mx = 0.0;
    for (int64_t i = threadIdx.x; i < n_total; i += blockDim.x) mx = fmax(mx, fabs(r[i]));
    mx = block_reduce(mx, true, red);
    int E = -1000;
    if (mx > 0.0) {
        int e;
        (void)frexp(mx / 127.0, &e);
        if (mx > 127.0 * ldexp(1.0, e)) ++e;    // mx / 127 was rounded down
        E = e > -1000 ? e : -1000;
    }
    double e2 = 0.0, w2 = 0.0;
    for (int64_t i = threadIdx.x; i < n_pad; i += blockDim.x) {
        double t = i < n_total ? r[i] : 0.0;
        double w = 0.0;
#pragma unroll
        for (int k = 0; k < I8P; ++k) {
            const int ek = E - I8_SHIFT * k;
            const double q = fmin(127.0, fmax(-127.0, rint(ldexp(t, -ek))));
            pc[(int64_t)k * n_pad + i] = (int8_t)(int)q;
            const double sq = ldexp(q, ek);
            t -= sq;                              // exact: |t - sq| <= 2^(ek-1) on the grid of t
            w += fabs(sq);
        }
        e2 = fma(t, t, e2);
        w2 = fma(w, w, w2);
    }
    e2 = block_reduce(e2, false, red);
    w2 = block_reduce(w2, false, red);
    if (threadIdx.x == 0) {
        const double u = 1.0 / 9007199254740992.0;
#pragma unroll
        for (int k = 0; k < I8P; ++k) sc->i8_scale[k] = ldexp(1.0, E - I8_SHIFT * k);
        sc->i8_a = (sqrt(e2) + 3.0 * u / (1.0 - 3.0 * u) * sqrt(w2)) * (1.0 + 1.0 / 1048576.0);
    }
}

// The scan is a matrix-vector product bound by HBM: each wavefront streams I8_COLS columns at a time, lane l
// reading rows 16 l .. 16 l + 15 of a 1,024-row chunk of each (one 1 KB coalesced load per column and chunk),
// and multiplies every 4-byte word into the four pieces' words with v_dot4_i32_i8 (exact int32 sums:
// |x_i q_ik| <= 128 * 127 < 2^14 and a lane sees at most 2^15 rows for n <= 2^21, so a lane's sum stays below
// 2^29, as wave_isum needs).  The pieces sit in LDS (16-byte
// reads at 16-byte lane strides).  The next chunk's loads are in flight while the current one is multiplied.
// The last, partial chunk reads each word that starts past the last row at the last word instead (in bounds);
// the pieces are zero on every row past n_total, so those products vanish.
constexpr int I8_COLS = 4;
constexpr int64_t I8_CHUNK = (int64_t)WAVE * 16;

// exact sum over the wavefront of per-lane int32 values below 2^29 in magnitude (4-lane partials stay below
// 2^31; from there on the sums are FP64 integers below 2^53)
__device__ __forceinline__ double wave_isum(int v) {
    v += __shfl_xor(v, 1, WAVE);
    v += __shfl_xor(v, 2, WAVE);
    double d = (double)v;
#pragma unroll
    for (int o = 4; o < WAVE; o <<= 1) d += __shfl_xor(d, o, WAVE);
    return d;
}

// KEEP: a keep array is given (a template parameter rather than a null test: a pointer chosen at run time between
// it and a constant turns the load into one the wait counters cannot order, and every chunk would then wait for
// all loads in flight)
template <bool PLDS, bool KEEP>
__global__ __launch_bounds__(256) void k_scan_i8(const int8_t* __restrict__ X, int64_t ldx, int64_t n_total,
                                                 int64_t n_pad, const int8_t* __restrict__ pieces,
                                                 const int32_t* __restrict__ cols, const int64_t* __restrict__ len_dev,
                                                 int64_t len_host, const DevScalars* __restrict__ sc,
                                                 const double* __restrict__ c, const double* __restrict__ s,
                                                 const uint8_t* __restrict__ keep, double* __restrict__ z) {
    extern __shared__ v4i32 pl8[];
    const int64_t len = len_dev ? *len_dev : len_host;
    const int wpb = blockDim.x / WAVE;
    const int64_t nunits = (len + I8_COLS - 1) / I8_COLS;
    const int64_t gw0 = (int64_t)blockIdx.x * wpb;
    if (gw0 >= nunits) return;
    const int8_t* P = pieces;
    if constexpr (PLDS) {
        const v4i32* src = reinterpret_cast<const v4i32*>(pieces);
        const int64_t nv = (int64_t)I8P * n_pad / 16;
        for (int64_t k = threadIdx.x; k < nv; k += blockDim.x) pl8[k] = src[k];
        __syncthreads();
        P = reinterpret_cast<const int8_t*>(pl8);
    }
    const int lane = threadIdx.x & (WAVE - 1);
    const double sum_r = sc->sum_r;
    const double inv_n = 1.0 / (double)sc->n_rows;
    double sk[I8P];
#pragma unroll
    for (int k = 0; k < I8P; ++k) sk[k] = sc->i8_scale[k];
    const int64_t nch = (n_total + I8_CHUNK - 1) / I8_CHUNK;   // chunks per column, the last partial
    const int64_t last_word = (n_total - 1) & ~(int64_t)15;
    const int64_t ustride = (int64_t)gridDim.x * wpb;
    const int8_t* pl = P + 16 * lane;
    // column cc of unit u (entries past the end of the list read column 0; their sums are not written); the
    // index load is unconditional (clamped), so nothing waits for it before its use
    auto column = [&](int64_t u, int cc) -> int64_t {
        const int64_t t_ = u * I8_COLS + cc;
        const int64_t jl = cols[t_ < len ? t_ : len - 1];
        return t_ < len ? jl : 0;
    };
    // the unit is the same in every lane (readfirstlane makes that visible to the compiler, so the column
    // indices and statistics live in scalar registers)
    int64_t unit = __builtin_amdgcn_readfirstlane((int)(gw0 + threadIdx.x / WAVE));
    int64_t jc[I8_COLS];
#pragma unroll
    for (int cc = 0; cc < I8_COLS; ++cc) jc[cc] = column(unit < nunits ? unit : gw0, cc);
    for (; unit < nunits; unit += ustride) {
        // the next unit's column indices a unit ahead, this unit's statistics at its start
        int64_t jn[I8_COLS];
        const int64_t un = unit + ustride < nunits ? unit + ustride : unit;
#pragma unroll
        for (int cc = 0; cc < I8_COLS; ++cc) jn[cc] = column(un, cc);
        double cj[I8_COLS], sj[I8_COLS];
        bool kept[I8_COLS];
        const int8_t* xc[I8_COLS];
#pragma unroll
        for (int cc = 0; cc < I8_COLS; ++cc) {
            cj[cc] = c[jc[cc]];
            sj[cc] = s[jc[cc]];
            kept[cc] = KEEP ? keep[jc[cc]] != 0 : true;
            xc[cc] = X + jc[cc] * ldx;
        }
        int acc[I8_COLS][I8P];
#pragma unroll
        for (int cc = 0; cc < I8_COLS; ++cc)
#pragma unroll
            for (int k = 0; k < I8P; ++k) acc[cc][k] = 0;
        auto load = [&](v4i32 (&dst)[I8_COLS], int64_t ch) {
            const int64_t row = ch * I8_CHUNK + 16 * lane;
            const int64_t rl = row < last_word ? row : last_word;
#pragma unroll
            for (int cc = 0; cc < I8_COLS; ++cc) dst[cc] = *reinterpret_cast<const v4i32*>(xc[cc] + rl);
        };
        auto compute = [&](const v4i32 (&w)[I8_COLS], int64_t ch) {
            v4i32 pw[I8P];
#pragma unroll
            for (int k = 0; k < I8P; ++k) pw[k] = *reinterpret_cast<const v4i32*>(pl + k * n_pad + ch * I8_CHUNK);
#pragma unroll
            for (int cc = 0; cc < I8_COLS; ++cc)
#pragma unroll
                for (int k = 0; k < I8P; ++k)
#pragma unroll
                    for (int d = 0; d < 4; ++d) acc[cc][k] = __builtin_amdgcn_sdot4(w[cc][d], pw[k][d], acc[cc][k], false);
        };
        // pairs of chunks, two register sets taking turns (no branch between a prefetch and its use)
        v4i32 wa[I8_COLS], wb[I8_COLS];
        load(wa, 0);
        issue_fence();
        for (int64_t ch = 0; ch + 1 < nch; ch += 2) {
            load(wb, ch + 1);
            issue_fence();
            compute(wa, ch);
            load(wa, ch + 2 < nch ? ch + 2 : nch - 1);
            issue_fence();
            compute(wb, ch + 1);
        }
        if (nch & 1) compute(wa, nch - 1);
        // exact column sums per piece, scaled (exact) and added in FP64; lane cc writes column cc
        double zv = 0.0;
#pragma unroll
        for (int cc = 0; cc < I8_COLS; ++cc) {
            double v[I8P];
#pragma unroll
            for (int k = 0; k < I8P; ++k) v[k] = wave_isum(acc[cc][k]) * sk[k];
            const double tot = ((v[0] + v[1]) + v[2]) + v[3];
            const double zc = kept[cc] ? (tot - cj[cc] * sum_r) * inv_n / sj[cc] : 0.0;
            zv = lane == cc ? zc : zv;
        }
        if (lane < I8_COLS && unit * I8_COLS + lane < len) {
            int64_t jw = jc[0];
#pragma unroll
            for (int cc = 1; cc < I8_COLS; ++cc) jw = lane == cc ? jc[cc] : jw;
            z[jw] = zv;
        }
#pragma unroll
        for (int cc = 0; cc < I8_COLS; ++cc) jc[cc] = jn[cc];
    }
}

// Bound on |z~_j - z_j| (see the header of this file): A ||x_j||_2 / (n s_j), ||x_j||_2^2 = n (s_j^2 + c_j^2), with
//   BF16 form: A = (u_r + (1 + 2^-7) gamma_c + gamma_64) ||r||_2, gamma_c for FP32 chunks of 64 rows,
//   int8 form: A = sc->i8_a + gamma_64 ||r||_2   (gamma_64 covers the FP64 scan that re-takes the decisions)
__device__ __forceinline__ double lowp_bound(double cj, double sj, double n, double A) {
    return A * sqrt(n * (sj * sj + cj * cj)) / (n * sj);
}

// flag[j] = 1 when a decision on z~_j lies within its bound: the check against lam (only for
// j in in_s and not in excl), or the strong-rule threshold thr2 (when thr2 >= 0)
__global__ void k_band(const int32_t* __restrict__ cols, const int64_t* __restrict__ len_dev, const double* __restrict__ z,
                       const double* __restrict__ c, const double* __restrict__ s, const DevScalars* __restrict__ sc,
                       double coef, int i8, double lam, const uint8_t* __restrict__ in_s,
                       const uint8_t* __restrict__ excl, double thr2, uint8_t* __restrict__ flag,
                       double* __restrict__ err_out) {
    const int64_t len = *len_dev;
    const double n = (double)sc->n_rows;
    const double A = coef * sqrt(sc->rss) + (i8 ? sc->i8_a : 0.0);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (int64_t)gridDim.x * blockDim.x) {
        const int j = cols[t];
        const double d = lowp_bound(c[j], s[j], n, A) + 1e-14 * fabs(z[j]);
        const double az = fabs(z[j]);
        bool f = false;
        if ((in_s == nullptr || in_s[j]) && (excl == nullptr || !excl[j]) && fabs(az - lam) <= d) f = true;
        if (thr2 >= 0.0 && fabs(az - thr2) <= d) f = true;
        if (flag && f) flag[j] = 1;
        if (err_out) err_out[j] = d;
    }
}

// post-convergence check on (corrected) z: violators join the working set
__global__ void k_viol(const int32_t* __restrict__ cols, const int64_t* __restrict__ len_dev, const double* __restrict__ z,
                       const uint8_t* __restrict__ in_s, uint8_t* __restrict__ inE, double lam,
                       uint32_t* __restrict__ nviol) {
    const int64_t len = *len_dev;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (int64_t)gridDim.x * blockDim.x) {
        const int j = cols[t];
        if (in_s[j] && !inE[j] && fabs(z[j]) > lam) {
            inE[j] = 1;
            atomicAdd(nviol, 1u);
        }
    }
}

int grid_for(int64_t work, int per_block, int max_blocks) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > max_blocks) g = max_blocks;
    return (int)g;
}

}  // namespace

int64_t lowp_pad(int64_t n_total) { return (n_total + SCAN_KC - 1) / SCAN_KC * SCAN_KC; }

// rows of each int8 piece: whole 1,024-row chunks (the scan reads the pieces of every row of a chunk)
int64_t lowp_pad_i8(int64_t n_total) { return (n_total + I8_CHUNK - 1) / I8_CHUNK * I8_CHUNK; }

size_t lowp_piece_bytes(int64_t n_total) {
    const size_t bf = (size_t)NPIECE * lowp_pad(n_total) * sizeof(__bf16), i8 = (size_t)I8P * lowp_pad_i8(n_total);
    return bf > i8 ? bf : i8;
}

double lowp_coef() {
    const double u8 = 1.0 / 256.0, u24 = 1.0 / 16777216.0, u53 = 1.0 / 9007199254740992.0;
    double ur = 1.0;
    for (int k = 0; k < NPIECE; ++k) ur *= (u8 + u24);  // residual left after the pieces, relative to |r_i|
    const double gc = SCAN_PROMOTE * u24 / (1.0 - SCAN_PROMOTE * u24);   // FP32 sums of SCAN_PROMOTE products
    const double g64 = 65536.0 * u53;                   // FP64 chunk and piece additions (n / 64 + 3 terms)
    return ur + (1.0 + 1.0 / 128.0) * gc + g64;
}

bool lowp_supported(const Mat& m) {
    return m.xtype == 2 && ((uintptr_t)m.X % 16 == 0) && (m.ldx % 16 == 0) && m.n_total <= (int64_t(1) << 21);
}

hipError_t launch_r_pieces(const double* r, int64_t n_total, __bf16* pieces, hipStream_t st) {
    const int64_t n_pad = lowp_pad(n_total);
    k_r_pieces<<<grid_for(n_pad, 256, 1024), 256, 0, st>>>(r, n_total, n_pad, pieces);
    return hipGetLastError();
}

hipError_t launch_scan_bf16(const Mat& m, const __bf16* pieces, const int32_t* cols, const int64_t* len_dev,
                            int64_t len_host, const DevScalars* sc, const double* c, const double* s,
                            const uint8_t* keep, double* z, hipStream_t st) {
    const int64_t n_pad = lowp_pad(m.n_total);
    const size_t lds = (size_t)NPIECE * n_pad * sizeof(__bf16);
    const int64_t work = len_dev ? m.p : len_host;
    const int64_t groups = (work + 15) / 16;
    const int threads = 256, wpb = threads / WAVE;
    if (lds <= 64 * 1024) {
        const int per_cu = lds <= 40 * 1024 ? 4 : 2;
        const int g = grid_for(groups, wpb, device_cu_count() * per_cu);
        k_scan_bf16<true><<<g, threads, lds, st>>>((const int8_t*)m.X, m.ldx, m.n_total, n_pad, pieces, cols, len_dev,
                                                   len_host, sc, c, s, keep, z);
    } else {
        const int g = grid_for(groups, wpb, device_cu_count() * 8);
        k_scan_bf16<false><<<g, threads, 0, st>>>((const int8_t*)m.X, m.ldx, m.n_total, n_pad, pieces, cols, len_dev,
                                                  len_host, sc, c, s, keep, z);
    }
    return hipGetLastError();
}

hipError_t launch_r_pieces_i8(const double* r, int64_t n_total, int8_t* pieces, DevScalars* sc, hipStream_t st) {
    k_r_pieces_i8<<<1, PIECE_THREADS, 0, st>>>(r, n_total, lowp_pad_i8(n_total), pieces, sc);
    return hipGetLastError();
}

hipError_t launch_scan_i8(const Mat& m, const int8_t* pieces, const int32_t* cols, const int64_t* len_dev,
                          int64_t len_host, const DevScalars* sc, const double* c, const double* s,
                          const uint8_t* keep, double* z, hipStream_t st) {
    if (!cols) return hipErrorInvalidValue;   // the kernel reads the column list unconditionally
    const int64_t n_pad = lowp_pad_i8(m.n_total);
    const size_t lds = (size_t)I8P * n_pad;
    const int64_t work = len_dev ? m.p : len_host;
    const int64_t groups = (work + I8_COLS - 1) / I8_COLS;
    const int threads = 256, wpb = threads / WAVE;
    const int8_t* X = (const int8_t*)m.X;
    const bool plds = lds <= 64 * 1024;
    const int g = grid_for(groups, wpb, device_cu_count() * (plds ? (lds <= 40 * 1024 ? 4 : 2) : 8));
    const size_t dyn = plds ? lds : 0;
    if (plds && keep)
        k_scan_i8<true, true><<<g, threads, dyn, st>>>(X, m.ldx, m.n_total, n_pad, pieces, cols, len_dev, len_host, sc,
                                                       c, s, keep, z);
    else if (plds)
        k_scan_i8<true, false><<<g, threads, dyn, st>>>(X, m.ldx, m.n_total, n_pad, pieces, cols, len_dev, len_host, sc,
                                                        c, s, keep, z);
    else if (keep)
        k_scan_i8<false, true><<<g, threads, dyn, st>>>(X, m.ldx, m.n_total, n_pad, pieces, cols, len_dev, len_host, sc,
                                                        c, s, keep, z);
    else
        k_scan_i8<false, false><<<g, threads, dyn, st>>>(X, m.ldx, m.n_total, n_pad, pieces, cols, len_dev, len_host,
                                                         sc, c, s, keep, z);
    return hipGetLastError();
}

hipError_t launch_band(const int32_t* cols, const int64_t* len_dev, const double* z, const double* c, const double* s,
                       const DevScalars* sc, double lam, const uint8_t* in_s, const uint8_t* excl, double thr2,
                       uint8_t* flag, double* err_out, int64_t p, bool i8, hipStream_t st) {
    const double coef = i8 ? 65536.0 / 9007199254740992.0 : lowp_coef();
    k_band<<<grid_for(p, 256, device_cu_count() * 8), 256, 0, st>>>(cols, len_dev, z, c, s, sc, coef, i8 ? 1 : 0,
                                                                     lam, in_s, excl, thr2, flag, err_out);
    return hipGetLastError();
}

hipError_t launch_viol(const int32_t* cols, const int64_t* len_dev, const double* z, const uint8_t* in_s, uint8_t* inE,
                       double lam, uint32_t* nviol, int64_t p, hipStream_t st) {
    k_viol<<<grid_for(p, 256, device_cu_count() * 8), 256, 0, st>>>(cols, len_dev, z, in_s, inE, lam, nviol);
    return hipGetLastError();
}

}  // namespace blk
