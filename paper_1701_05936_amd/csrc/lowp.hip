// Precision form of the scan: int8 design codes on BF16 matrix cores.
//
// z_j = (x_j' r - c_j sum(r)) / (n s_j) is computed as Z = X_T' [r1 r2 r3] with
//   r1 = bf16(r), r2 = bf16(r - r1), r3 = bf16(r - r1 - r2)   (residual pieces, FP64 differences)
// on v_mfma_f32_16x16x32_bf16.  Int8 codes convert to BF16 exactly (|x| <= 256),
// each product x * r_c is exact in FP32, the FP32 accumulator is promoted to FP64
// after every 32-row MFMA step, and the three pieces are added in FP64.  The error of z_j is
// bounded column by column (lowp_bound); a decision whose value lies within that
// bound of its threshold is taken again on the exact FP64 scan.
//
// Tile: a wavefront owns 16 columns of the scan list; lane (m = l%16, g = l/16)
// loads 32 consecutive codes of column m (rows i0 + 32g ..) per 128-row batch, so
// a wavefront load covers 16 full 128-byte segments.  The MFMA reduction order
// over rows is free, so step s of a batch feeds rows i0 + 32g + 8s .. +7 of lane
// group g to both operands.  The residual pieces sit in LDS.
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
constexpr int SCAN_PROMOTE = 32; // rows per FP32 chunk: the accumulator goes to FP64 after every MFMA step
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
        const bool bpiece = m < NPIECE;
        const __bf16* pr = P + (int64_t)(bpiece ? m : 0) * n_pad;
        // one batch of SCAN_KC rows: 4 MFMA steps of 32 rows, each FP32 result promoted to FP64
        auto batch = [&](const v4i32& w0, const v4i32& w1, int64_t ib) {
            // residual pieces of the 4 steps first (one wait for all), zero in lanes past the pieces
            bf16x8 bq[4];
            const bf16x8 bzero = {};
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const bf16x8 t = *reinterpret_cast<const bf16x8*>(pr + ib + lane_row(g, st));
                bq[st] = bpiece ? t : bzero;
            }
            const uint32_t wd[8] = {(uint32_t)w0.x, (uint32_t)w0.y, (uint32_t)w0.z, (uint32_t)w0.w,
                                    (uint32_t)w1.x, (uint32_t)w1.y, (uint32_t)w1.z, (uint32_t)w1.w};
            // the 4 steps go to the matrix cores back to back; each 32-row FP32 result is then promoted
            f32x4 r[4];
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const bf16x8 a = codes_to_bf16(wd[2 * st], wd[2 * st + 1]);
                const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
                r[st] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bq[st], zero, 0, 0, 0);
            }
#pragma unroll
            for (int st = 0; st < 4; ++st)
#pragma unroll
                for (int q = 0; q < 4; ++q) acc64[q] += (double)r[st][q];
        };
        // SCAN_U batches' loads are issued before the first is used (memory parallelism per wave)
        int64_t i0 = 0;
        for (; i0 + SCAN_U * SCAN_KC <= nfull; i0 += SCAN_U * SCAN_KC) {
            v4i32 w[SCAN_U][2];
#pragma unroll
            for (int u = 0; u < SCAN_U; ++u) {
                w[u][0] = (v4i32){0, 0, 0, 0};
                w[u][1] = (v4i32){0, 0, 0, 0};
                if (valid) {
                    const v4i32* xp = reinterpret_cast<const v4i32*>(xc + i0 + u * SCAN_KC + 16 * g);
                    w[u][0] = xp[0];
                    w[u][1] = xp[4];
                }
            }
#pragma unroll
            for (int u = 0; u < SCAN_U; ++u) batch(w[u][0], w[u][1], i0 + u * SCAN_KC);
        }
        for (; i0 < nfull; i0 += SCAN_KC) {
            v4i32 w0 = {0, 0, 0, 0}, w1 = {0, 0, 0, 0};
            if (valid) {
                const v4i32* xp = reinterpret_cast<const v4i32*>(xc + i0 + 16 * g);
                w0 = xp[0];
                w1 = xp[4];
            }
            batch(w0, w1, i0);
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
#pragma unroll
            for (int st = 0; st < 4; ++st) {
                const bf16x8 a = codes_to_bf16(wd[2 * st], wd[2 * st + 1]);
                bf16x8 b = {};
                if (bpiece) b = *reinterpret_cast<const bf16x8*>(pr + i0 + lane_row(g, st));
                const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
                const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, zero, 0, 0, 0);
#pragma unroll
                for (int q = 0; q < 4; ++q) acc64[q] += (double)acc[q];
            }
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

// Bound on |z~_j - z_j| for the BF16 scan (see lowp.hip header):
//   (u_r + (1 + 2^-7) gamma_32 + gamma64) * ||x_j||_2 ||r||_2 / (n s_j),  ||x_j||_2^2 = n (s_j^2 + c_j^2)
__device__ __forceinline__ double lowp_bound(double cj, double sj, double n, double rnorm, double coef) {
    return coef * sqrt(n * (sj * sj + cj * cj)) * rnorm / (n * sj);
}

// flag[j] = 1 when a decision on z~_j lies within its bound: the check against lam (only for
// j in in_s and not in excl), or the strong-rule threshold thr2 (when thr2 >= 0)
__global__ void k_band(const int32_t* __restrict__ cols, const int64_t* __restrict__ len_dev, const double* __restrict__ z,
                       const double* __restrict__ c, const double* __restrict__ s, const DevScalars* __restrict__ sc,
                       double coef, double lam, const uint8_t* __restrict__ in_s, const uint8_t* __restrict__ excl,
                       double thr2, uint8_t* __restrict__ flag, double* __restrict__ err_out) {
    const int64_t len = *len_dev;
    const double n = (double)sc->n_rows;
    const double rnorm = sqrt(sc->rss);
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (int64_t)gridDim.x * blockDim.x) {
        const int j = cols[t];
        const double d = lowp_bound(c[j], s[j], n, rnorm, coef) + 1e-14 * fabs(z[j]);
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

double lowp_coef() {
    const double u8 = 1.0 / 256.0, u24 = 1.0 / 16777216.0, u53 = 1.0 / 9007199254740992.0;
    double ur = 1.0;
    for (int k = 0; k < NPIECE; ++k) ur *= (u8 + u24);  // residual left after the pieces, relative to |r_i|
    const double g32 = SCAN_PROMOTE * u24 / (1.0 - SCAN_PROMOTE * u24);
    const double g64 = 65536.0 * u53;                   // FP64 chunk and piece additions (n / 32 + 3 terms)
    return ur + (1.0 + 1.0 / 128.0) * g32 + g64;
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

hipError_t launch_band(const int32_t* cols, const int64_t* len_dev, const double* z, const double* c, const double* s,
                       const DevScalars* sc, double lam, const uint8_t* in_s, const uint8_t* excl, double thr2,
                       uint8_t* flag, double* err_out, int64_t p, hipStream_t st) {
    k_band<<<grid_for(p, 256, device_cu_count() * 8), 256, 0, st>>>(cols, len_dev, z, c, s, sc, lowp_coef(), lam,
                                                                     in_s, excl, thr2, flag, err_out);
    return hipGetLastError();
}

hipError_t launch_viol(const int32_t* cols, const int64_t* len_dev, const double* z, const uint8_t* in_s, uint8_t* inE,
                       double lam, uint32_t* nviol, int64_t p, hipStream_t st) {
    k_viol<<<grid_for(p, 256, device_cu_count() * 8), 256, 0, st>>>(cols, len_dev, z, in_s, inE, lam, nviol);
    return hipGetLastError();
}

}  // namespace blk
