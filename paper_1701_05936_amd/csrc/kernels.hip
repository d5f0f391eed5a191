// HIP kernels of the pathwise lasso for CDNA4 (gfx950, wave64).
//
// Column-major X is streamed once per scan: one wavefront owns one column at
// a time, reads it with 16-byte loads (1 KiB per wavefront instruction), takes
// the residual from LDS and reduces across the wavefront.  Coordinate descent
// is one persistent workgroup that keeps the residual in registers.  All
// reductions have a fixed order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace blk {

namespace {

constexpr int WAVE = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

// Block-wide sum with a fixed order: wave sums, then wave 0 adds the partials in wave order.
// Every thread gets the result.  `buf` holds at least blockDim.x/64 doubles.
__device__ double block_sum(double v, double* buf) {
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) buf[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < nw; ++k) t += buf[k];
    return t;
}

// Broadcast lane 0's value as a wave-uniform (scalar) value.
__device__ __forceinline__ double uniform(double v) {
    uint64_t b = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ double soft_threshold(double u, double l) {
    return u > l ? u - l : (u < -l ? u + l : 0.0);
}

template <typename XT>
__device__ __forceinline__ double xval(XT v) { return (double)v; }

// Raw buffer resource over one column: loads past num_records bytes return 0, so the
// ragged tail of a column needs no branch.  0x00020000 is the gfx9-family word 3.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t column_rsrc(const void* base, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}
template <typename XT>
__device__ __forceinline__ double buf_x(__amdgpu_buffer_rsrc_t rs, int voff);
template <>
__device__ __forceinline__ double buf_x<double>(__amdgpu_buffer_rsrc_t rs, int voff) {
    typedef unsigned int u2 __attribute__((ext_vector_type(2)));
    u2 v = __builtin_amdgcn_raw_buffer_load_b64(rs, voff, 0, 0);
    return __builtin_bit_cast(double, v);
}
template <>
__device__ __forceinline__ double buf_x<float>(__amdgpu_buffer_rsrc_t rs, int voff) {
    unsigned int v = __builtin_amdgcn_raw_buffer_load_b32(rs, voff, 0, 0);
    return (double)__builtin_bit_cast(float, v);
}
template <>
__device__ __forceinline__ double buf_x<int8_t>(__amdgpu_buffer_rsrc_t rs, int voff) {
    unsigned char v = __builtin_amdgcn_raw_buffer_load_b8(rs, voff, 0, 0);
    return (double)(int)(int8_t)v;
}

// ---- vector loads of W consecutive elements (16 bytes) -----------------------------------
typedef double v2f64 __attribute__((ext_vector_type(2)));
typedef float v4f32 __attribute__((ext_vector_type(4)));
typedef int v4i32 __attribute__((ext_vector_type(4)));

template <typename XT> struct Vec16;
template <> struct Vec16<double> { static constexpr int W = 2;  using T = v2f64; };
template <> struct Vec16<float>  { static constexpr int W = 4;  using T = v4f32; };
template <> struct Vec16<int8_t> { static constexpr int W = 16; using T = v4i32; };

template <typename XT>
__device__ __forceinline__ void unpack(const typename Vec16<XT>::T& v, double* o);
template <>
__device__ __forceinline__ void unpack<double>(const v2f64& v, double* o) { o[0] = v.x; o[1] = v.y; }
template <>
__device__ __forceinline__ void unpack<float>(const v4f32& v, double* o) {
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
template <>
__device__ __forceinline__ void unpack<int8_t>(const v4i32& v, double* o) {
    const int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int b = 0; b < 4; ++b) o[q * 4 + b] = (double)(int)(int8_t)((w[q] >> (8 * b)) & 0xff);
}

// Dot product of column x (n elements) with r (LDS or global), by one wavefront.
// VEC: 16-byte vector loads (x must be 16-byte aligned); otherwise element loads.
template <typename XT, bool VEC, int U>
__device__ __forceinline__ double wave_col_dot(const XT* __restrict__ x, const double* __restrict__ r, int64_t n) {
    const int lane = threadIdx.x & (WAVE - 1);
    double acc0 = 0.0, acc1 = 0.0;
    int64_t base = 0;
    if constexpr (VEC && sizeof(XT) == 1) {
        // int8 codes: lane l takes the 4-byte word of rows 4l .. 4l+3 of each 256-row step (one coalesced
        // 256-byte load per wavefront), so its residual values are 32 contiguous bytes at a 32-byte lane stride
        // (16 codes per lane would put the lanes 128 bytes apart: LDS bank conflicts, 8 bytes of r per code)
        constexpr int64_t STEP = (int64_t)WAVE * 4;
        constexpr int UI = 2 * U;
        const int64_t nfull = (n / STEP) * STEP;
        auto word = [&](int v, const double* rr, double acc) {
            acc = fma((double)(int)(int8_t)(v & 0xff), rr[0], acc);
            acc = fma((double)(int)(int8_t)((v >> 8) & 0xff), rr[1], acc);
            acc = fma((double)(int)(int8_t)((v >> 16) & 0xff), rr[2], acc);
            return fma((double)(v >> 24), rr[3], acc);
        };
        for (; base + UI * STEP <= nfull; base += UI * STEP) {
            int v[UI];
#pragma unroll
            for (int u = 0; u < UI; ++u)
                v[u] = __builtin_nontemporal_load(reinterpret_cast<const int*>(x + base + u * STEP + 4 * lane));
#pragma unroll
            for (int u = 0; u < UI; ++u) {
                const double* rr = r + base + u * STEP + 4 * lane;
                if (u & 1) acc1 = word(v[u], rr, acc1);
                else acc0 = word(v[u], rr, acc0);
            }
        }
        for (; base < nfull; base += STEP)
            acc0 = word(*reinterpret_cast<const int*>(x + base + 4 * lane), r + base + 4 * lane, acc0);
    } else if constexpr (VEC) {
        using VT = typename Vec16<XT>::T;
        constexpr int W = Vec16<XT>::W;
        constexpr int64_t STEP = (int64_t)WAVE * W;
        const int64_t nfull = (n / STEP) * STEP;
        for (; base + U * STEP <= nfull; base += U * STEP) {
            VT v[U];
#pragma unroll
            for (int u = 0; u < U; ++u)
                v[u] = __builtin_nontemporal_load(reinterpret_cast<const VT*>(x + base + u * STEP + lane * W));
#pragma unroll
            for (int u = 0; u < U; ++u) {
                double xd[W];
                unpack<XT>(v[u], xd);
                const double* rr = r + base + u * STEP + lane * W;
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    if (u & 1) acc1 = fma(xd[w], rr[w], acc1);
                    else acc0 = fma(xd[w], rr[w], acc0);
                }
            }
        }
        for (; base < nfull; base += STEP) {
            VT v = *reinterpret_cast<const VT*>(x + base + lane * W);
            double xd[W];
            unpack<XT>(v, xd);
            const double* rr = r + base + lane * W;
#pragma unroll
            for (int w = 0; w < W; ++w) acc0 = fma(xd[w], rr[w], acc0);
        }
    }
    for (int64_t i = base + lane; i < n; i += WAVE) acc1 = fma(xval(x[i]), r[i], acc1);
    return wave_sum(acc0 + acc1);
}

// ---- column statistics -----------------------------------------------------------------------
template <typename XT, bool MASK>
__global__ __launch_bounds__(256) void k_colstats(const XT* __restrict__ X, int64_t ldx, int64_t n_total, int64_t p,
                                                  const uint8_t* __restrict__ mask, int64_t n_rows,
                                                  double* __restrict__ c, double* __restrict__ s,
                                                  uint8_t* __restrict__ keep, bool vec) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t wid = (int64_t)blockIdx.x * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int64_t nw = (int64_t)gridDim.x * (blockDim.x / WAVE);
    const double inv_n = 1.0 / (double)n_rows;
    for (int64_t j = wid; j < p; j += nw) {
        const XT* x = X + j * ldx;
        double mean, var;
        if constexpr (sizeof(XT) == 1) {
            // integer codes: exact sums
            int64_t s1 = 0, s2 = 0;
            if (vec) {
                // 16-byte words, four per lane in flight (a word that starts past the last row is read at the
                // last word instead and cleared); sum x and x^2 with v_dot4_i32_i8, exact in int32 per lane
                // (a lane sees at most n / 64 rows: |sum x^2| < 2^14 n / 64 < 2^31 for n <= 2^23)
                const int64_t last_word = (n_total - 1) & ~(int64_t)15;
                int a1 = 0, a2 = 0;
                for (int64_t base = 16 * lane; base < n_total; base += 4 * 16 * WAVE) {
                    v4i32 w[4], mk[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int64_t r0 = base + u * 16 * WAVE;
                        const int64_t rl = r0 < last_word ? r0 : last_word;
                        w[u] = *reinterpret_cast<const v4i32*>(x + rl);
                        if constexpr (MASK) mk[u] = *reinterpret_cast<const v4i32*>(mask + rl);
                    }
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int64_t r0 = base + u * 16 * WAVE;
#pragma unroll
                        for (int d = 0; d < 4; ++d) {
                            const int64_t nv = n_total - r0 - 4 * d;
                            uint32_t keepb = nv >= 4 ? 0xFFFFFFFFu : (nv <= 0 ? 0u : ((1u << (8 * (int)nv)) - 1u));
                            if constexpr (MASK) {
                                const uint32_t mv = (uint32_t)mk[u][d];
                                keepb &= (((((mv & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | mv) & 0x80808080u) >> 7) * 0xFFu;
                            }
                            const int v = (int)((uint32_t)w[u][d] & keepb);
                            a1 = __builtin_amdgcn_sdot4(v, 0x01010101, a1, false);
                            a2 = __builtin_amdgcn_sdot4(v, v, a2, false);
                        }
                    }
                }
                s1 = a1;
                s2 = a2;
            } else {
                for (int64_t i = lane; i < n_total; i += WAVE) {
                    if (MASK && !mask[i]) continue;
                    int64_t v = (int64_t)x[i];
                    s1 += v;
                    s2 += v * v;
                }
            }
            s1 = wave_sum_i64(s1);
            s2 = wave_sum_i64(s2);
            mean = (double)s1 * inv_n;
            // (n s2 - s1^2) / n^2, numerator exact in 64-bit integers
            var = (double)(n_rows * s2 - s1 * s1) * inv_n * inv_n;
        } else {
            // E consecutive rows per lane and wave-wide word of E * 64 rows: lane l takes rows E l .. E l + E - 1
            // of every word, one accumulator per position in the word.  With 16-byte aligned columns (vec) the
            // whole words are read as 16-byte loads, four words in flight; otherwise element by element in the
            // same order, so both give the same sums.  Rows of the last, partial word are read one by one.
            constexpr int E = 16 / (int)sizeof(XT);
            constexpr int64_t WR = (int64_t)E * WAVE;
            const int64_t nw = n_total / WR;   // whole words
            const int64_t l0 = (int64_t)E * lane;
            auto word = [&](int64_t k, double (&v)[E], bool (&ok)[E]) {
                const int64_t r = k * WR + l0;
                if (vec) {
                    if constexpr (E == 2) {
                        const double2 w = *reinterpret_cast<const double2*>(x + r);
                        v[0] = (double)w.x;
                        v[1] = (double)w.y;
                    } else {
                        const float4 w = *reinterpret_cast<const float4*>(x + r);
                        v[0] = (double)w.x;
                        v[1] = (double)w.y;
                        v[2] = (double)w.z;
                        v[3] = (double)w.w;
                    }
                    uint32_t mb = 0xFFFFFFFFu;
                    if constexpr (MASK) {
                        if constexpr (E == 2) mb = *reinterpret_cast<const uint16_t*>(mask + r);
                        else mb = *reinterpret_cast<const uint32_t*>(mask + r);
                    }
#pragma unroll
                    for (int e = 0; e < E; ++e) ok[e] = ((mb >> (8 * e)) & 0xFFu) != 0;
                } else {
#pragma unroll
                    for (int e = 0; e < E; ++e) {
                        ok[e] = !MASK || mask[r + e];
                        v[e] = ok[e] ? (double)x[r + e] : 0.0;
                    }
                }
            };
            auto tail = [&](double (&v)[E], bool (&ok)[E]) {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int64_t r = nw * WR + l0 + e;
                    ok[e] = r < n_total && (!MASK || mask[r]);
                    v[e] = ok[e] ? (double)x[r] : 0.0;
                }
            };
            // One pass: each lane keeps the count, mean and sum of squared deviations of its rows, taking four
            // words at a time (their own mean and squared deviations, then the pairwise update of Chan, Golub
            // and LeVeque: M2 = M2a + M2b + d^2 na nb / (na + nb)); the lanes are then combined the same way.
            // X is read once; rows outside the fit add nothing.
            double ln = 0.0, lm = 0.0, lq = 0.0;
            auto merge = [](double& na, double& ma, double& qa, double nb, double mb, double qb) {
                const double nn = na + nb;
                if (nb > 0.0) {
                    const double d = mb - ma, f = nb / nn;
                    ma = fma(d, f, ma);
                    qa = qa + qb + d * d * na * f;
                    na = nn;
                }
            };
            auto chunk = [&](const double* v, const bool* ok, int cnt_max) {
                double cnt = 0.0, sm = 0.0;
                for (int i = 0; i < cnt_max; ++i) {
                    cnt += ok[i] ? 1.0 : 0.0;
                    sm += ok[i] ? v[i] : 0.0;
                }
                const double cm = cnt > 0.0 ? sm / cnt : 0.0;
                double cq = 0.0;
                for (int i = 0; i < cnt_max; ++i) {
                    const double d = ok[i] ? v[i] - cm : 0.0;
                    cq = fma(d, d, cq);
                }
                merge(ln, lm, lq, cnt, cm, cq);
            };
            {
                int64_t k = 0;
                for (; k + 4 <= nw; k += 4) {
                    double v[4 * E];
                    bool ok[4 * E];
#pragma unroll
                    for (int u = 0; u < 4; ++u)
                        word(k + u, *reinterpret_cast<double(*)[E]>(v + u * E), *reinterpret_cast<bool(*)[E]>(ok + u * E));
                    chunk(v, ok, 4 * E);
                }
                for (; k <= nw; ++k) {
                    double v[E];
                    bool ok[E];
                    if (k < nw) word(k, v, ok);
                    else tail(v, ok);
                    chunk(v, ok, E);
                }
            }
            // lanes combined pairwise, lane l with lane l ^ 2^i (every lane ends with the same figures)
#pragma unroll
            for (int sh = 1; sh < WAVE; sh <<= 1) {
                const double on = __shfl_xor(ln, sh), om = __shfl_xor(lm, sh), oq = __shfl_xor(lq, sh);
                // the lower lane of each pair is taken as "a", so both lanes form the same sums
                if (lane & sh) {
                    double n2 = on, m2 = om, q2 = oq;
                    merge(n2, m2, q2, ln, lm, lq);
                    ln = n2;
                    lm = m2;
                    lq = q2;
                } else {
                    merge(ln, lm, lq, on, om, oq);
                }
            }
            mean = lm;
            var = lq * inv_n;
        }
        if (lane == 0) {
            double sd = sqrt(var > 0.0 ? var : 0.0);
            c[j] = mean;
            s[j] = sd;
            keep[j] = sd > 1e-6 ? 1 : 0;
        }
    }
}

__global__ __launch_bounds__(1024) void k_count_rows(const uint8_t* __restrict__ mask, int64_t n_total,
                                                     int64_t* __restrict__ out) {
    __shared__ double buf[16];
    double cnt = 0.0;
    for (int64_t i = threadIdx.x; i < n_total; i += blockDim.x) cnt += mask ? (mask[i] ? 1.0 : 0.0) : 1.0;
    double t = block_sum(cnt, buf);
    if (threadIdx.x == 0) *out = (int64_t)t;
}

// y_mean, y~ and ||y~||^2 in one workgroup (two passes over y)
__global__ __launch_bounds__(1024) void k_center_y(const uint8_t* __restrict__ mask, int64_t n_total,
                                                   const double* __restrict__ y, double* __restrict__ yt,
                                                   double* __restrict__ r, DevScalars* __restrict__ sc) {
    __shared__ double buf[16];
    double sy = 0.0, cnt = 0.0;
    for (int64_t i = threadIdx.x; i < n_total; i += blockDim.x) {
        bool in = mask ? mask[i] != 0 : true;
        if (in) {
            sy += y[i];
            cnt += 1.0;
        }
    }
    double tot = block_sum(sy, buf);
    double n = block_sum(cnt, buf);
    double mean = n > 0.0 ? tot / n : 0.0;
    double ss = 0.0;
    for (int64_t i = threadIdx.x; i < n_total; i += blockDim.x) {
        bool in = mask ? mask[i] != 0 : true;
        double v = in ? y[i] - mean : 0.0;
        yt[i] = v;
        if (r) r[i] = v;
        ss = fma(v, v, ss);
    }
    double yy = block_sum(ss, buf);
    if (threadIdx.x == 0) {
        sc->y_mean = mean;
        sc->yy = yy;
        sc->n_rows = (int64_t)n;
    }
}

__global__ __launch_bounds__(1024) void k_sum_r(int64_t n_total, const double* __restrict__ r,
                                                DevScalars* __restrict__ sc, int want_rss) {
    __shared__ double buf[16];
    double a = 0.0, q = 0.0;
    for (int64_t i = threadIdx.x; i < n_total; i += blockDim.x) {
        a += r[i];
        q = fma(r[i], r[i], q);
    }
    double ta = block_sum(a, buf);
    double tq = block_sum(q, buf);
    if (threadIdx.x == 0) {
        sc->sum_r = ta;
        if (want_rss) sc->rss = tq;
    }
}

template <typename XT>
__global__ void k_std_column(const XT* __restrict__ xj, const uint8_t* __restrict__ mask, int64_t n_total,
                             double cj_dummy, const double* __restrict__ c, const double* __restrict__ s, int64_t j,
                             double* __restrict__ v) {
    (void)cj_dummy;
    const double cj = c[j], inv = 1.0 / s[j];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_total; i += (int64_t)gridDim.x * blockDim.x) {
        bool in = mask ? mask[i] != 0 : true;
        v[i] = in ? ((double)xj[i] - cj) * inv : 0.0;
    }
}

// ---- the scan: z_j = (x_j' r - c_j sum_r) / (n s_j) --------------------------------------------
template <typename XT, bool VEC, bool RLDS>
__global__ __launch_bounds__(512) void k_scan(const XT* __restrict__ X, int64_t ldx, int64_t n_total, ScanArgs a) {
    extern __shared__ double r_lds[];
    const int wpb = blockDim.x / WAVE;
    const int64_t len = a.len_dev ? *a.len_dev : a.len_host;
    if (a.len_out && blockIdx.x == 0 && threadIdx.x == 0) *a.len_out = len;
    const int64_t wid0 = (int64_t)blockIdx.x * wpb;
    if (wid0 >= len) return;  // whole block idle (uniform)
    const double* r = a.r;
    if constexpr (RLDS) {
        for (int64_t i = threadIdx.x; i < n_total; i += blockDim.x) r_lds[i] = a.r[i];
        __syncthreads();
        r = r_lds;
    }
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t nw = (int64_t)gridDim.x * wpb;
    const double sum_r = a.sc->sum_r;
    const double inv_n = 1.0 / (double)a.sc->n_rows;
    for (int64_t t = wid0 + threadIdx.x / WAVE; t < len; t += nw) {
        const int64_t j = a.cols ? (int64_t)a.cols[t] : t;
        const bool kept = a.keep == nullptr || a.keep[j] != 0;
        double dot = 0.0;
        if (kept) dot = wave_col_dot<XT, VEC, 8>(X + j * ldx, r, n_total);
        if (lane == 0) {
            double z = kept ? (dot - a.c[j] * sum_r) * inv_n / a.s[j] : 0.0;
            a.z[j] = z;
            if (a.check && kept && (a.in_s == nullptr || a.in_s[j]) && (a.excl == nullptr || a.excl[j] == 0) &&
                fabs(z) > (a.w ? a.lam * a.w[j] : a.lam)) {
                a.mark[j] = 1;
                atomicAdd(a.nviol, 1u);
            }
        }
    }
}

// ---- lambda_max: argmax |a_j| over kept j, ties to the smallest index -------------------------
__device__ __forceinline__ void better(double& bv, int64_t& bi, double v, int64_t i) {
    if (v > bv || (v == bv && i >= 0 && (bi < 0 || i < bi))) {
        bv = v;
        bi = i;
    }
}

__global__ __launch_bounds__(256) void k_argmax_part(const double* __restrict__ a, const uint8_t* __restrict__ keep,
                                                     int64_t p, double* __restrict__ pv, int64_t* __restrict__ pi) {
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    double bv = -1.0;
    int64_t bi = -1;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x)
        if (keep[j]) better(bv, bi, fabs(a[j]), j);
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            double v = sv[threadIdx.x];
            int64_t i = si[threadIdx.x];
            better(v, i, sv[threadIdx.x + w], si[threadIdx.x + w]);
            sv[threadIdx.x] = v;
            si[threadIdx.x] = i;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pv[blockIdx.x] = sv[0];
        pi[blockIdx.x] = si[0];
    }
}

__global__ __launch_bounds__(256) void k_argmax_final(const double* __restrict__ pv, const int64_t* __restrict__ pi,
                                                      int nparts, DevScalars* __restrict__ sc) {
    __shared__ double sv[256];
    __shared__ int64_t si[256];
    double bv = -1.0;
    int64_t bi = -1;
    for (int k = threadIdx.x; k < nparts; k += blockDim.x) better(bv, bi, pv[k], pi[k]);
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            double v = sv[threadIdx.x];
            int64_t i = si[threadIdx.x];
            better(v, i, sv[threadIdx.x + w], si[threadIdx.x + w]);
            sv[threadIdx.x] = v;
            si[threadIdx.x] = i;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sc->lmax = sv[0] < 0.0 ? 0.0 : sv[0];
        sc->jstar = si[0];
    }
}

// ---- screening ------------------------------------------------------------------------------------
__global__ void k_bedpp(int64_t p, const double* __restrict__ a, const double* __restrict__ b,
                        const uint8_t* __restrict__ keep, int bedpp, double lm, double sgn, double lam, double rhs,
                        uint8_t* __restrict__ safe) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x) {
        uint8_t out = keep[j];
        if (out && bedpp) {
            double lhs = fabs((lm + lam) * a[j] - (lm - lam) * sgn * lm * b[j]);
            if (lhs < rhs) out = 0;
        }
        safe[j] = out;
    }
}

__global__ void k_ssr(int64_t p, const uint8_t* __restrict__ safe, const uint8_t* __restrict__ active,
                      const double* __restrict__ beta, const double* __restrict__ zprev, int ssr, double thr,
                      const double* __restrict__ w, uint8_t* __restrict__ strong) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x) {
        uint8_t out = 0;
        if (safe[j]) {
            bool act = active ? active[j] != 0 : (beta ? beta[j] != 0.0 : false);
            out = (!ssr || act || (zprev && fabs(zprev[j]) >= (w ? thr * w[j] : thr))) ? 1 : 0;
        }
        strong[j] = out;
    }
}

__global__ void k_enet_lmax_terms(const double* __restrict__ a, const double* __restrict__ w, double alpha, int64_t p,
                                  double* __restrict__ out) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x)
        out[j] = fabs(a[j]) / (alpha * (w ? w[j] : 1.0));
}

// ---- ordered compaction of a byte mask -------------------------------------------------------------
constexpr int CMP_THREADS = 256;
constexpr int CMP_ITEMS = 16;
constexpr int CMP_TILE = CMP_THREADS * CMP_ITEMS;

__global__ __launch_bounds__(CMP_THREADS) void k_cmp_count(const uint8_t* __restrict__ mask, int64_t p,
                                                           int32_t* __restrict__ counts) {
    __shared__ int32_t buf[CMP_THREADS / WAVE];
    const int64_t base = (int64_t)blockIdx.x * CMP_TILE + (int64_t)threadIdx.x * CMP_ITEMS;
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < CMP_ITEMS; ++k)
        if (base + k < p && mask[base + k]) ++cnt;
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) buf[threadIdx.x / WAVE] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < CMP_THREADS / WAVE; ++w) t += buf[w];
        counts[blockIdx.x] = t;
    }
}

// exclusive scan of nb block counts in one workgroup (sequential chunks of blockDim)
__global__ __launch_bounds__(1024) void k_cmp_scan(int32_t* __restrict__ counts, int64_t nb,
                                                   int64_t* __restrict__ total) {
    __shared__ int64_t sh[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nb; b0 += blockDim.x) {
        int64_t k = b0 + threadIdx.x;
        int64_t v = k < nb ? counts[k] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < (int)blockDim.x; off <<= 1) {
            int64_t add = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        int64_t incl = sh[threadIdx.x];
        if (k < nb) counts[k] = (int32_t)(carry + incl - v);
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry += incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ __launch_bounds__(CMP_THREADS) void k_cmp_write(const uint8_t* __restrict__ mask, int64_t p,
                                                           const int32_t* __restrict__ offsets,
                                                           int32_t* __restrict__ out) {
    __shared__ int32_t sh[CMP_THREADS];
    const int64_t base = (int64_t)blockIdx.x * CMP_TILE + (int64_t)threadIdx.x * CMP_ITEMS;
    uint8_t f[CMP_ITEMS];
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < CMP_ITEMS; ++k) {
        f[k] = (base + k < p) ? mask[base + k] : 0;
        cnt += f[k] ? 1 : 0;
    }
    sh[threadIdx.x] = cnt;
    __syncthreads();
    for (int off = 1; off < CMP_THREADS; off <<= 1) {
        int add = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    int pos = offsets[blockIdx.x] + sh[threadIdx.x] - cnt;
#pragma unroll
    for (int k = 0; k < CMP_ITEMS; ++k)
        if (f[k]) out[pos++] = (int32_t)(base + k);
}

// ---- cyclic coordinate descent: one persistent workgroup --------------------------------------------
//
// Thread t owns rows t + 1024*m (m < R) and keeps r there in registers.  The
// next D columns of the set are prefetched into a register ring while the
// current coordinate is reduced.  Coefficients of the set live in LDS, in
// windows of CD_WIN positions.
constexpr int CD_THREADS = 1024;
constexpr int CD_WAVES = CD_THREADS / WAVE;
constexpr int CD_WIN = 8192;

// Sum of the CD_WAVES partials in red[], the same value and order in every wave:
// lane k < CD_WAVES loads partial k, then a fixed butterfly over those lanes.
__device__ __forceinline__ double cd_total(const double* red, int lane) {
    double v = lane < CD_WAVES ? red[lane] : 0.0;
#pragma unroll
    for (int off = CD_WAVES / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return __shfl(v, 0, WAVE);
}

template <typename XT, int R, int D, bool MASK>
__global__ __launch_bounds__(CD_THREADS) void k_cd(const XT* __restrict__ X, int64_t ldx, int64_t n_total,
                                                   const uint8_t* __restrict__ mask, CdArgs a) {
    __shared__ double red[2][CD_WAVES];
    __shared__ double bwin[CD_WIN];
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
    const int64_t m = a.len_dev ? *a.len_dev : a.len_host;
    const double inv_n = 1.0 / (double)a.sc->n_rows;
    const double lam = a.lam;

    double rr[R];
    uint32_t mbits = 0;  // bit q: row tid + 1024 q is in the fit
#pragma unroll
    for (int q = 0; q < R; ++q) {
        int64_t i = tid + (int64_t)CD_THREADS * q;
        rr[q] = i < n_total ? a.r[i] : 0.0;
        if (i < n_total && (!MASK || mask[i])) mbits |= 1u << q;
    }

    int sweeps = 0, status = 0;
    if (m > 0) {
        // Register ring with the next D coordinates: column values, center, 1/scale.
        double xr[D][R];
        double cr[D], sr[D], wr[D];
        int64_t pf = 0;  // set position of the next coordinate to prefetch
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int j = a.set[pf];
            pf = (pf + 1 == m) ? 0 : pf + 1;
            cr[d] = a.c[j];
            sr[d] = 1.0 / a.s[j];
            wr[d] = a.w ? a.w[j] : 1.0;
            const __amdgpu_buffer_rsrc_t rs = column_rsrc(X + (int64_t)j * ldx, n_total * (int64_t)sizeof(XT));
#pragma unroll
            for (int q = 0; q < R; ++q)
                xr[d][q] = buf_x<XT>(rs, (tid + CD_THREADS * q) * (int)sizeof(XT));
        }

        // Coefficients of the current window of set positions [w0, w0 + wlen) live in LDS.
        // Thread 0 writes an update one step late (after the next barrier) so that no wave
        // can read a slot while it changes; the same step's value is forwarded in registers.
        int64_t w0 = 0;
        int64_t wlen = m < CD_WIN ? m : CD_WIN;
        for (int64_t k = tid; k < wlen; k += CD_THREADS) bwin[k] = a.beta[a.set[k]];
        __syncthreads();

        int64_t e = 0;  // set position of the current coordinate
        double maxd = 0.0;
        int par = 0;
        bool pend = false;
        int64_t pend_pos = 0;
        double pend_val = 0.0;
        bool done = false;
        while (!done) {
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const double cj = cr[d], isj = sr[d];
                double part = 0.0;
#pragma unroll
                for (int q = 0; q < R; ++q) part = fma(xr[d][q] - cj, rr[q], part);
                part = wave_sum(part);
                if (lane == 0) red[par][wv] = part;
                __syncthreads();
                const double dot = uniform(cd_total(red[par], lane));
                par ^= 1;
                const int64_t pos = e - w0;
                double bj = uniform(bwin[pos]);
                if (pend) {
                    if (pend_pos == pos) bj = pend_val;
                    if (tid == 0) bwin[pend_pos] = pend_val;
                }
                // elastic-net step S(u, lam alpha w) / (1 + lam (1 - alpha) w); the lasso step when alpha = 1, w = 1
                const double bnew = soft_threshold(dot * isj * inv_n + bj, lam * a.alpha * wr[d]) /
                                    (1.0 + lam * (1.0 - a.alpha) * wr[d]);
                const double delta = bnew - bj;
                pend = delta != 0.0;
                if (pend) {
                    pend_pos = pos;
                    pend_val = bnew;
                    const double f = delta * isj;
#pragma unroll
                    for (int q = 0; q < R; ++q)
                        if ((mbits >> q) & 1u) rr[q] = fma(-f, xr[d][q] - cj, rr[q]);
                }
                maxd = fmax(maxd, fabs(delta));
                // refill this slot with the coordinate D steps ahead
                {
                    const int j = a.set[pf];
                    pf = (pf + 1 == m) ? 0 : pf + 1;
                    cr[d] = a.c[j];
                    sr[d] = 1.0 / a.s[j];
                    wr[d] = a.w ? a.w[j] : 1.0;
                    const __amdgpu_buffer_rsrc_t rs =
                        column_rsrc(X + (int64_t)j * ldx, n_total * (int64_t)sizeof(XT));
#pragma unroll
                    for (int q = 0; q < R; ++q)
                        xr[d][q] = buf_x<XT>(rs, (tid + CD_THREADS * q) * (int)sizeof(XT));
                }
                ++e;
                const bool wrap = (e == m);
                if (wrap) {
                    ++sweeps;
                    if (maxd < a.tol) {
                        done = true;
                    } else if (sweeps >= a.max_sweeps) {
                        status = 1;
                        done = true;
                    }
                    maxd = 0.0;
                }
                if (!done && m > CD_WIN && (wrap || e == w0 + CD_WIN)) {
                    // move the coefficient window
                    if (tid == 0 && pend) bwin[pend_pos] = pend_val;
                    pend = false;
                    __syncthreads();
                    for (int64_t k = tid; k < wlen; k += CD_THREADS) a.beta[a.set[w0 + k]] = bwin[k];
                    __syncthreads();
                    if (wrap) e = 0;
                    w0 = e;
                    wlen = (m - w0) < CD_WIN ? (m - w0) : CD_WIN;
                    for (int64_t k = tid; k < wlen; k += CD_THREADS) bwin[k] = a.beta[a.set[w0 + k]];
                    __syncthreads();
                } else if (wrap) {
                    e = 0;
                }
                if (done) break;
            }
        }
        if (tid == 0 && pend) bwin[pend_pos] = pend_val;
        __syncthreads();
        for (int64_t k = tid; k < wlen; k += CD_THREADS) a.beta[a.set[w0 + k]] = bwin[k];
    } else {
        sweeps = 1;
    }

    // write back r; sum and sum of squares for the following scan and the record
    double sr_ = 0.0, sq = 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        int64_t i = tid + (int64_t)CD_THREADS * q;
        if (i < n_total) a.r[i] = rr[q];
        sr_ += rr[q];
        sq = fma(rr[q], rr[q], sq);
    }
    __syncthreads();
    double tsum = block_sum(sr_, &red[0][0]);
    double tsq = block_sum(sq, &red[0][0]);
    if (tid == 0) {
        a.sc->sum_r = tsum;
        a.sc->rss = tsq;
        a.sc->round.sweeps = sweeps;
        a.sc->round.status = status;
        a.sc->round.cd_len = (int32_t)m;
    }
}

// ---- per-lambda record --------------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_record(const int32_t* __restrict__ set, const int64_t* __restrict__ len_dev,
                                                 const int64_t* __restrict__ len_safe,
                                                 const int64_t* __restrict__ len_scan,
                                                 const double* __restrict__ beta, const double* __restrict__ c,
                                                 const double* __restrict__ s, const DevScalars* __restrict__ sc,
                                                 double lam, LamStats* __restrict__ out, double alpha,
                                                 const double* __restrict__ w) {
    __shared__ double buf[16];
    const int64_t m = set ? *len_dev : 0;
    const bool enet = alpha < 1.0 || w != nullptr;
    double l1 = 0.0, cb = 0.0, na = 0.0, pen = 0.0;
    for (int64_t t = threadIdx.x; t < m; t += blockDim.x) {
        const int j = set[t];
        const double b = beta[j];
        if (b != 0.0) {
            l1 += fabs(b);
            cb += c[j] * b / s[j];
            na += 1.0;
            if (enet) pen += (w ? w[j] : 1.0) * (alpha * fabs(b) + 0.5 * (1.0 - alpha) * b * b);
        }
    }
    double tl1 = block_sum(l1, buf);
    double tcb = block_sum(cb, buf);
    double tna = block_sum(na, buf);
    double tpen = enet ? block_sum(pen, buf) : 0.0;
    if (threadIdx.x == 0) {
        const double rss = sc->rss;
        out->rss = rss;
        out->l1 = tl1;
        out->n_active = (int64_t)tna;
        out->intercept = sc->y_mean - tcb;
        out->obj = rss / (2.0 * (double)sc->n_rows) + lam * (enet ? tpen : tl1);
        out->n_strong = m;
        out->n_safe = len_safe ? *len_safe : 0;
        out->n_scan = len_scan ? *len_scan : 0;
    }
}

// flag[set[e]] = 1 where beta[set[e]] != 0 (e < *len_dev); flag is cleared beforehand
__global__ void k_mark_nonzero(const int32_t* __restrict__ set, const int64_t* __restrict__ len_dev,
                               const double* __restrict__ beta, uint8_t* __restrict__ flag) {
    const int64_t m = *len_dev;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = set[e];
        if (beta[j] != 0.0) flag[j] = 1;
    }
}

// the totals of a solve made of several: sweeps, status and the set size, where the check round reads them
__global__ void k_set_round(DevScalars* __restrict__ sc, int32_t sweeps, int32_t status, int32_t cd_len) {
    sc->round.sweeps = sweeps;
    sc->round.status = status;
    sc->round.cd_len = cd_len;
}

__global__ void k_fill_u8(uint8_t* p, uint8_t v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_f64(double* p, double v, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_or_u8(uint8_t* dst, const uint8_t* src, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = (dst[i] || src[i]) ? 1 : 0;
}

int elem_size(int xtype) { return xtype == 0 ? 8 : (xtype == 1 ? 4 : 1); }

int grid_for(int64_t work, int per_block, int max_blocks) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > max_blocks) g = max_blocks;
    return (int)g;
}

}  // namespace

int device_cu_count() {
    static int cached = 0;
    if (!cached) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cached = prop.multiProcessorCount;
        if (cached <= 0) cached = 256;
    }
    return cached;
}

// dynamic LDS one workgroup may take on this device (64 KB assumed when the query fails)
int64_t device_lds_per_block() {
    static int64_t cached = 0;
    if (!cached) {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess) dev = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
            cached = v;
        else
            cached = 64 * 1024;
    }
    return cached;
}

hipError_t launch_colstats(const Mat& m, double* c, double* s, uint8_t* keep, int64_t n_rows, hipStream_t st) {
    const int g = grid_for(m.p, 4, device_cu_count() * 16);
    const bool mk = m.mask != nullptr;
    // int8 codes read as 16-byte words: columns (and the row mask) 16-byte aligned, and few enough rows that a
    // lane's int32 sum of squares cannot overflow
    // FP64 / FP32 X: whole 16-byte words when every column starts 16-byte aligned (the sums are the same either way)
    const int64_t esz = m.xtype == 0 ? 8 : (m.xtype == 1 ? 4 : 1);
    // (with a mask the last word of it read must lie inside its n_total bytes)
    const bool vec = m.xtype == 2 ? ((uintptr_t)m.X % 16 == 0 && m.ldx % 16 == 0 && (uintptr_t)m.mask % 16 == 0 &&
                                     (!mk || m.n_total % 16 == 0) && m.n_total <= (int64_t(1) << 22))
                                  : ((uintptr_t)m.X % 16 == 0 && (m.ldx * esz) % 16 == 0 &&
                                     (uintptr_t)m.mask % (16 / esz) == 0);
    switch (m.xtype) {
        case 0:
            if (mk) k_colstats<double, true><<<g, 256, 0, st>>>((const double*)m.X, m.ldx, m.n_total, m.p, m.mask, n_rows, c, s, keep, vec);
            else k_colstats<double, false><<<g, 256, 0, st>>>((const double*)m.X, m.ldx, m.n_total, m.p, m.mask, n_rows, c, s, keep, vec);
            break;
        case 1:
            if (mk) k_colstats<float, true><<<g, 256, 0, st>>>((const float*)m.X, m.ldx, m.n_total, m.p, m.mask, n_rows, c, s, keep, vec);
            else k_colstats<float, false><<<g, 256, 0, st>>>((const float*)m.X, m.ldx, m.n_total, m.p, m.mask, n_rows, c, s, keep, vec);
            break;
        default:
            if (mk) k_colstats<int8_t, true><<<g, 256, 0, st>>>((const int8_t*)m.X, m.ldx, m.n_total, m.p, m.mask, n_rows, c, s, keep, vec);
            else k_colstats<int8_t, false><<<g, 256, 0, st>>>((const int8_t*)m.X, m.ldx, m.n_total, m.p, m.mask, n_rows, c, s, keep, vec);
    }
    return hipGetLastError();
}

hipError_t launch_count_rows(const Mat& m, int64_t* out_dev, hipStream_t st) {
    k_count_rows<<<1, 1024, 0, st>>>(m.mask, m.n_total, out_dev);
    return hipGetLastError();
}

hipError_t launch_center_y(const Mat& m, const double* y, double* ytilde, double* r, DevScalars* sc, hipStream_t st) {
    k_center_y<<<1, 1024, 0, st>>>(m.mask, m.n_total, y, ytilde, r, sc);
    return hipGetLastError();
}

hipError_t launch_sum_r(const Mat& m, const double* r, DevScalars* sc, bool want_rss, hipStream_t st) {
    k_sum_r<<<1, 1024, 0, st>>>(m.n_total, r, sc, want_rss ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_std_column(const Mat& m, int64_t j, const double* c, const double* s, double* v, hipStream_t st) {
    const int g = grid_for(m.n_total, 256, 1024);
    const int64_t off = j * m.ldx;
    switch (m.xtype) {
        case 0: k_std_column<double><<<g, 256, 0, st>>>((const double*)m.X + off, m.mask, m.n_total, 0.0, c, s, j, v); break;
        case 1: k_std_column<float><<<g, 256, 0, st>>>((const float*)m.X + off, m.mask, m.n_total, 0.0, c, s, j, v); break;
        default: k_std_column<int8_t><<<g, 256, 0, st>>>((const int8_t*)m.X + off, m.mask, m.n_total, 0.0, c, s, j, v);
    }
    return hipGetLastError();
}

template <typename XT>
static hipError_t scan_typed(const Mat& m, const ScanArgs& a, hipStream_t st) {
    const int threads = 512;
    const int wpb = threads / WAVE;
    // r in LDS while two workgroups of 8 waves still fit a CU (160 KB of LDS per CU on gfx950)
    const size_t lds = (size_t)m.n_total * sizeof(double);
    const bool rlds = lds <= 80 * 1024 && (int64_t)lds <= device_lds_per_block();
    const bool vec = (((uintptr_t)m.X) % 16 == 0) && ((m.ldx * (int64_t)sizeof(XT)) % 16 == 0);
    const int64_t work = a.len_dev ? m.p : a.len_host;  // upper bound when the length lives on the device
    const int per_cu = rlds ? (lds <= 40 * 1024 ? 4 : (lds <= 53 * 1024 ? 3 : 2)) : 4;
    const int g = grid_for(work, wpb, device_cu_count() * per_cu);
    const XT* X = (const XT*)m.X;
    if (rlds) {
        if (vec) k_scan<XT, true, true><<<g, threads, lds, st>>>(X, m.ldx, m.n_total, a);
        else k_scan<XT, false, true><<<g, threads, lds, st>>>(X, m.ldx, m.n_total, a);
    } else {
        if (vec) k_scan<XT, true, false><<<g, threads, 0, st>>>(X, m.ldx, m.n_total, a);
        else k_scan<XT, false, false><<<g, threads, 0, st>>>(X, m.ldx, m.n_total, a);
    }
    return hipGetLastError();
}

hipError_t launch_scan(const Mat& m, const ScanArgs& a, hipStream_t st) {
    switch (m.xtype) {
        case 0: return scan_typed<double>(m, a, st);
        case 1: return scan_typed<float>(m, a, st);
        default: return scan_typed<int8_t>(m, a, st);
    }
}

hipError_t launch_argmax_abs(const double* a, const uint8_t* keep, int64_t p, double* part_v, int64_t* part_i,
                             DevScalars* sc, hipStream_t st) {
    const int g = grid_for(p, 256, 256);
    k_argmax_part<<<g, 256, 0, st>>>(a, keep, p, part_v, part_i);
    k_argmax_final<<<1, 256, 0, st>>>(part_v, part_i, g, sc);
    return hipGetLastError();
}

hipError_t launch_bedpp(int64_t p, const double* a, const double* b, const uint8_t* keep, bool bedpp, double lmax,
                        double sgn, double lam, double rhs, uint8_t* safe, hipStream_t st) {
    const int g = grid_for(p, 256, device_cu_count() * 8);
    k_bedpp<<<g, 256, 0, st>>>(p, a, b, keep, bedpp ? 1 : 0, lmax, sgn, lam, rhs, safe);
    return hipGetLastError();
}

hipError_t launch_ssr(int64_t p, const uint8_t* safe, const uint8_t* active, const double* beta, const double* zprev,
                      bool ssr, double thr, uint8_t* strong, hipStream_t st, const double* w) {
    const int g = grid_for(p, 256, device_cu_count() * 8);
    k_ssr<<<g, 256, 0, st>>>(p, safe, active, beta, zprev, ssr ? 1 : 0, thr, w, strong);
    return hipGetLastError();
}

hipError_t launch_enet_lmax_terms(const double* a, const double* w, double alpha, int64_t p, double* out,
                                  hipStream_t st) {
    k_enet_lmax_terms<<<grid_for(p, 256, 4096), 256, 0, st>>>(a, w, alpha, p, out);
    return hipGetLastError();
}

size_t compact_scratch_bytes(int64_t p) {
    int64_t nb = (p + CMP_TILE - 1) / CMP_TILE;
    if (nb < 1) nb = 1;
    return (size_t)nb * sizeof(int32_t);
}

hipError_t launch_compact(const uint8_t* mask, int64_t p, int32_t* out, int64_t* len_dev, void* scratch,
                          hipStream_t st) {
    int64_t nb = (p + CMP_TILE - 1) / CMP_TILE;
    if (nb < 1) nb = 1;
    int32_t* counts = (int32_t*)scratch;
    k_cmp_count<<<(unsigned)nb, CMP_THREADS, 0, st>>>(mask, p, counts);
    k_cmp_scan<<<1, 1024, 0, st>>>(counts, nb, len_dev);
    k_cmp_write<<<(unsigned)nb, CMP_THREADS, 0, st>>>(mask, p, counts, out);
    return hipGetLastError();
}

bool cd_supported(int64_t n_total) { return n_total >= 1 && n_total <= 16 * CD_THREADS; }

template <typename XT, bool MASK>
static hipError_t cd_typed(const Mat& m, const CdArgs& a, hipStream_t st) {
    const XT* X = (const XT*)m.X;
    const int64_t n = m.n_total;
    if (n <= 2 * CD_THREADS) k_cd<XT, 2, 8, MASK><<<1, CD_THREADS, 0, st>>>(X, m.ldx, n, m.mask, a);
    else if (n <= 4 * CD_THREADS) k_cd<XT, 4, 4, MASK><<<1, CD_THREADS, 0, st>>>(X, m.ldx, n, m.mask, a);
    else if (n <= 5 * CD_THREADS) k_cd<XT, 5, 4, MASK><<<1, CD_THREADS, 0, st>>>(X, m.ldx, n, m.mask, a);
    else if (n <= 8 * CD_THREADS) k_cd<XT, 8, 2, MASK><<<1, CD_THREADS, 0, st>>>(X, m.ldx, n, m.mask, a);
    else if (n <= 10 * CD_THREADS) k_cd<XT, 10, 2, MASK><<<1, CD_THREADS, 0, st>>>(X, m.ldx, n, m.mask, a);
    else k_cd<XT, 16, 1, MASK><<<1, CD_THREADS, 0, st>>>(X, m.ldx, n, m.mask, a);
    return hipGetLastError();
}

hipError_t launch_cd(const Mat& m, const CdArgs& a, hipStream_t st) {
    const bool mk = m.mask != nullptr;
    switch (m.xtype) {
        case 0: return mk ? cd_typed<double, true>(m, a, st) : cd_typed<double, false>(m, a, st);
        case 1: return mk ? cd_typed<float, true>(m, a, st) : cd_typed<float, false>(m, a, st);
        default: return mk ? cd_typed<int8_t, true>(m, a, st) : cd_typed<int8_t, false>(m, a, st);
    }
}

hipError_t launch_record(const int32_t* set, const int64_t* len_dev, const int64_t* len_safe, const int64_t* len_scan,
                         const double* beta, const double* c, const double* s, const DevScalars* sc, double lam,
                         LamStats* out, hipStream_t st, double alpha, const double* w) {
    k_record<<<1, 1024, 0, st>>>(set, len_dev, len_safe, len_scan, beta, c, s, sc, lam, out, alpha, w);
    return hipGetLastError();
}

hipError_t launch_mark_nonzero(const int32_t* set, const int64_t* len_dev, int64_t m_max, const double* beta,
                               uint8_t* flag, hipStream_t st) {
    k_mark_nonzero<<<grid_for(m_max > 0 ? m_max : 1, 256, 1024), 256, 0, st>>>(set, len_dev, beta, flag);
    return hipGetLastError();
}

hipError_t launch_set_round(DevScalars* sc, int32_t sweeps, int32_t status, int32_t cd_len, hipStream_t st) {
    k_set_round<<<1, 1, 0, st>>>(sc, sweeps, status, cd_len);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t st) {
    k_fill_u8<<<grid_for(n, 256, 4096), 256, 0, st>>>(p, v, n);
    return hipGetLastError();
}
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t st) {
    k_fill_f64<<<grid_for(n, 256, 4096), 256, 0, st>>>(p, v, n);
    return hipGetLastError();
}
hipError_t launch_or_u8(uint8_t* dst, const uint8_t* src, int64_t n, hipStream_t st) {
    k_or_u8<<<grid_for(n, 256, 4096), 256, 0, st>>>(dst, src, n);
    return hipGetLastError();
}

}  // namespace blk
