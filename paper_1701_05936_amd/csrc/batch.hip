// Batched form: many lasso problems (responses and cross-validation row subsets)
// over one design matrix, advanced through their lambda grids in lockstep.
//
// Everything that reads X does so once for all problems: a right-hand side of
// up to BNP = 64 columns (problem b in column b) is contracted against the
// columns of X on FP64 matrix cores (v_mfma_f64_16x16x4f64).  The masked
// column sums for per-problem standardization, the type (2) and type (1)
// products of lambda_max and BEDPP, and every post-convergence scan use it.
// The rest (screening, compaction, Gram pools, coordinate descent, residual
// updates) runs as batched kernels with the problem in the grid.
//
// Layouts: right-hand sides and residuals are row-major n_pad x 64
// (R[i*64 + b]); per-problem vectors over features are problem-major
// (v[b*p + j]).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "chain.h"
#include "internal.h"

namespace blk {

namespace {

constexpr int WAVE = 64;

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
    return v;
}

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

int grid_for(int64_t work, int per_block, int max_blocks) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > max_blocks) g = max_blocks;
    return (int)g;
}

// ---- the shared contraction: OUT = X_cols' B on FP64 matrix cores ----------------------------------------
// Workgroup tile: 32 WAVES columns x 64 problems; wavefront w covers columns 32w .. 32w+31 (two 16-row MFMA
// tiles) against four 16-problem tiles.  Rows go in batches of BS_K = 64: lane (m, kq) holds 16 consecutive
// rows of its column (rows i0 + 16kq .. +15) and feeds row i0 + 16kq + st at MFMA step st; the same rows of B
// come from LDS (double buffered, padded rows against bank conflicts).  The next batch's X values are loaded
// into registers while the current batch is on the matrix cores when PF is set (more registers, fewer waves
// in flight); X values are converted to FP64 only as the matrix cores take them.  WAVES (2, 4 or 8) and PF are picked per shape by the autotuner: wider workgroups stage each
// B batch for more columns, narrower ones give more workgroups.
constexpr int BS_K = 64;
constexpr int BS_LD = BNP + 2;   // LDS row stride of the staged B rows (doubles)

// Work split of a column list over the G workgroups of a launch (as many as the device holds at once), for
// the one-pass scans (k_bscan modes 0-2 and k_bscan_bf16): the list is T = ceil(len / TW) tiles of TW columns,
// each C chunks of 64 rows.  Every workgroup first runs Tf = floor(T / G) whole tiles, tile i + k G for
// workgroup i, all of them moving through the rows in step so that each chunk of the right-hand sides is read
// from L2 by every workgroup at about the same time.  The T - Tf G tiles left over are cut by rows: their
// (tile, chunk) units, tile-major, go out in equal contiguous ranges of at least BF_QMIN chunks, one per
// workgroup, so that every workgroup finishes at about the same time however T falls against G.  A tile run
// whole by one workgroup is written out directly; the rows of a cut tile that one workgroup ran are stored as
// raw FP64 sums in its part slot (slot 0 for the first leftover tile the workgroup touches, slot 1 for the
// second, layout [slot][problem][column of the tile]), and a join kernel adds the slots of each cut tile in
// row order.
constexpr int SPLIT_CHUNK = 64;  // rows per chunk of the split (the batch of both scans)
constexpr int BF_QMIN = 8;       // fewest chunks in a range of leftover units (bounds the rows a tile is cut into)
struct BfSplit {
    int64_t T, C, Tf, Trem, q;   // tiles, chunks per tile, whole tiles per workgroup, leftover tiles, units per range
};
template <int TW>
__device__ __forceinline__ BfSplit tile_split(int64_t len, int64_t n_pad, int64_t G) {
    BfSplit s;
    s.T = (len + TW - 1) / TW;
    s.C = n_pad / SPLIT_CHUNK;
    s.Tf = s.T / G;
    s.Trem = s.T - s.Tf * G;
    s.q = max((s.Trem * s.C + G - 1) / G, (int64_t)BF_QMIN);
    return s;
}
// the workgroup's jobs: its Tf whole tiles, then the one or two leftover tiles its range of units touches; job
// k runs rows [r0, r1) of tile tt and stores them in part slot `slot` unless `whole`
struct TileJob {
    int64_t tt, r0, r1;
    int slot;
    bool whole;
};
struct TileJobs {
    BfSplit sp;
    int64_t G, wg, u0, u1, head, n;
};
template <int TW>
__device__ __forceinline__ TileJobs tile_jobs(int64_t len, int64_t n_pad, int64_t G, int64_t wg) {
    TileJobs J;
    J.sp = tile_split<TW>(len, n_pad, G);
    J.G = G;
    J.wg = wg;
    J.u0 = wg * J.sp.q;
    J.u1 = min(J.u0 + J.sp.q, J.sp.Trem * J.sp.C);
    J.head = J.sp.C > 0 ? J.u0 / J.sp.C : 0;
    J.n = J.sp.Tf + (J.u0 < J.u1 ? (J.u1 - 1) / J.sp.C - J.head + 1 : 0);
    return J;
}
__device__ __forceinline__ TileJob tile_job(const TileJobs& J, int64_t k) {
    TileJob t;
    const int64_t C = J.sp.C;
    if (k < J.sp.Tf) {
        t.tt = J.wg + k * J.G;
        t.r0 = 0;
        t.r1 = C * SPLIT_CHUNK;
        t.slot = 0;
        t.whole = true;
    } else {
        const int64_t tr = J.head + (k - J.sp.Tf);
        const int64_t c0 = max(J.u0 - tr * C, (int64_t)0), c1 = min(J.u1 - tr * C, C);
        t.tt = J.sp.Tf * J.G + tr;
        t.r0 = c0 * SPLIT_CHUNK;
        t.r1 = c1 * SPLIT_CHUNK;
        t.slot = tr == J.head ? 0 : 1;
        t.whole = c0 == 0 && c1 == C;
    }
    return t;
}
// the leftover tile tr of a launch with G workgroups is cut if more than one workgroup ran rows of it; if so,
// its stored rows lie in slots of workgroups i0 .. i1
__device__ __forceinline__ bool tile_cut(const BfSplit& sp, int64_t tr, int64_t& i0, int64_t& i1) {
    i0 = tr * sp.C / sp.q;
    i1 = ((tr + 1) * sp.C - 1) / sp.q;
    return i0 != i1;
}
__device__ __forceinline__ int tile_slot(const BfSplit& sp, int64_t i, int64_t tr) {
    return i * sp.q / sp.C == tr ? 0 : 1;
}

// mode 0: raw dot products; mode 1: squared X (masked second moments); mode 2: standardized correlations;
// modes 0-2 split the list over the launch's workgroups (tile_jobs; part: the rows of cut tiles, added by
// k_bscan_join); mode 3: raw dot products of the rows [rc * blockIdx.y, rc * (blockIdx.y + 1)) of tile
// blockIdx.x only, written to out[(blockIdx.y * len + t) * BNP + b] (split over rows for short column lists;
// k_bscan_reduce adds them)
template <typename XT, int MODE, int WAVES, bool PF>
__global__ __launch_bounds__(64 * WAVES) __attribute__((amdgpu_waves_per_eu(WAVES >= 4 ? 2 : 1))) void k_bscan(const XT* __restrict__ X, int64_t ldx, int64_t n_total,
                                                      int64_t n_pad, const int32_t* __restrict__ cols,
                                                      const int64_t* __restrict__ len_dev, int64_t len_host,
                                                      const double* __restrict__ B, int nprob, int64_t p,
                                                      BatchScalars* __restrict__ bs, const double* __restrict__ c,
                                                      const double* __restrict__ s, const uint8_t* __restrict__ keep,
                                                      double* __restrict__ part, double* __restrict__ out, int64_t rc) {
    constexpr int NT = 64 * WAVES, TF = 32 * WAVES;
    static_assert(BS_K == SPLIT_CHUNK, "the split's chunks are the scan's row batches");
    __shared__ double Bl[2][BS_K * BS_LD];
    const int64_t len = len_dev ? *len_dev : len_host;
    TileJobs J{};
    int64_t njobs;
    if constexpr (MODE == 3) {
        njobs = (int64_t)blockIdx.x * TF < len ? 1 : 0;
    } else {
        J = tile_jobs<TF>(len, n_pad, gridDim.x, blockIdx.x);
        njobs = J.n;
    }
    if (njobs == 0) return;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), w = tid / WAVE;
    const int m = lane & 15, kq = lane >> 4;
    // a batch of B (64 rows x 64 problems) is staged in two halves: its loads are issued before the current
    // batch goes to the matrix cores and its LDS stores after, so the wave does not wait on them in between
    constexpr int SPT = BS_K * BNP / NT;   // B values per thread
    double sreg[SPT];
    auto stage_load = [&](int64_t i0) {
#pragma unroll
        for (int q = 0; q < SPT; ++q) sreg[q] = B[(i0 + (tid + q * NT) / BNP) * BNP + (tid + q * NT) % BNP];
    };
    auto stage_store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < SPT; ++q) Bl[buf][((tid + q * NT) / BNP) * BS_LD + (tid + q * NT) % BNP] = sreg[q];
    };
    for (int64_t job = 0; job < njobs; ++job) {
        int64_t tt, row0, row1;
        int slot = 0;
        bool whole;
        if constexpr (MODE == 3) {
            tt = blockIdx.x;
            row0 = rc * (int64_t)blockIdx.y;
            row1 = row0 + rc < n_pad ? row0 + rc : n_pad;
            whole = false;
        } else {
            const TileJob tj = tile_job(J, job);
            tt = tj.tt;
            row0 = tj.r0;
            row1 = tj.r1;
            slot = tj.slot;
            whole = tj.whole;
        }
        const int64_t f0 = tt * TF;
        // the two columns this lane feeds (tiles ft = 0, 1)
        const XT* xc[2];
        bool ok[2];
#pragma unroll
        for (int ft = 0; ft < 2; ++ft) {
            const int64_t t = f0 + 32 * w + 16 * ft + m;
            ok[ft] = t < len;
            const int64_t j = ok[ft] ? (cols ? (int64_t)cols[t] : t) : 0;
            xc[ft] = X + j * ldx;
        }
        f64x4 acc[2][4];
#pragma unroll
        for (int ft = 0; ft < 2; ++ft)
#pragma unroll
            for (int pt = 0; pt < 4; ++pt) acc[ft][pt] = (f64x4){0.0, 0.0, 0.0, 0.0};
        // raw X values of the lane's rows of one batch (zero past n_total or for an idle column), converted to
        // FP64 as the matrix cores take them; with PF the next batch's values load into xn meanwhile
        XT xr[2][16], xn[2][16];
        auto load = [&](XT (&dst)[2][16], int64_t i0) {
#pragma unroll
            for (int ft = 0; ft < 2; ++ft) {
                const int64_t r0 = i0 + 16 * kq;
                if (ok[ft] && r0 + 16 <= n_total) {
#pragma unroll
                    for (int q = 0; q < 16; ++q) dst[ft][q] = xc[ft][r0 + q];
                } else {
#pragma unroll
                    for (int q = 0; q < 16; ++q) dst[ft][q] = (ok[ft] && r0 + q < n_total) ? xc[ft][r0 + q] : (XT)0;
                }
            }
        };
        // buffer 0 was last read before the barrier that ended the previous job
        int buf = 0;
        if (PF) load(xr, row0);
        stage_load(row0);
        stage_store(0);
        __syncthreads();
        for (int64_t i0 = row0; i0 < row1; i0 += BS_K) {
            if (!PF) load(xr, i0);
            const bool more = i0 + BS_K < row1;
            if (more) {
                if (PF) load(xn, i0 + BS_K);
                stage_load(i0 + BS_K);
            }
            const double* Bb = Bl[buf];
#pragma unroll
            for (int st = 0; st < 16; ++st) {
                const int row = 16 * kq + st;
                double xa[2];
#pragma unroll
                for (int ft = 0; ft < 2; ++ft) {
                    const double v = (double)xr[ft][st];
                    xa[ft] = MODE == 1 ? v * v : v;
                }
#pragma unroll
                for (int pt = 0; pt < 4; ++pt) {
                    const double bv = Bb[row * BS_LD + 16 * pt + m];
#pragma unroll
                    for (int ft = 0; ft < 2; ++ft)
                        acc[ft][pt] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[ft], bv, acc[ft][pt], 0, 0, 0);
                }
            }
            if (more) stage_store(buf ^ 1);   // the other buffer was last read before the previous barrier
            __syncthreads();
            buf ^= 1;
            if (PF) {
#pragma unroll
                for (int ft = 0; ft < 2; ++ft)
#pragma unroll
                    for (int q = 0; q < 16; ++q) xr[ft][q] = xn[ft][q];
            }
        }
        // lane (m, kq), register q of tile (ft, pt) holds column 32w + 16ft + kq + 4q against problem 16pt + m
        double* pp = part + (J.wg * 2 + slot) * (int64_t)BNP * TF;
#pragma unroll
        for (int ft = 0; ft < 2; ++ft) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int ci = 32 * w + 16 * ft + kq + 4 * q;
                const int64_t t = f0 + ci;
                if (t >= len) continue;
                const int64_t j = cols ? (int64_t)cols[t] : t;
#pragma unroll
                for (int pt = 0; pt < 4; ++pt) {
                    const int b = 16 * pt + m;
                    if (b >= nprob) continue;
                    const double v = acc[ft][pt][q];
                    if (MODE == 3) {
                        out[((int64_t)blockIdx.y * len + t) * BNP + b] = v;
                    } else if (!whole) {
                        pp[(int64_t)b * TF + ci] = v;
                    } else if (MODE == 2) {
                        const int64_t bj = (int64_t)b * p + j;
                        const bool kept = keep == nullptr || keep[bj] != 0;
                        out[bj] = kept ? (v - c[bj] * bs[b].sum_r) / ((double)bs[b].n_rows * s[bj]) : 0.0;
                    } else {
                        out[(int64_t)b * p + j] = v;
                    }
                }
            }
        }
    }
}

// The cut leftover tiles of a k_bscan launch (modes 0-2) with G workgroups: one thread per (leftover tile,
// problem, column) adds the tile's stored rows in row order, then writes the mode's result.
template <int TF, int MODE>
__global__ __launch_bounds__(256) void k_bscan_join(const int64_t* __restrict__ len_dev, int64_t len_host,
                                                    int64_t n_pad, int64_t G, const int32_t* __restrict__ cols,
                                                    int nprob, int64_t p, const BatchScalars* __restrict__ bs,
                                                    const double* __restrict__ c, const double* __restrict__ s,
                                                    const uint8_t* __restrict__ keep, const double* __restrict__ part,
                                                    double* __restrict__ out) {
    const int64_t len = len_dev ? *len_dev : len_host;
    const BfSplit sp = tile_split<TF>(len, n_pad, G);
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tr = e / (TF * BNP);
    const int b = (int)(e / TF % BNP), ci = (int)(e % TF);
    if (tr >= sp.Trem || b >= nprob) return;
    const int64_t t = (sp.Tf * G + tr) * TF + ci;
    int64_t i0, i1;
    if (t >= len || !tile_cut(sp, tr, i0, i1)) return;
    double v = 0.0;
#pragma unroll 8
    for (int64_t i = i0; i <= i1; ++i) v += part[((i * 2 + tile_slot(sp, i, tr)) * BNP + b) * TF + ci];
    const int64_t j = cols ? (int64_t)cols[t] : t;
    const int64_t bj = (int64_t)b * p + j;
    if (MODE == 2) {
        const bool kept = keep == nullptr || keep[bj] != 0;
        out[bj] = kept ? (v - c[bj] * bs[b].sum_r) / ((double)bs[b].n_rows * s[bj]) : 0.0;
    } else {
        out[bj] = v;
    }
}

// ---- the shared contraction on BF16 matrix cores (f32 X) ----------------------------------------------
// The check scans of the batched form as Z = X_cols' R with both operands split into PC = 2 or 3 BF16
// pieces (round to nearest at every step):
//   x = x_1 + .. + x_PC + dx,  x_1 = bf16(x), x_k = bf16(x - x_1 - .. - x_k-1)  (the differences are exact in FP32),
//   r = r_1 + .. + r_PC + dr,  r_k = bf16((float)(r - r_1 - .. - r_k-1))      (the differences are exact in FP64),
// |dx| <= e^PC |x| and |dr| <= (e + 2u)^PC |r| with e = 2^-8, u = 2^-24.  The products x_a r_b with
// a + b <= PC + 1 are taken on v_mfma_f32_16x16x32_bf16 (PC = 3: six, PC = 2: three); the rest are dropped.
// x_1 r_1 sums in an FP32 accumulator for one 64-row chunk (two 32-row steps), then goes to FP64; the smaller
// products (at most 2^-7 (1 + 2^-6) |x| |r| together) share a second FP32 accumulator that goes to FP64
// every BF_PROMO chunks.  bscan_bf16_rel() bounds the difference from the FP64 scan; decisions within that
// band are re-taken on the FP64 scan of those columns.
// Tile: a wavefront owns 16 columns against the 64 problems (four 16-problem tiles); lane (m, g) feeds rows
// 8g .. 8g+7 of a 32-row step of column m (A) and of problem 16 nt + m (B).  The residual pieces of a
// 64-row chunk sit in LDS, [piece][problem][row] with a padded row stride, double buffered; the lane's X
// values of the next two chunks are in flight in three register buffers taken in turn (the chunk loop is
// unrolled three times so that no buffer is copied).
constexpr int BF_K = 64;          // rows per chunk (two 32-row matrix-core steps)
constexpr int BF_RS = BF_K + 16;  // LDS stride of a (piece, problem) row block, bf16 elements (160 bytes: the
                                  // matrix-core operand reads and the staging writes measured free of bank conflicts)
constexpr int BF_PROMO = 9;       // chunks between promotions of the second accumulator (a multiple of 3)

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x8 __attribute__((ext_vector_type(8)));
typedef int v4i32 __attribute__((ext_vector_type(4)));

// residual pieces of every problem, problem-major per piece: Rp[(c * BNP + b) * n_pad + i], c < PC
__global__ void k_b_r_pieces(const double* __restrict__ R, int64_t n_total, int64_t n_pad, int nprob, int pc,
                             __bf16* __restrict__ Rp) {
    const int64_t total = n_pad * BNP;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx % n_pad;
        const int b = (int)(idx / n_pad);
        double rem = (i < n_total && b < nprob) ? R[i * BNP + b] : 0.0;
        for (int c = 0; c < pc; ++c) {
            const __bf16 v = (__bf16)(float)rem;
            Rp[((int64_t)c * BNP + b) * n_pad + i] = v;
            rem -= (double)(float)v;
        }
    }
}

// z_j of problem b from its raw sum x_j' r_b (the implicit standardization of the column)
__device__ __forceinline__ void bf_store(double acc, int b, int64_t jq, int64_t p, const BatchScalars* bs,
                                         const double* c, const double* s, const uint8_t* keep, double* out) {
    const int64_t bj = (int64_t)b * p + jq;
    const bool kept = keep == nullptr || keep[bj] != 0;
    out[bj] = kept ? (acc - c[bj] * bs[b].sum_r) / ((double)bs[b].n_rows * s[bj]) : 0.0;
}

template <int WAVES, int PC>
__global__ __launch_bounds__(64 * WAVES, 8 / WAVES) void k_bscan_bf16(const float* __restrict__ X, int64_t ldx, int64_t n_total,
                                                           int64_t n_pad, const __bf16* __restrict__ Rp,
                                                           const int32_t* __restrict__ cols,
                                                           const int64_t* __restrict__ len_dev, int64_t len_host,
                                                           int nprob, int64_t p, const BatchScalars* __restrict__ bs,
                                                           const double* __restrict__ c, const double* __restrict__ s,
                                                           const uint8_t* __restrict__ keep, double* __restrict__ part,
                                                           double* __restrict__ out) {
    static_assert(PC == 2 || PC == 3, "two or three pieces");
    static_assert(BF_PROMO % 3 == 0, "the main loop promotes after whole groups of three chunks");
    constexpr int NT = 64 * WAVES, TW = 16 * WAVES;
    constexpr int PLANE = PC * BNP * BF_RS;
    __shared__ __bf16 Rl[2 * PLANE];
    const int64_t len = len_dev ? *len_dev : len_host;
    const int64_t G = gridDim.x, wg = blockIdx.x;
    const BfSplit sp = tile_split<16 * WAVES>(len, n_pad, G);
    const int64_t C = sp.C, F = n_total / BF_K;   // chunks; chunks wholly inside n_total
    // this workgroup's range of leftover units
    const int64_t u0 = wg * sp.q, u1 = min(u0 + sp.q, sp.Trem * C);
    if (sp.Tf == 0 && u0 >= u1) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid / 64;
    const int m = lane & 15, g = lane >> 4;
    const float* xc = X;   // the lane's column of the tile being run
    // staging of one chunk's pieces: PC x 64 problems x 64 rows in 16-byte blocks
    constexpr int SB = PC * BNP * (BF_K / 8);
    constexpr int SPT = (SB + NT - 1) / NT;
    v4i32 sreg[SPT];
    auto stage_load = [&](int64_t ck) {
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int blk = tid + q * NT;
            if (blk < SB) {
                const int cb = blk / (BF_K / 8), r8 = blk % (BF_K / 8);
                sreg[q] = *reinterpret_cast<const v4i32*>(Rp + (int64_t)cb * n_pad + ck * BF_K + 8 * r8);
            }
        }
    };
    auto stage_store = [&](__bf16* dst) {
#pragma unroll
        for (int q = 0; q < SPT; ++q) {
            const int blk = tid + q * NT;
            if (blk < SB) {
                const int cb = blk / (BF_K / 8), r8 = blk % (BF_K / 8);
                *reinterpret_cast<v4i32*>(dst + cb * BF_RS + 8 * r8) = sreg[q];
            }
        }
    };
    // the lane's 16 values of chunk ck: rows 64 ck + 32 ks + 8 g .. +7 for ks = 0, 1; load_fast for chunks
    // inside n_total, load_x zero past it
    auto load_fast = [&](float (&dst)[16], int64_t ck) {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const float4* src = reinterpret_cast<const float4*>(xc + ck * BF_K + 32 * ks + 8 * g);
            const float4 a = src[0], b = src[1];
            dst[8 * ks + 0] = a.x; dst[8 * ks + 1] = a.y; dst[8 * ks + 2] = a.z; dst[8 * ks + 3] = a.w;
            dst[8 * ks + 4] = b.x; dst[8 * ks + 5] = b.y; dst[8 * ks + 6] = b.z; dst[8 * ks + 7] = b.w;
        }
    };
    auto load_x = [&](float (&dst)[16], int64_t ck) {
        if ((ck + 1) * BF_K <= n_total) {
            load_fast(dst, ck);
        } else {
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int64_t i = ck * BF_K + 32 * ks + 8 * g + q;
                    dst[8 * ks + q] = i < n_total ? xc[i] : 0.f;
                }
        }
    };
    double acc64[4][4];
    f32x4 a2[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        a2[nt] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 4; ++q) acc64[nt][q] = 0.0;
    }
    int ch = 0;   // chunks done; the chunk being computed reads LDS buffer ch & 1
    // one chunk's matrix-core steps on the lane's values xr; x_1 r_1 goes to FP64 at the end
    auto compute = [&](const float (&xr)[16]) {
        const __bf16* Rb = Rl + (ch & 1) * PLANE;
        f32x4 a1[4];
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            f32x8 xv;
#pragma unroll
            for (int q = 0; q < 8; ++q) xv[q] = xr[8 * ks + q];
            bf16x8 xp[PC];
            xp[0] = __builtin_convertvector(xv, bf16x8);
            f32x8 d = xv - __builtin_convertvector(xp[0], f32x8);
            xp[1] = __builtin_convertvector(d, bf16x8);
            if constexpr (PC == 3) {
                d = d - __builtin_convertvector(xp[1], f32x8);
                xp[2] = __builtin_convertvector(d, bf16x8);
            }
            const int roff = 32 * ks + 8 * g;
            bf16x8 rb[PC][4];
#pragma unroll
            for (int pc = 0; pc < PC; ++pc)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt)
                    rb[pc][nt] = *reinterpret_cast<const bf16x8*>(Rb + (pc * BNP + 16 * nt + m) * BF_RS + roff);
            const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                a1[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xp[0], rb[0][nt], ks == 0 ? zero : a1[nt], 0, 0, 0);
            // the smaller products, in decreasing order of magnitude: x1 r2, x2 r1 (, x1 r3, x2 r2, x3 r1)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) a2[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xp[0], rb[1][nt], a2[nt], 0, 0, 0);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) a2[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xp[1], rb[0][nt], a2[nt], 0, 0, 0);
            if constexpr (PC == 3) {
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) a2[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xp[0], rb[2][nt], a2[nt], 0, 0, 0);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) a2[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xp[1], rb[1][nt], a2[nt], 0, 0, 0);
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) a2[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xp[2], rb[0][nt], a2[nt], 0, 0, 0);
            }
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc64[nt][q] += (double)a1[nt][q];
    };
    auto promote2 = [&]() {
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) {
#pragma unroll
            for (int q = 0; q < 4; ++q) acc64[nt][q] += (double)a2[nt][q];
            a2[nt] = (f32x4){0.f, 0.f, 0.f, 0.f};
        }
    };
    // next chunk's pieces into the other LDS buffer (last read before the previous barrier), then the barrier
    auto next = [&]() {
        stage_store(Rl + ((ch & 1) ^ 1) * PLANE);
        __syncthreads();
        ++ch;
    };
    float xb[3][16];
    // the workgroup's jobs: its Tf whole tiles, then the one or two tiles its range of leftover units touches;
    // a job runs chunks c0 .. c1 - 1 of tile tt into acc64 (zero on entry) and writes the sums out (the whole
    // tile) or stores them in part slot `slot` (some of its rows)
    const int64_t head = u0 / C;
    const int64_t njobs = sp.Tf + (u0 < u1 ? (u1 - 1) / C - head + 1 : 0);
    for (int64_t job = 0; job < njobs; ++job) {
        int64_t tt = wg + job * G, c0 = 0, c1 = C;
        int slot = 0;
        if (job >= sp.Tf) {
            const int64_t tr = head + (job - sp.Tf);
            tt = sp.Tf * G + tr;
            c0 = max(u0 - tr * C, (int64_t)0);
            c1 = min(u1 - tr * C, C);
            slot = tr == head ? 0 : 1;
        }
        const int64_t t = tt * TW + 16 * w + m;
        const int64_t j = t < len ? (cols ? (int64_t)cols[t] : t) : 0;   // lanes past the list read column 0, unused
        xc = X + j * ldx;
        // main loop: groups of three chunks, one per register buffer, whose loads (the pieces of the next
        // chunk, then X two chunks ahead) are all unguarded; the pieces are issued first so that waiting for
        // them leaves the X loads in flight
        const int64_t E = min(F, c1);
        const int64_t Cmain = E - c0 >= 2 ? 3 * ((E - c0 - 2) / 3) : 0;
        load_x(xb[0], c0);
        if (c0 + 1 < c1) load_x(xb[1], c0 + 1);
        // this LDS buffer was last read by the chunk before the previous one, which the last barrier ended
        stage_load(c0);
        stage_store(Rl + (ch & 1) * PLANE);
        __syncthreads();
        int grp = 0;
        for (int64_t ck = c0; ck < c0 + Cmain; ck += 3) {
            stage_load(ck + 1);
            load_fast(xb[2], ck + 2);
            compute(xb[0]);
            next();
            stage_load(ck + 2);
            load_fast(xb[0], ck + 3);
            compute(xb[1]);
            next();
            stage_load(ck + 3);
            load_fast(xb[1], ck + 4);
            compute(xb[2]);
            next();
            if (++grp == BF_PROMO / 3) {
                grp = 0;
                promote2();
            }
        }
        promote2();
        // the last chunks (at most five): guarded loads, one chunk ahead of the pieces and two of X
        for (int64_t ck = c0 + Cmain; ck < c1; ++ck) {
            const bool more = ck + 1 < c1;
            if (more) stage_load(ck + 1);
            float xn[16] = {};
            if (ck + 2 < c1) load_x(xn, ck + 2);
            compute(xb[0]);
            if (more) stage_store(Rl + ((ch & 1) ^ 1) * PLANE);
            __syncthreads();
            ++ch;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                xb[0][q] = xb[1][q];
                xb[1][q] = xn[q];
            }
        }
        promote2();
        // lane (m, g), register q of problem tile nt: column 16 w + 4 g + q of the tile, problem 16 nt + m
        const bool whole = c0 == 0 && c1 == C;
        double* pp = part + (wg * 2 + slot) * (int64_t)TW * BNP;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ci = 16 * w + 4 * g + q;
            const int64_t tq = tt * TW + ci;
            if (tq >= len) continue;
            const int64_t jq = cols ? (int64_t)cols[tq] : tq;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                const int b = 16 * nt + m;
                if (b >= nprob) continue;
                if (whole) bf_store(acc64[nt][q], b, jq, p, bs, c, s, keep, out);
                else pp[(int64_t)b * TW + ci] = acc64[nt][q];
            }
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc64[nt][q] = 0.0;
    }
}

// The cut leftover tiles of a k_bscan_bf16 launch with G workgroups: one thread per (leftover tile, problem,
// column) adds the tile's stored rows in row order, if the tile was cut (a leftover tile one workgroup ran
// whole is written already).
template <int WAVES>
__global__ __launch_bounds__(256) void k_bscan_bf16_join(const int64_t* __restrict__ len_dev, int64_t len_host,
                                                         int64_t n_pad, int64_t G, const int32_t* __restrict__ cols,
                                                         int nprob, int64_t p, const BatchScalars* __restrict__ bs,
                                                         const double* __restrict__ c, const double* __restrict__ s,
                                                         const uint8_t* __restrict__ keep,
                                                         const double* __restrict__ part, double* __restrict__ out) {
    constexpr int TW = 16 * WAVES;
    const int64_t len = len_dev ? *len_dev : len_host;
    const BfSplit sp = tile_split<16 * WAVES>(len, n_pad, G);
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tr = e / (TW * BNP);
    const int b = (int)(e / TW % BNP), ci = (int)(e % TW);
    if (tr >= sp.Trem || b >= nprob) return;
    const int64_t tq = (sp.Tf * G + tr) * TW + ci;
    const int64_t i0 = tr * sp.C / sp.q, i1 = ((tr + 1) * sp.C - 1) / sp.q;
    if (tq >= len || i0 == i1) return;
    double acc = 0.0;
#pragma unroll 8
    for (int64_t i = i0; i <= i1; ++i) {
        const int slot = i * sp.q / sp.C == tr ? 0 : 1;
        acc += part[((i * 2 + slot) * BNP + b) * TW + ci];
    }
    bf_store(acc, b, cols ? (int64_t)cols[tq] : tq, p, bs, c, s, keep, out);
}

// Flag the columns whose matrix-core z, for some problem, lies within its error bound of a threshold the path
// decides on: lambda_k (the check) or thr_k+1 = 2 lambda_{k+1} - lambda_k (the next strong rule; thr null: none).
// rel = bscan_bf16_rel(n_total).
__global__ void k_b_band(const int32_t* __restrict__ cols, const int64_t* __restrict__ len_dev, int64_t p, int nprob,
                         const double* __restrict__ z, const double* __restrict__ c, const double* __restrict__ s,
                         const uint8_t* __restrict__ keep, const BatchScalars* __restrict__ bs,
                         const double* __restrict__ lam, const double* __restrict__ thr, double rel,
                         uint8_t* __restrict__ flag) {
    const int64_t len = *len_dev;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = cols[t];
        uint8_t f = 0;
        for (int b = 0; b < nprob && !f; ++b) {
            const int64_t bj = (int64_t)b * p + j;
            if (keep[bj] == 0) continue;
            const double nb = (double)bs[b].n_rows;
            const double sj = s[bj], cj = c[bj];
            const double az = fabs(z[bj]);
            const double err = rel * sqrt(nb * (sj * sj + cj * cj)) * sqrt(bs[b].rss) / (nb * sj) + 1e-14 * az;
            if (fabs(az - lam[b]) <= err) f = 1;
            if (thr && fabs(az - thr[b]) <= err) f = 1;
        }
        flag[j] = f;
    }
}

// ---- per-problem set-up ---------------------------------------------------------------------------------
// masks (problem-major bytes) -> row-major FP64 right-hand side and row counts
__global__ void k_b_masks(const uint8_t* __restrict__ masks, int64_t n_total, int64_t n_pad, int nprob,
                          double* __restrict__ Mb) {
    const int64_t total = n_pad * BNP;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = idx / BNP;
        const int b = (int)(idx % BNP);
        Mb[idx] = (i < n_total && b < nprob && masks[(int64_t)b * n_total + i]) ? 1.0 : 0.0;
    }
}

// one workgroup per problem: n_b, y_mean, y~ (into the row-major residual and Y~), ||y~||^2
__global__ __launch_bounds__(1024) void k_b_center_y(const uint8_t* __restrict__ masks, const double* __restrict__ Y,
                                                     int64_t n_total, double* __restrict__ Yt, double* __restrict__ R,
                                                     BatchScalars* __restrict__ bs) {
    __shared__ double buf[16];
    const int b = blockIdx.x;
    const uint8_t* mk = masks + (int64_t)b * n_total;
    const double* y = Y + (int64_t)b * n_total;
    double sy = 0.0, cnt = 0.0;
    for (int64_t i = threadIdx.x; i < n_total; i += blockDim.x)
        if (mk[i]) {
            sy += y[i];
            cnt += 1.0;
        }
    const double tot = block_sum(sy, buf), n = block_sum(cnt, buf);
    const double mean = n > 0.0 ? tot / n : 0.0;
    double ss = 0.0;
    for (int64_t i = threadIdx.x; i < n_total; i += blockDim.x) {
        const double v = mk[i] ? y[i] - mean : 0.0;
        Yt[i * BNP + b] = v;
        R[i * BNP + b] = v;
        ss = fma(v, v, ss);
    }
    const double yy = block_sum(ss, buf);
    if (threadIdx.x == 0) {
        bs[b].y_mean = mean;
        bs[b].yy = yy;
        bs[b].n_rows = (int64_t)n;
        bs[b].rss = yy;
    }
}

// sum and sum of squares of each problem's residual column
__global__ __launch_bounds__(1024) void k_b_sum_r(const double* __restrict__ R, int64_t n_total,
                                                  BatchScalars* __restrict__ bs) {
    __shared__ double buf[16];
    const int b = blockIdx.x;
    double a = 0.0, q = 0.0;
    for (int64_t i = threadIdx.x; i < n_total; i += blockDim.x) {
        const double v = R[i * BNP + b];
        a += v;
        q = fma(v, v, q);
    }
    const double ta = block_sum(a, buf), tq = block_sum(q, buf);
    if (threadIdx.x == 0) {
        bs[b].sum_r = ta;
        bs[b].rss = tq;
    }
}

// centers, scales, keep from the masked first and second moments
__global__ void k_b_stats(const double* __restrict__ S1, const double* __restrict__ S2, int64_t p, int nprob,
                          const BatchScalars* __restrict__ bs, double* __restrict__ c, double* __restrict__ s,
                          uint8_t* __restrict__ keep) {
    const int b = blockIdx.y;
    if (b >= nprob) return;
    const double n = (double)bs[b].n_rows;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t bj = (int64_t)b * p + j;
        const double mean = S1[bj] / n;
        const double var = S2[bj] / n - mean * mean;
        const double sd = sqrt(var > 0.0 ? var : 0.0);
        c[bj] = mean;
        s[bj] = sd;
        keep[bj] = sd > 1e-6 ? 1 : 0;
    }
}

// lambda_max and the column attaining it, per problem (ties to the smallest index)
__global__ __launch_bounds__(1024) void k_b_argmax(const double* __restrict__ a, const uint8_t* __restrict__ keep,
                                                   int64_t p, BatchScalars* __restrict__ bs) {
    __shared__ double sv[1024];
    __shared__ int64_t si[1024];
    const int b = blockIdx.x;
    double bv = -1.0;
    int64_t bi = -1;
    for (int64_t j = threadIdx.x; j < p; j += blockDim.x) {
        const int64_t bj = (int64_t)b * p + j;
        if (keep[bj]) {
            const double v = fabs(a[bj]);
            if (v > bv) {
                bv = v;
                bi = j;
            }
        }
    }
    sv[threadIdx.x] = bv;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            const double ov = sv[threadIdx.x + w];
            const int64_t oi = si[threadIdx.x + w];
            if (ov > sv[threadIdx.x] || (ov == sv[threadIdx.x] && oi >= 0 && (si[threadIdx.x] < 0 || oi < si[threadIdx.x]))) {
                sv[threadIdx.x] = ov;
                si[threadIdx.x] = oi;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        bs[b].lmax = sv[0] < 0.0 ? 0.0 : sv[0];
        bs[b].jstar = si[0];
        bs[b].sign_star = (si[0] >= 0 && a[(int64_t)b * p + si[0]] < 0.0) ? -1.0 : 1.0;
    }
}

// right-hand side column b = standardized column jstar_b on problem b's rows
template <typename XT>
__global__ void k_b_std_column(const XT* __restrict__ X, int64_t ldx, int64_t n_total, const uint8_t* __restrict__ masks,
                               int64_t p, int nprob, const BatchScalars* __restrict__ bs, const double* __restrict__ c,
                               const double* __restrict__ s, double* __restrict__ Bm) {
    const int b = blockIdx.y;
    const int64_t js = b < nprob ? bs[b].jstar : -1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_total; i += (int64_t)gridDim.x * blockDim.x) {
        double v = 0.0;
        if (js >= 0 && masks[(int64_t)b * n_total + i]) {
            const int64_t bj = (int64_t)b * p + js;
            v = ((double)X[js * ldx + i] - c[bj]) / s[bj];
        }
        Bm[i * BNP + b] = v;
    }
}

// ---- screening ----------------------------------------------------------------------------------------
// lambda values of step k: lamg[k * BNP + b]; k = koff, plus *kdev when kdev is given (graph replays)
__device__ __forceinline__ const double* step_row(const double* lamg, int koff, const int64_t* kdev) {
    return lamg + ((kdev ? *kdev : 0) + koff) * (int64_t)BNP;
}

__global__ void k_b_bedpp(int64_t p, int nprob, const double* __restrict__ a, const double* __restrict__ bb,
                          const uint8_t* __restrict__ keep, int bedpp, const BatchScalars* __restrict__ bs,
                          const double* __restrict__ lamg, int koff, const int64_t* __restrict__ kdev,
                          uint8_t* __restrict__ safe) {
    const int b = blockIdx.y;
    if (b >= nprob) return;
    const double* lam = step_row(lamg, koff, kdev);
    const double lm = bs[b].lmax, l = lam[b], sg = bs[b].sign_star;
    double slack = bs[b].yy / (double)bs[b].n_rows - lm * lm;
    if (slack < 0.0) slack = 0.0;
    const double rhs = 2.0 * l * lm - (lm - l) * sqrt(slack);
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t bj = (int64_t)b * p + j;
        uint8_t o = keep[bj];
        if (o && bedpp && fabs((lm + l) * a[bj] - (lm - l) * sg * lm * bb[bj]) < rhs) o = 0;
        safe[bj] = o;
    }
}

__global__ void k_b_ssr(int64_t p, int nprob, const uint8_t* __restrict__ safe, const double* __restrict__ beta,
                        const double* __restrict__ zprev, int ssr, const double* __restrict__ thrg, int koff,
                        const int64_t* __restrict__ kdev, const uint8_t* __restrict__ want,
                        uint8_t* __restrict__ strong) {
    const int b = blockIdx.y;
    if (b >= nprob || !want[b]) return;
    const double t = step_row(thrg, koff, kdev)[b];
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t bj = (int64_t)b * p + j;
        uint8_t o = 0;
        if (safe[bj]) o = (!ssr || beta[bj] != 0.0 || fabs(zprev[bj]) >= t) ? 1 : 0;
        strong[bj] = o;
    }
}

// union over problems of a per-problem mask
__global__ void k_b_union(int64_t p, int nprob, const uint8_t* __restrict__ mask, uint8_t* __restrict__ out) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x) {
        uint8_t o = 0;
        for (int b = 0; b < nprob && !o; ++b) o = mask[(int64_t)b * p + j];
        out[j] = o;
    }
}

// post-convergence check per problem over the scanned list
__global__ void k_b_viol(const int32_t* __restrict__ cols, const int64_t* __restrict__ len_dev, int64_t p, int nprob,
                         const double* __restrict__ z, const uint8_t* __restrict__ in_s, uint8_t* __restrict__ inE,
                         const double* __restrict__ lam, const uint8_t* __restrict__ want,
                         BatchScalars* __restrict__ bs) {
    const int b = blockIdx.y;
    if (b >= nprob || !want[b]) return;
    const int64_t len = *len_dev;
    const double l = lam[b];
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < len; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t bj = (int64_t)b * p + cols[t];
        if (in_s[bj] && !inE[bj] && fabs(z[bj]) > l) {
            inE[bj] = 1;
            atomicAdd(&bs[b].n_viol, 1u);
        }
    }
}

// ---- ordered compaction, one problem per grid row -----------------------------------------------------
constexpr int CT = 256, CI = 16, CTILE = CT * CI;

__global__ __launch_bounds__(CT) void k_b_cmp_count(const uint8_t* __restrict__ mask, int64_t p,
                                                    const uint8_t* __restrict__ want, int32_t* __restrict__ counts,
                                                    int64_t nblk) {
    __shared__ int32_t sh[CT / WAVE];
    const int b = blockIdx.y;
    if (!want[b]) return;
    const uint8_t* mk = mask + (int64_t)b * p;
    const int64_t base = (int64_t)blockIdx.x * CTILE + (int64_t)threadIdx.x * CI;
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < CI; ++k)
        if (base + k < p && mk[base + k]) ++cnt;
#pragma unroll
    for (int off = WAVE / 2; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < CT / WAVE; ++w) t += sh[w];
        counts[(int64_t)b * nblk + blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_b_cmp_scan(int32_t* __restrict__ counts, int64_t nblk,
                                                     const uint8_t* __restrict__ want, int64_t* __restrict__ total) {
    __shared__ int64_t sh[1024];
    __shared__ int64_t carry;
    const int b = blockIdx.x;
    if (!want[b]) return;
    int32_t* cb = counts + (int64_t)b * nblk;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < nblk; b0 += blockDim.x) {
        const int64_t k = b0 + threadIdx.x;
        const int64_t v = k < nblk ? cb[k] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < (int)blockDim.x; off <<= 1) {
            const int64_t add = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        const int64_t incl = sh[threadIdx.x];
        if (k < nblk) cb[k] = (int32_t)(carry + incl - v);
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry += incl;
        __syncthreads();
    }
    if (threadIdx.x == 0) total[b] = carry;
}

__global__ __launch_bounds__(CT) void k_b_cmp_write(const uint8_t* __restrict__ mask, int64_t p,
                                                    const uint8_t* __restrict__ want,
                                                    const int32_t* __restrict__ offsets, int64_t nblk,
                                                    int32_t* __restrict__ out) {
    __shared__ int32_t sh[CT];
    const int b = blockIdx.y;
    if (!want[b]) return;
    const uint8_t* mk = mask + (int64_t)b * p;
    const int64_t base = (int64_t)blockIdx.x * CTILE + (int64_t)threadIdx.x * CI;
    uint8_t f[CI];
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < CI; ++k) {
        f[k] = (base + k < p) ? mk[base + k] : 0;
        cnt += f[k] ? 1 : 0;
    }
    sh[threadIdx.x] = cnt;
    __syncthreads();
    for (int off = 1; off < CT; off <<= 1) {
        const int add = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    int pos = offsets[(int64_t)b * nblk + blockIdx.x] + sh[threadIdx.x] - cnt;
    int32_t* ob = out + (int64_t)b * p;
#pragma unroll
    for (int k = 0; k < CI; ++k)
        if (f[k]) ob[pos++] = (int32_t)(base + k);
}

// ---- Gram pools, one per problem ------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_b_pool_add(const int32_t* __restrict__ sets, const int64_t* __restrict__ lens,
                                                     int64_t p, const uint8_t* __restrict__ want,
                                                     int32_t* __restrict__ pool_pos, int32_t* __restrict__ pool_list,
                                                     BatchScalars* __restrict__ bs) {
    __shared__ int32_t sh[1024];
    __shared__ int64_t carry;
    const int b = blockIdx.x;
    if (!want[b]) return;
    const int32_t* set = sets + (int64_t)b * p;
    int32_t* pos_b = pool_pos + (int64_t)b * p;
    int32_t* list_b = pool_list + (int64_t)b * p;
    const int64_t len = lens[b];
    const int64_t base_size = bs[b].pool_size;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b0 = 0; b0 < len; b0 += blockDim.x) {
        const int64_t t = b0 + threadIdx.x;
        int32_t j = -1;
        int flag = 0;
        if (t < len) {
            j = set[t];
            flag = pos_b[j] < 0 ? 1 : 0;
        }
        sh[threadIdx.x] = flag;
        __syncthreads();
        for (int off = 1; off < (int)blockDim.x; off <<= 1) {
            const int add = (int)threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (flag) {
            const int64_t ps = base_size + carry + sh[threadIdx.x] - 1;
            pos_b[j] = (int32_t)ps;
            list_b[ps] = j;
        }
        __syncthreads();
        if (threadIdx.x == blockDim.x - 1) carry += sh[threadIdx.x];
        __syncthreads();
    }
    if (threadIdx.x == 0) bs[b].n_new = carry;
}

// after a pool update: pool_size += n_new; and the per-round counters start again
__global__ void k_b_commit(int nprob, const uint8_t* __restrict__ want, BatchScalars* __restrict__ bs) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nprob && want[b]) {
        bs[b].pool_size += bs[b].n_new;
        bs[b].n_new = 0;
        bs[b].n_viol = 0u;
    }
}

// Gram entries of problem b's new pool members against its pool (grid.z = problem; masked rows), on FP64
// matrix cores: each workgroup holds a 32 x 16 tile of C[k, t] = sum_i m_b(i) x_{pool[k], i} x_{pool[P0+t], i},
// its four waves take a quarter of the rows each (64 rows a step, the next step's values loaded while the
// current one is multiplied) and their partial tiles are added in wave order through LDS.  Lane (m, kq)
// feeds rows i0 + 16 kq .. + 15 of pool columns kb + m, kb + 16 + m and new column tb + m; register q of its
// result holds C[kb + kq + 4q (+ 16), tb + m].  A pair of two new columns is written by the tile with
// k - P0 <= t only, so each problem's G stays exactly symmetric.
// VEC: columns and every problem's mask row are 16-byte aligned: full 64-row steps read each lane's 16 values
// as 16-byte words with no per-element test (the same operands as the guarded path, which only a final partial
// step takes), the next step's loads in flight during the current step's matrix-core work.
constexpr int BG_W = 4, BG_K = 32, BG_N = 16, BG_R = 64;

// 16 consecutive elements of a column, read as 16-byte words (p 16-byte aligned)
template <typename XT>
__device__ __forceinline__ void bload16(const XT* p, XT (&dst)[16]) {
    typedef int v4w __attribute__((ext_vector_type(4)));
    constexpr int NV = 16 * (int)sizeof(XT) / 16;
    v4w t[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) t[i] = reinterpret_cast<const v4w*>(p)[i];
    __builtin_memcpy(dst, t, sizeof(t));
}

template <typename XT, bool VEC>
__global__ __launch_bounds__(64 * BG_W) void k_b_gram_update(const XT* __restrict__ X, int64_t ldx, int64_t n_total,
                                                            const uint8_t* __restrict__ masks, int64_t p,
                                                            const int32_t* __restrict__ pool_list,
                                                            const BatchScalars* __restrict__ bs,
                                                            const double* __restrict__ c,
                                                            const double* __restrict__ s, double* __restrict__ Gp,
                                                            int64_t cap, const uint8_t* __restrict__ want) {
    __shared__ f64x4 red[BG_W - 1][2][WAVE];
    const int b = blockIdx.z;
    if (!want[b]) return;
    const int64_t N = bs[b].n_new, P0 = bs[b].pool_size, P = P0 + N;
    const int64_t kb = (int64_t)blockIdx.x * BG_K, tb = (int64_t)blockIdx.y * BG_N;
    if (kb >= P || tb >= N) return;   // whole workgroup, before its barrier
    const int32_t* list = pool_list + (int64_t)b * p;
    const uint8_t* mk = masks + (int64_t)b * n_total;
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int m = lane & 15, kq = lane >> 4;
    const XT* ac[2];
    bool aok[2];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
        const int64_t k = kb + 16 * f + m;
        aok[f] = k < P;
        ac[f] = X + (int64_t)(aok[f] ? list[k] : 0) * ldx;
    }
    const bool bok = tb + m < N;
    const XT* bc = X + (int64_t)(bok ? list[P0 + tb + m] : 0) * ldx;
    const int64_t ns = (n_total + BG_R - 1) / BG_R;
    const int64_t s0 = ns * w / BG_W, s1 = ns * (w + 1) / BG_W;
    XT ra[2][16], rb[16];
    bool rm[16];
    auto load = [&](int64_t step) {
        const int64_t r0 = step * BG_R + 16 * kq;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const bool in = r0 + q < n_total;
            ra[0][q] = (aok[0] && in) ? ac[0][r0 + q] : (XT)0;
            ra[1][q] = (aok[1] && in) ? ac[1][r0 + q] : (XT)0;
            rb[q] = (bok && in) ? bc[r0 + q] : (XT)0;
            rm[q] = in && mk[r0 + q] != 0;
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
        auto load_full = [&](int64_t step) {
            const int64_t r0 = step * BG_R + 16 * kq;
            bload16<XT>(ac[0] + r0, ra[0]);
            bload16<XT>(ac[1] + r0, ra[1]);
            bload16<XT>(bc + r0, rb);
            typedef int v4w __attribute__((ext_vector_type(4)));
            const v4w mw = *reinterpret_cast<const v4w*>(mk + r0);
#pragma unroll
            for (int q = 0; q < 16; ++q) rm[q] = ((mw[q >> 2] >> (8 * (q & 3))) & 0xff) != 0;
        };
        const int64_t nfs = n_total / BG_R;
        const int64_t f1 = s1 < nfs ? s1 : nfs;
        if (s0 < f1) load_full(s0);
        for (int64_t step = s0; step < f1; ++step) {
            auto run = step_mfma();                          // the current step's operands, converted
            load_full(step + 1 < f1 ? step + 1 : f1 - 1);   // unconditional (the last full step reloads)
            asm volatile("" ::: "memory");
            __builtin_amdgcn_sched_barrier(0);
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
    for (int v = 0; v < BG_W - 1; ++v) {
        acc[0] += red[v][0][lane];
        acc[1] += red[v][1][lane];
    }
    const int64_t t = tb + m;
    if (t >= N) return;
    const double* cb = c + (int64_t)b * p;
    const double* sb = s + (int64_t)b * p;
    double* G = Gp + (int64_t)b * cap * cap;
    const double nb = (double)bs[b].n_rows;
    const int jt = list[P0 + t];
#pragma unroll
    for (int f = 0; f < 2; ++f) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t k = kb + 16 * f + kq + 4 * q;
            if (k >= P) continue;
            if (k >= P0 && k - P0 > t) continue;   // written by the tile of its mirror
            const int jk = list[k];
            const double gv = (acc[f][q] - nb * (cb[jk] * cb[jt])) / (nb * (sb[jk] * sb[jt]));
            G[k * cap + (P0 + t)] = gv;
            G[(P0 + t) * cap + k] = gv;
        }
    }
}

// working-set Gram, start gradient and coefficients of each problem (grid.y = problem)
__global__ void k_b_gather(const int32_t* __restrict__ sets, const int64_t* __restrict__ lens, int64_t p,
                           const uint8_t* __restrict__ want, const int32_t* __restrict__ pool_pos,
                           const double* __restrict__ Gp, int64_t cap, const double* __restrict__ z,
                           const double* __restrict__ beta, double* __restrict__ GE, int64_t ge_stride,
                           double* __restrict__ g0, double* __restrict__ b0) {
    const int b = blockIdx.y;
    if (!want[b]) return;
    const int64_t m = lens[b];
    const int32_t* set = sets + (int64_t)b * p;
    const int32_t* pos = pool_pos + (int64_t)b * p;
    const double* G = Gp + (int64_t)b * cap * cap;
    double* ge = GE + (int64_t)b * ge_stride;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < m * m; idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = idx / m, f = idx - e * m;
        ge[idx] = G[(int64_t)pos[set[e]] * cap + pos[set[f]]];
    }
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t bj = (int64_t)b * p + set[e];
        g0[(int64_t)b * p + e] = z[bj];
        b0[(int64_t)b * p + e] = beta[bj];
    }
}

// ---- coordinate descent, one workgroup per problem ---------------------------------------------------------
// The single-workgroup covariance solve (blocked chain in one wavefront, block changes pushed by the
// workgroup) for problem blockIdx.x.
constexpr int BCD_T = 512, BCD_B = 64;

__global__ __launch_bounds__(BCD_T) void k_b_gcd(const int32_t* __restrict__ sets, const int64_t* __restrict__ lens,
                                                 int64_t p, const uint8_t* __restrict__ want,
                                                 const double* __restrict__ GE, int64_t ge_stride,
                                                 const double* __restrict__ g0, const double* __restrict__ b0,
                                                 double* __restrict__ b1, double* __restrict__ beta,
                                                 const double* __restrict__ lam, double tol, int max_sweeps,
                                                 BatchScalars* __restrict__ bs) {
    __shared__ double g[BCD_MAX];
    __shared__ double bE[BCD_MAX];
    __shared__ double Gbb[BCD_B * BCD_B];
    __shared__ double dlt[BCD_B];
    __shared__ int nz[BCD_B];
    __shared__ int nnz_sh;
    __shared__ double maxd_sh;
    const int pb = blockIdx.x;
    if (!want[pb]) return;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wv = tid / WAVE;
    const int64_t m = lens[pb];
    const double l = lam[pb];
    const double* G = GE + (int64_t)pb * ge_stride;
    const int32_t* set = sets + (int64_t)pb * p;
    for (int64_t e = tid; e < m; e += BCD_T) {
        g[e] = g0[(int64_t)pb * p + e];
        bE[e] = b0[(int64_t)pb * p + e];
    }
    int sweeps = 0, status = 0;
    if (tid == 0) maxd_sh = 0.0;
    __syncthreads();
    if (m > 0) {
        for (;;) {
            for (int64_t q0 = 0; q0 < m; q0 += BCD_B) {
                const int bl = (int)((m - q0) < BCD_B ? (m - q0) : BCD_B);
                for (int idx = tid; idx < BCD_B * BCD_B; idx += BCD_T) {
                    const int t = idx / BCD_B, r = idx % BCD_B;
                    Gbb[idx] = (t < bl && r < bl) ? G[(q0 + t) * m + q0 + r] : 0.0;
                }
                __syncthreads();
                if (wv == 0) {
                    double gl = lane < bl ? g[q0 + lane] : 0.0;
                    double bv = lane < bl ? bE[q0 + lane] : 0.0;
                    double dl = 0.0, wmax = 0.0;
                    auto col = [&](int t) { return Gbb[t * BCD_B + lane]; };
                    if (!chain_fast<BCD_B>(gl, bv, col, l, bl, dl, wmax)) chain_exact<BCD_B>(gl, bv, col, l, bl, dl, wmax);
                    if (lane < bl) {
                        g[q0 + lane] = gl;
                        bE[q0 + lane] = bv;
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
                    for (int64_t k = tid; k < m; k += BCD_T) {
                        if (k >= q0 && k < q0 + bl) continue;
                        double acc = g[k];
                        for (int q = 0; q < nnz; ++q) {
                            const int t = nz[q];
                            acc = fma(-dlt[t], G[(q0 + t) * m + k], acc);
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
            if (md < tol) break;
            if (sweeps >= max_sweeps) {
                status = 1;
                break;
            }
            __syncthreads();
        }
    } else {
        sweeps = 1;
    }
    __syncthreads();
    for (int64_t e = tid; e < m; e += BCD_T) {
        b1[(int64_t)pb * p + e] = bE[e];
        beta[(int64_t)pb * p + set[e]] = bE[e];
    }
    if (tid == 0) {
        bs[pb].sweeps = sweeps;
        bs[pb].status = status;
    }
}

// residual update of every problem after its solve: R[:, b] -= X~_{E_b} (b1 - b0) on b's rows
constexpr int BRU_CHUNK = 64;

template <typename XT>
__global__ __launch_bounds__(256) void k_b_r_update(const XT* __restrict__ X, int64_t ldx, int64_t n_total,
                                                    const uint8_t* __restrict__ masks, const int32_t* __restrict__ sets,
                                                    const int64_t* __restrict__ lens, int64_t p,
                                                    const uint8_t* __restrict__ want, const double* __restrict__ b0,
                                                    const double* __restrict__ b1, const double* __restrict__ c,
                                                    const double* __restrict__ s, double* __restrict__ R) {
    const int b = blockIdx.y;
    if (!want[b]) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_total || !masks[(int64_t)b * n_total + i]) return;
    const int64_t m = lens[b];
    const int32_t* set = sets + (int64_t)b * p;
    double acc = 0.0;
    for (int64_t e = 0; e < m; ++e) {
        const double d = b1[(int64_t)b * p + e] - b0[(int64_t)b * p + e];
        if (d == 0.0) continue;
        const int64_t bj = (int64_t)b * p + set[e];
        acc = fma(d / s[bj], (double)X[(int64_t)set[e] * ldx + i] - c[bj], acc);
    }
    R[i * BNP + b] -= acc;
}

// per-lambda record of every problem
__global__ __launch_bounds__(1024) void k_b_record(const int32_t* __restrict__ sets, const int64_t* __restrict__ lens,
                                                   int64_t p, const double* __restrict__ beta, const double* __restrict__ c,
                                                   const double* __restrict__ s, const BatchScalars* __restrict__ bs,
                                                   const double* __restrict__ lam, LamStats* __restrict__ out,
                                                   int k, int K, const int64_t* __restrict__ n_safe) {
    __shared__ double buf[16];
    const int b = blockIdx.x;
    const int64_t m = lens ? lens[b] : 0;
    const int32_t* set = sets + (int64_t)b * p;
    double l1 = 0.0, cb = 0.0, na = 0.0;
    for (int64_t t = threadIdx.x; t < m; t += blockDim.x) {
        const int64_t bj = (int64_t)b * p + set[t];
        const double v = beta[bj];
        if (v != 0.0) {
            l1 += fabs(v);
            cb += c[bj] * v / s[bj];
            na += 1.0;
        }
    }
    const double tl1 = block_sum(l1, buf), tcb = block_sum(cb, buf), tna = block_sum(na, buf);
    if (threadIdx.x == 0) {
        LamStats* o = out + (int64_t)b * K + k;
        o->rss = bs[b].rss;
        o->l1 = tl1;
        o->n_active = (int64_t)tna;
        o->intercept = bs[b].y_mean - tcb;
        o->obj = bs[b].rss / (2.0 * (double)bs[b].n_rows) + lam[b] * tl1;
        o->n_strong = m;
        o->n_safe = n_safe ? n_safe[b] : 0;
        o->n_scan = 0;
    }
}

}  // namespace

// ---- launchers -------------------------------------------------------------------------------------------------
int64_t batch_pad(int64_t n_total) { return (n_total + BS_K - 1) / BS_K * BS_K; }

// workgroups of k_bscan<XT, MODE, WAVES, PF> the device holds at once, at most two per CU (the size of the
// part scratch, bscan_part_bytes, assumes that bound; the 67.5 KB of LDS a workgroup takes allows no more)
template <typename XT, int MODE, int WAVES, bool PF>
static int bscan_slots() {
    static int cached = 0;
    if (!cached) {
        int per_cu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bscan<XT, MODE, WAVES, PF>, 64 * WAVES, 0) !=
                hipSuccess ||
            per_cu < 1) {
            (void)hipGetLastError();
            per_cu = 1;
        }
        cached = (per_cu < 2 ? per_cu : 2) * device_cu_count();
    }
    return cached;
}

size_t bscan_part_bytes() { return (size_t)2 * device_cu_count() * 2 * (32 * 8) * BNP * sizeof(double); }

template <typename XT, int MODE, int WAVES, bool PF>
static hipError_t bscan_mode(const Mat& mt, const int32_t* cols, const int64_t* len_dev, int64_t len_host,
                             const double* B, int nprob, BatchScalars* bs, const double* c, const double* s,
                             const uint8_t* keep, double* part, double* out, hipStream_t st) {
    constexpr int TF = 32 * WAVES;
    const int64_t n_pad = batch_pad(mt.n_total);
    const int g = bscan_slots<XT, MODE, WAVES, PF>();
    k_bscan<XT, MODE, WAVES, PF><<<g, 64 * WAVES, 0, st>>>((const XT*)mt.X, mt.ldx, mt.n_total, n_pad, cols, len_dev,
                                                           len_host, B, nprob, mt.p, bs, c, s, keep, part, out, n_pad);
    // at most g - 1 leftover tiles (fewer when the list length is on the host)
    int64_t tiles = g - 1;
    if (!len_dev) tiles = std::min(tiles, (len_host + TF - 1) / TF);
    if (tiles > 0)
        k_bscan_join<TF, MODE><<<(int)(tiles * TF * BNP / 256), 256, 0, st>>>(len_dev, len_host, n_pad, g, cols, nprob,
                                                                            mt.p, bs, c, s, keep, part, out);
    return hipGetLastError();
}

template <typename XT, int WAVES, bool PF>
static hipError_t bscan_typed(const Mat& mt, int mode, const int32_t* cols, const int64_t* len_dev, int64_t len_host,
                              const double* B, int nprob, BatchScalars* bs, const double* c, const double* s,
                              const uint8_t* keep, double* part, double* out, hipStream_t st) {
    if (!len_dev && len_host <= 0) return hipSuccess;
    if (batch_pad(mt.n_total) <= 0) return hipErrorInvalidValue;
    if (mode == 0) return bscan_mode<XT, 0, WAVES, PF>(mt, cols, len_dev, len_host, B, nprob, bs, c, s, keep, part, out, st);
    if (mode == 1) return bscan_mode<XT, 1, WAVES, PF>(mt, cols, len_dev, len_host, B, nprob, bs, c, s, keep, part, out, st);
    return bscan_mode<XT, 2, WAVES, PF>(mt, cols, len_dev, len_host, B, nprob, bs, c, s, keep, part, out, st);
}

// sum of the row-range partials in range order, then the standardized correlation of each (column, problem)
__global__ void k_bscan_reduce(const double* __restrict__ part, int nch, int64_t len, const int32_t* __restrict__ cols,
                               int64_t p, int nprob, const BatchScalars* __restrict__ bs, const double* __restrict__ c,
                               const double* __restrict__ s, const uint8_t* __restrict__ keep, double* __restrict__ out) {
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < len * BNP;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int64_t t = idx / BNP;
        const int b = (int)(idx % BNP);
        if (b >= nprob) continue;
        double v = 0.0;
        for (int q = 0; q < nch; ++q) v += part[((int64_t)q * len + t) * BNP + b];
        const int64_t j = cols[t];
        const int64_t bj = (int64_t)b * p + j;
        const bool kept = keep == nullptr || keep[bj] != 0;
        out[bj] = kept ? (v - c[bj] * bs[b].sum_r) / ((double)bs[b].n_rows * s[bj]) : 0.0;
    }
}

constexpr int SPLIT_ROWS = 2048;   // rows per partial of the split scan (a multiple of BS_K)

template <typename XT>
static hipError_t bscan_split_typed(const Mat& mt, const int32_t* cols, int64_t len, const double* B, int nprob,
                                    const BatchScalars* bs, const double* c, const double* s, const uint8_t* keep,
                                    double* part, double* out, hipStream_t st) {
    constexpr int W = 2, TF = 32 * W;
    const int64_t n_pad = batch_pad(mt.n_total);
    const int nch = (int)((n_pad + SPLIT_ROWS - 1) / SPLIT_ROWS);
    dim3 grid((unsigned)((len + TF - 1) / TF), (unsigned)nch);
    k_bscan<XT, 3, W, false><<<grid, 64 * W, 0, st>>>((const XT*)mt.X, mt.ldx, mt.n_total, n_pad, cols, nullptr, len, B,
                                                      nprob, mt.p, nullptr, nullptr, nullptr, nullptr, nullptr, part,
                                                      SPLIT_ROWS);
    k_bscan_reduce<<<grid_for(len * BNP, 256, 4096), 256, 0, st>>>(part, nch, len, cols, mt.p, nprob, bs, c, s, keep,
                                                                    out);
    return hipGetLastError();
}

template <typename XT>
static hipError_t bscan_waves(int variant, const Mat& mt, int mode, const int32_t* cols, const int64_t* len_dev,
                              int64_t len_host, const double* B, int nprob, BatchScalars* bs, const double* c,
                              const double* s, const uint8_t* keep, double* part, double* out, hipStream_t st) {
#define BSCAN_CASE(V, W, P) \
    case V: return bscan_typed<XT, W, P>(mt, mode, cols, len_dev, len_host, B, nprob, bs, c, s, keep, part, out, st);
    switch (variant) {
        BSCAN_CASE(0, 2, false)
        BSCAN_CASE(2, 8, false)
        BSCAN_CASE(3, 2, true)
        BSCAN_CASE(4, 4, true)
        BSCAN_CASE(5, 8, true)
        default: return bscan_typed<XT, 4, false>(mt, mode, cols, len_dev, len_host, B, nprob, bs, c, s, keep, part, out, st);
    }
#undef BSCAN_CASE
}

int bscan_variant_cols(int variant) { return 32 * (variant % 3 == 0 ? 2 : (variant % 3 == 1 ? 4 : 8)); }

size_t bscan_split_part_bytes(int64_t n_total, int64_t len) {
    const int64_t nch = (batch_pad(n_total) + SPLIT_ROWS - 1) / SPLIT_ROWS;
    return (size_t)nch * (size_t)(len > 0 ? len : 1) * BNP * sizeof(double);
}

hipError_t launch_bscan_split(const Mat& mt, const int32_t* cols, int64_t len, const double* B, int nprob,
                              const BatchScalars* bs, const double* c, const double* s, const uint8_t* keep,
                              double* part, double* out, hipStream_t st) {
    if (len <= 0) return hipSuccess;
    if (mt.xtype == 0) return bscan_split_typed<double>(mt, cols, len, B, nprob, bs, c, s, keep, part, out, st);
    return bscan_split_typed<float>(mt, cols, len, B, nprob, bs, c, s, keep, part, out, st);
}

hipError_t launch_bscan(const Mat& mt, int mode, const int32_t* cols, const int64_t* len_dev, int64_t len_host,
                        const double* B, int nprob, BatchScalars* bs, const double* c, const double* s,
                        const uint8_t* keep, double* part, double* out, hipStream_t st, int variant) {
    if (mt.xtype == 0)
        return bscan_waves<double>(variant, mt, mode, cols, len_dev, len_host, B, nprob, bs, c, s, keep, part, out, st);
    return bscan_waves<float>(variant, mt, mode, cols, len_dev, len_host, B, nprob, bs, c, s, keep, part, out, st);
}

// Relative factor of the BF16 scan's bound on |z~ - z_fp64| (times sqrt(n_b (s^2 + c^2)) ||r_b||_2 / (n_b s),
// which bounds sum_i |x_ij| |r_ib| / (n_b s_j) by Cauchy-Schwarz), for pc pieces of x and r.  With e = 2^-8,
// er = e + 2u (u = 2^-24) and |x_a| <= e^(a-1) (1 + e) |x|, |r_b| <= er^(b-1) (1 + er) |r|:
//   the dropped products (a + b > pc + 1), the remainders dx (e^pc |x|, kept although x is exact for pc = 3 and
//   normal f32 values) and dr (er^pc |r|);
//   the FP32 sums, bounded as sequential FP32 additions of every product (a matrix-core step adds 32 exact
//   products of BF16 pieces to its accumulator): gamma_64 on x_1 r_1 (one chunk) and gamma_N2 on the other
//   products (N2 = 64 BF_PROMO (products - 1) terms between promotions);
//   the FP64 sums of the promoted values (one per chunk, one per BF_PROMO chunks, at most 2 n / 64 + 8 terms)
//   and the FP64 scan's own rounding over n rows (2 n 2^-53), so that decisions outside the band are the FP64
//   scan's.
double bscan_bf16_rel(int64_t n_total, int pc) {
    const double u = std::ldexp(1.0, -24), u64 = std::ldexp(1.0, -53), e = std::ldexp(1.0, -8), er = e + 2.0 * u;
    auto gam = [&](double k) { return k * u / (1.0 - k * u); };
    double dropped = 0.0, kept_small = 0.0;
    int nprod = 0;
    for (int a = 1; a <= pc; ++a)
        for (int b = 1; b <= pc; ++b) {
            const double mag = std::pow(e, a - 1) * (1.0 + e) * std::pow(er, b - 1) * (1.0 + er);
            if (a + b > pc + 1) {
                dropped += mag;
            } else {
                ++nprod;
                if (a + b > 2) kept_small += mag;
            }
        }
    const double rem = std::pow(e, pc) * (1.0 + std::pow(er, pc)) + std::pow(er, pc) * (1.0 + std::pow(e, pc));
    const double first = gam(64.0) * (1.0 + e) * (1.0 + er);
    const double rest = gam(64.0 * BF_PROMO * (nprod - 1)) * kept_small;
    const double g64 = (2.0 * (double)(n_total / BF_K) + 8.0) * u64 * (1.0 + first + kept_small) + 2.0 * (double)n_total * u64;
    return (dropped + rem + first + rest) * (1.0 + 1e-6) + g64;
}

int64_t bscan_bf16_pieces_bytes(int64_t n_total, int pc) { return (int64_t)pc * BNP * batch_pad(n_total) * 2; }

hipError_t launch_b_r_pieces(const double* R, int64_t n_total, int nprob, int pc, __bf16* Rp, hipStream_t st) {
    const int64_t n_pad = batch_pad(n_total);
    k_b_r_pieces<<<grid_for(n_pad * BNP, 256, 4096), 256, 0, st>>>(R, n_total, n_pad, nprob, pc, Rp);
    return hipGetLastError();
}

// workgroups of k_bscan_bf16 the device holds at once (its launches take exactly that many)
constexpr int BF_W = 8;   // 128 columns per workgroup share each staged chunk of residual pieces
int bscan_bf16_slots(int pc) {
    static int cached[2] = {0, 0};
    int& n = cached[pc == 3 ? 1 : 0];
    if (!n) {
        int per_cu = 0;
        const hipError_t e = pc == 3
            ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bscan_bf16<BF_W, 3>, 64 * BF_W, 0)
            : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_bscan_bf16<BF_W, 2>, 64 * BF_W, 0);
        if (e != hipSuccess || per_cu < 1) {
            (void)hipGetLastError();
            per_cu = 1;
        }
        n = per_cu * device_cu_count();
    }
    return n;
}

size_t bscan_bf16_part_bytes(int pc) { return (size_t)bscan_bf16_slots(pc) * 2 * 16 * BF_W * BNP * sizeof(double); }

hipError_t launch_bscan_bf16(const Mat& mt, const int32_t* cols, const int64_t* len_dev, int64_t len_host, int pc,
                             const __bf16* Rp, int nprob, const BatchScalars* bs, const double* c, const double* s,
                             const uint8_t* keep, double* part, double* out, hipStream_t st) {
    const int g = bscan_bf16_slots(pc);
    const float* X = (const float*)mt.X;
    const int64_t n_pad = batch_pad(mt.n_total);
    if (n_pad <= 0) return hipErrorInvalidValue;
    if (pc == 2)
        k_bscan_bf16<BF_W, 2><<<g, 64 * BF_W, 0, st>>>(X, mt.ldx, mt.n_total, n_pad, Rp, cols, len_dev, len_host, nprob,
                                                      mt.p, bs, c, s, keep, part, out);
    else
        k_bscan_bf16<BF_W, 3><<<g, 64 * BF_W, 0, st>>>(X, mt.ldx, mt.n_total, n_pad, Rp, cols, len_dev, len_host, nprob,
                                                      mt.p, bs, c, s, keep, part, out);
    // at most g - 1 leftover tiles (fewer when the list length is on the host)
    int64_t tiles = g - 1;
    if (!len_dev) tiles = std::min(tiles, (len_host + 16 * BF_W - 1) / (16 * BF_W));
    if (tiles > 0)
        k_bscan_bf16_join<BF_W><<<(int)(tiles * 16 * BF_W * BNP / 256), 256, 0, st>>>(len_dev, len_host, n_pad, g, cols,
                                                                                     nprob, mt.p, bs, c, s, keep, part,
                                                                                     out);
    return hipGetLastError();
}

hipError_t launch_b_band(const int32_t* cols, const int64_t* len_dev, int64_t p, int nprob, const double* z,
                         const double* c, const double* s, const uint8_t* keep, const BatchScalars* bs,
                         const double* lam, const double* thr, double rel, uint8_t* flag, hipStream_t st) {
    k_b_band<<<grid_for(p, 256, 4096), 256, 0, st>>>(cols, len_dev, p, nprob, z, c, s, keep, bs, lam, thr, rel, flag);
    return hipGetLastError();
}

hipError_t launch_b_masks(const uint8_t* masks, int64_t n_total, int nprob, double* Mb, hipStream_t st) {
    const int64_t n_pad = batch_pad(n_total);
    k_b_masks<<<grid_for(n_pad * BNP, 256, 4096), 256, 0, st>>>(masks, n_total, n_pad, nprob, Mb);
    return hipGetLastError();
}

hipError_t launch_b_center_y(const uint8_t* masks, const double* Y, int64_t n_total, int nprob, double* Yt, double* R,
                             BatchScalars* bs, hipStream_t st) {
    k_b_center_y<<<nprob, 1024, 0, st>>>(masks, Y, n_total, Yt, R, bs);
    return hipGetLastError();
}

hipError_t launch_b_sum_r(const double* R, int64_t n_total, int nprob, BatchScalars* bs, hipStream_t st) {
    k_b_sum_r<<<nprob, 1024, 0, st>>>(R, n_total, bs);
    return hipGetLastError();
}

hipError_t launch_b_stats(const double* S1, const double* S2, int64_t p, int nprob, const BatchScalars* bs, double* c,
                          double* s, uint8_t* keep, hipStream_t st) {
    dim3 grid(grid_for(p, 256, 256), nprob);
    k_b_stats<<<grid, 256, 0, st>>>(S1, S2, p, nprob, bs, c, s, keep);
    return hipGetLastError();
}

hipError_t launch_b_argmax(const double* a, const uint8_t* keep, int64_t p, int nprob, BatchScalars* bs,
                           hipStream_t st) {
    k_b_argmax<<<nprob, 1024, 0, st>>>(a, keep, p, bs);
    return hipGetLastError();
}

hipError_t launch_b_std_column(const Mat& mt, const uint8_t* masks, int nprob, const BatchScalars* bs, const double* c,
                               const double* s, double* Bm, hipStream_t st) {
    dim3 grid(grid_for(mt.n_total, 256, 64), BNP);
    if (mt.xtype == 0)
        k_b_std_column<double><<<grid, 256, 0, st>>>((const double*)mt.X, mt.ldx, mt.n_total, masks, mt.p, nprob, bs,
                                                     c, s, Bm);
    else
        k_b_std_column<float><<<grid, 256, 0, st>>>((const float*)mt.X, mt.ldx, mt.n_total, masks, mt.p, nprob, bs, c,
                                                    s, Bm);
    return hipGetLastError();
}

hipError_t launch_b_bedpp(int64_t p, int nprob, const double* a, const double* bb, const uint8_t* keep, bool bedpp,
                          const BatchScalars* bs, const double* lamg, int koff, const int64_t* kdev, uint8_t* safe,
                          hipStream_t st) {
    dim3 grid(grid_for(p, 256, 256), nprob);
    k_b_bedpp<<<grid, 256, 0, st>>>(p, nprob, a, bb, keep, bedpp ? 1 : 0, bs, lamg, koff, kdev, safe);
    return hipGetLastError();
}

hipError_t launch_b_ssr(int64_t p, int nprob, const uint8_t* safe, const double* beta, const double* zprev, bool ssr,
                        const double* thrg, int koff, const int64_t* kdev, const uint8_t* want, uint8_t* strong,
                        hipStream_t st) {
    dim3 grid(grid_for(p, 256, 256), nprob);
    k_b_ssr<<<grid, 256, 0, st>>>(p, nprob, safe, beta, zprev, ssr ? 1 : 0, thrg, koff, kdev, want, strong);
    return hipGetLastError();
}

hipError_t launch_b_union(int64_t p, int nprob, const uint8_t* mask, uint8_t* out, hipStream_t st) {
    k_b_union<<<grid_for(p, 256, 2048), 256, 0, st>>>(p, nprob, mask, out);
    return hipGetLastError();
}

hipError_t launch_b_viol(const int32_t* cols, const int64_t* len_dev, int64_t p, int nprob, const double* z,
                         const uint8_t* in_s, uint8_t* inE, const double* lam, const uint8_t* want, BatchScalars* bs,
                         hipStream_t st) {
    dim3 grid(grid_for(p, 256, 256), nprob);
    k_b_viol<<<grid, 256, 0, st>>>(cols, len_dev, p, nprob, z, in_s, inE, lam, want, bs);
    return hipGetLastError();
}

size_t b_compact_scratch_bytes(int64_t p) {
    const int64_t nblk = (p + CTILE - 1) / CTILE;
    return (size_t)BNP * (size_t)(nblk < 1 ? 1 : nblk) * sizeof(int32_t);
}

hipError_t launch_b_compact(const uint8_t* mask, int64_t p, int nprob, const uint8_t* want, int32_t* out,
                            int64_t* lens, void* scratch, hipStream_t st) {
    int64_t nblk = (p + CTILE - 1) / CTILE;
    if (nblk < 1) nblk = 1;
    int32_t* counts = (int32_t*)scratch;
    dim3 grid((unsigned)nblk, nprob);
    k_b_cmp_count<<<grid, CT, 0, st>>>(mask, p, want, counts, nblk);
    k_b_cmp_scan<<<nprob, 1024, 0, st>>>(counts, nblk, want, lens);
    k_b_cmp_write<<<grid, CT, 0, st>>>(mask, p, want, counts, nblk, out);
    return hipGetLastError();
}

hipError_t launch_b_pool_add(const int32_t* sets, const int64_t* lens, int64_t p, int nprob, const uint8_t* want,
                             int32_t* pool_pos, int32_t* pool_list, BatchScalars* bs, hipStream_t st) {
    k_b_pool_add<<<nprob, 1024, 0, st>>>(sets, lens, p, want, pool_pos, pool_list, bs);
    return hipGetLastError();
}

hipError_t launch_b_commit(int nprob, const uint8_t* want, BatchScalars* bs, hipStream_t st) {
    k_b_commit<<<1, BNP, 0, st>>>(nprob, want, bs);
    return hipGetLastError();
}

hipError_t launch_b_gram_update(const Mat& mt, const uint8_t* masks, int nprob, const int32_t* pool_list,
                                const BatchScalars* bs, const double* c, const double* s, double* Gp, int64_t cap,
                                int64_t max_P, int64_t max_N, const uint8_t* want, hipStream_t st) {
    if (max_N <= 0) return hipSuccess;
    dim3 grid((unsigned)((max_P + BG_K - 1) / BG_K), (unsigned)((max_N + BG_N - 1) / BG_N), nprob);
    const size_t es = mt.xtype == 0 ? 8 : 4;
    const bool vec = (uintptr_t)mt.X % 16 == 0 && (mt.ldx * (int64_t)es) % 16 == 0 && (uintptr_t)masks % 16 == 0 &&
                     mt.n_total % 16 == 0;
    if (mt.xtype == 0 && vec)
        k_b_gram_update<double, true><<<grid, 64 * BG_W, 0, st>>>((const double*)mt.X, mt.ldx, mt.n_total, masks, mt.p,
                                                                  pool_list, bs, c, s, Gp, cap, want);
    else if (mt.xtype == 0)
        k_b_gram_update<double, false><<<grid, 64 * BG_W, 0, st>>>((const double*)mt.X, mt.ldx, mt.n_total, masks, mt.p,
                                                                   pool_list, bs, c, s, Gp, cap, want);
    else if (vec)
        k_b_gram_update<float, true><<<grid, 64 * BG_W, 0, st>>>((const float*)mt.X, mt.ldx, mt.n_total, masks, mt.p,
                                                                 pool_list, bs, c, s, Gp, cap, want);
    else
        k_b_gram_update<float, false><<<grid, 64 * BG_W, 0, st>>>((const float*)mt.X, mt.ldx, mt.n_total, masks, mt.p,
                                                                  pool_list, bs, c, s, Gp, cap, want);
    return hipGetLastError();
}

hipError_t launch_b_gather(const int32_t* sets, const int64_t* lens, int64_t p, int nprob, const uint8_t* want,
                           const int32_t* pool_pos, const double* Gp, int64_t cap, const double* z, const double* beta,
                           double* GE, int64_t ge_stride, double* g0, double* b0, int64_t max_m, hipStream_t st) {
    dim3 grid(grid_for(max_m * max_m, 256, 2048), nprob);
    k_b_gather<<<grid, 256, 0, st>>>(sets, lens, p, want, pool_pos, Gp, cap, z, beta, GE, ge_stride, g0, b0);
    return hipGetLastError();
}

hipError_t launch_b_gcd(const int32_t* sets, const int64_t* lens, int64_t p, int nprob, const uint8_t* want,
                        const double* GE, int64_t ge_stride, const double* g0, const double* b0, double* b1,
                        double* beta, const double* lam, double tol, int max_sweeps, BatchScalars* bs,
                        hipStream_t st) {
    k_b_gcd<<<nprob, BCD_T, 0, st>>>(sets, lens, p, want, GE, ge_stride, g0, b0, b1, beta, lam, tol, max_sweeps, bs);
    return hipGetLastError();
}

hipError_t launch_b_r_update(const Mat& mt, const uint8_t* masks, const int32_t* sets, const int64_t* lens, int nprob,
                             const uint8_t* want, const double* b0, const double* b1, const double* c,
                             const double* s, double* R, hipStream_t st) {
    dim3 grid((unsigned)((mt.n_total + 255) / 256), nprob);
    if (mt.xtype == 0)
        k_b_r_update<double><<<grid, 256, 0, st>>>((const double*)mt.X, mt.ldx, mt.n_total, masks, sets, lens, mt.p,
                                                   want, b0, b1, c, s, R);
    else
        k_b_r_update<float><<<grid, 256, 0, st>>>((const float*)mt.X, mt.ldx, mt.n_total, masks, sets, lens, mt.p, want,
                                                  b0, b1, c, s, R);
    return hipGetLastError();
}

__global__ void k_b_kinc(int64_t* kdev) { *kdev += 1; }

hipError_t launch_b_kinc(int64_t* kdev, hipStream_t st) {
    k_b_kinc<<<1, 1, 0, st>>>(kdev);
    return hipGetLastError();
}

hipError_t launch_b_record(const int32_t* sets, const int64_t* lens, int64_t p, int nprob, const double* beta,
                           const double* c, const double* s, const BatchScalars* bs, const double* lam,
                           LamStats* out, int k, int K, const int64_t* n_safe, hipStream_t st) {
    k_b_record<<<nprob, 1024, 0, st>>>(sets, lens, p, beta, c, s, bs, lam, out, k, K, n_safe);
    return hipGetLastError();
}

}  // namespace blk
