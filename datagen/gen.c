/*
 * Seeded synthetic inputs for the lasso path (design matrices X).
 *
 * This module only draws random numbers; it holds none of the lasso
 * arithmetic.  Both the CPU oracle and the GPU library read what it writes.
 *
 * Random numbers come from a counter-based generator: every value is a pure
 * function of (seed, stream, counter), so any column can be regenerated on
 * its own and the output does not depend on the thread count.  The mixing
 * function is the SplitMix64 finalizer (Steele, Lea & Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014; constants as published by
 * Vigna for splitmix64.c).
 *
 * Streams: a stream id is (tag << 48) | index.  Tag 1 = column j of X,
 * tag 2 = per-column parameters (minor-allele frequency).
 */
#include <math.h>
#include <stdint.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL
#define TAG_XCOL 1ULL
#define TAG_COLPARAM 2ULL

static inline uint64_t mix64(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}

static inline uint64_t draw_u64(uint64_t seed, uint64_t stream, uint64_t ctr) {
    uint64_t key = mix64(seed + GOLDEN * (stream + 1ULL));
    return mix64(key + GOLDEN * (ctr + 1ULL));
}

/* uniform on the open interval (0, 1) with 53 random bits */
static inline double draw_unif(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return ((double)(draw_u64(seed, stream, ctr) >> 11) + 0.5) * 0x1.0p-53;
}

/* standard normal by the Box-Muller transform (cosine branch only) */
static inline double draw_normal(uint64_t seed, uint64_t stream, uint64_t ctr) {
    double u1 = draw_unif(seed, stream, 2 * ctr);
    double u2 = draw_unif(seed, stream, 2 * ctr + 1);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

static inline uint64_t stream_id(uint64_t tag, uint64_t idx) { return (tag << 48) | idx; }

/* exported for tests of the generator itself */
double dg_unif(uint64_t seed, uint64_t stream, uint64_t ctr) { return draw_unif(seed, stream, ctr); }
double dg_normal(uint64_t seed, uint64_t stream, uint64_t ctr) { return draw_normal(seed, stream, ctr); }

/* i.i.d. N(0,1) entries; columns j0 .. j0+p-1 of the full matrix, column-major with leading dim ld */
void dg_gaussian_f64(uint64_t seed, int64_t n, int64_t p, int64_t j0, double* X, int64_t ld) {
#pragma omp parallel for schedule(static)
    for (int64_t jj = 0; jj < p; ++jj) {
        uint64_t st = stream_id(TAG_XCOL, (uint64_t)(j0 + jj));
        double* col = X + jj * ld;
        for (int64_t i = 0; i < n; ++i) col[i] = draw_normal(seed, st, (uint64_t)i);
    }
}

/* per-column minor-allele frequencies, U(lo, hi) */
void dg_maf(uint64_t seed, int64_t p, int64_t j0, double lo, double hi, double* maf) {
#pragma omp parallel for schedule(static)
    for (int64_t jj = 0; jj < p; ++jj) {
        uint64_t st = stream_id(TAG_COLPARAM, (uint64_t)(j0 + jj));
        maf[jj] = lo + (hi - lo) * draw_unif(seed, st, 0);
    }
}

/* genotype codes x_ij ~ Binomial(2, maf_j): the sum of two Bernoulli(maf_j) draws */
void dg_genotype_u8(uint64_t seed, int64_t n, int64_t p, int64_t j0, const double* maf, uint8_t* X, int64_t ld) {
#pragma omp parallel for schedule(static)
    for (int64_t jj = 0; jj < p; ++jj) {
        uint64_t st = stream_id(TAG_XCOL, (uint64_t)(j0 + jj));
        double m = maf[jj];
        uint8_t* col = X + jj * ld;
        for (int64_t i = 0; i < n; ++i) {
            int a = draw_unif(seed, st, 2 * (uint64_t)i) < m;
            int b = draw_unif(seed, st, 2 * (uint64_t)i + 1) < m;
            col[i] = (uint8_t)(a + b);
        }
    }
}

/*
 * AR(1) correlation along the columns, stored as float32:
 *   x_{i,j} = e_{i,j}                                   at the first column of a block
 *   x_{i,j} = rho * x_{i,j-1} + sqrt(1-rho^2) * e_{i,j} otherwise
 * with e i.i.d. N(0,1).  block <= 0 means one block spanning all p columns.
 * The recursion runs in double and each value is rounded to float on store.
 * Parallel over row blocks, so the result does not depend on the thread count.
 */
void dg_ar1_f32(uint64_t seed, int64_t n, int64_t p, double rho, int64_t block, float* X, int64_t ld) {
    const int64_t RB = 256;
    const double w = sqrt(1.0 - rho * rho);
    int64_t nrb = (n + RB - 1) / RB;
#pragma omp parallel for schedule(static)
    for (int64_t rb = 0; rb < nrb; ++rb) {
        double prev[256];
        int64_t i0 = rb * RB;
        int64_t i1 = i0 + RB < n ? i0 + RB : n;
        for (int64_t j = 0; j < p; ++j) {
            uint64_t st = stream_id(TAG_XCOL, (uint64_t)j);
            int restart = (j == 0) || (block > 0 && (j % block) == 0);
            float* col = X + j * ld;
            for (int64_t i = i0; i < i1; ++i) {
                double e = draw_normal(seed, st, (uint64_t)i);
                double v = restart ? e : rho * prev[i - i0] + w * e;
                prev[i - i0] = v;
                col[i] = (float)v;
            }
        }
    }
}
