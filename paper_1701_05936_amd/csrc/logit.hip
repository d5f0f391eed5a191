// Lasso-penalized logistic regression on the GPU path: the per-row work of the majorize-minimize solve.
// With f(eta) = log(1 + e^eta) - y eta and f'' <= 1/4, the loss at (b0, beta) is bounded above by its value
// at the current point plus (pi - y)'(eta' - eta)/n plus ||eta' - eta||^2/(8n).  Minimizing that bound plus
// lambda ||beta||_1 is a lasso on the residual 4 (y - pi) with threshold 4 lambda (unit curvature after
// the factor 4), which the covariance coordinate descent solves on its Gram pool; the kernels here form
// that residual, take the intercept's step, and move eta by what the solve changed.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace blk {

namespace {

constexpr int LT = 1024;

__device__ __forceinline__ bool fitted(const uint8_t* mask, int64_t i) { return mask == nullptr || mask[i] != 0; }

__device__ __forceinline__ double sigmoid(double e) {
    return e >= 0.0 ? 1.0 / (1.0 + exp(-e)) : exp(e) / (1.0 + exp(e));
}

__device__ __forceinline__ double log1pexp(double e) { return e > 0.0 ? e + log1p(exp(-e)) : log1p(exp(e)); }

// fixed-order sum over one workgroup of LT threads
__device__ double wg_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = LT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(LT) void k_logit_check_y(const uint8_t* __restrict__ mask, int64_t n_total,
                                                      const double* __restrict__ y, DevScalars* __restrict__ sc) {
    __shared__ double sh[LT];
    double ones = 0.0, bad = 0.0;
    for (int64_t i = threadIdx.x; i < n_total; i += LT)
        if (fitted(mask, i)) {
            const double v = y[i];
            ones += v == 1.0 ? 1.0 : 0.0;
            bad += (v == 0.0 || v == 1.0) ? 0.0 : 1.0;
        }
    const double t1 = wg_sum(ones, sh);
    const double tb = wg_sum(bad, sh);
    if (threadIdx.x == 0) {
        sc->lg_n1 = t1;
        sc->lg_bad = tb;
    }
}

__global__ void k_logit_init(const uint8_t* __restrict__ mask, int64_t n_total, double b0, double* __restrict__ eta,
                             DevScalars* __restrict__ sc) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_total; i += (int64_t)gridDim.x * blockDim.x)
        eta[i] = fitted(mask, i) ? b0 : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) sc->lg_b0 = b0;
}

__global__ void k_logit_resid(const uint8_t* __restrict__ mask, int64_t n_total, const double* __restrict__ y,
                              const double* __restrict__ eta, double* __restrict__ g, double* __restrict__ r0) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_total; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = fitted(mask, i) ? y[i] - sigmoid(eta[i]) : 0.0;
        g[i] = v;
        if (r0) r0[i] = 4.0 * v;
    }
}

__global__ void k_logit_center(const uint8_t* __restrict__ mask, int64_t n_total, double* __restrict__ r0,
                               double* __restrict__ r0c, DevScalars* __restrict__ sc) {
    const double db0 = sc->sum_r / (double)sc->n_rows;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_total; i += (int64_t)gridDim.x * blockDim.x) {
        const double v = fitted(mask, i) ? r0[i] - db0 : 0.0;
        r0[i] = v;
        r0c[i] = v;
    }
}

__global__ void k_logit_b0(DevScalars* __restrict__ sc) {
    const double db0 = sc->sum_r / (double)sc->n_rows;
    sc->lg_db0 = db0;
    sc->lg_b0 += db0;
}

__global__ void k_logit_eta(const uint8_t* __restrict__ mask, int64_t n_total, const double* __restrict__ r0c,
                            const double* __restrict__ r, double* __restrict__ eta, const DevScalars* __restrict__ sc) {
    const double db0 = sc->lg_db0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_total; i += (int64_t)gridDim.x * blockDim.x)
        if (fitted(mask, i)) eta[i] += db0 + (r0c[i] - r[i]);
}

__global__ __launch_bounds__(LT) void k_logit_loss(const uint8_t* __restrict__ mask, int64_t n_total,
                                                   const double* __restrict__ y, const double* __restrict__ eta,
                                                   DevScalars* __restrict__ sc) {
    __shared__ double sh[LT];
    double l = 0.0;
    for (int64_t i = threadIdx.x; i < n_total; i += LT)
        if (fitted(mask, i)) l += log1pexp(eta[i]) - y[i] * eta[i];
    const double t = wg_sum(l, sh);
    if (threadIdx.x == 0) {
        sc->rss = 2.0 * t;
        sc->y_mean = sc->lg_b0;
    }
}

int grid_of(int64_t n) {
    int64_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 2048) g = 2048;
    return (int)g;
}

}  // namespace

hipError_t launch_logit_check_y(const Mat& m, const double* y, DevScalars* sc, hipStream_t st) {
    k_logit_check_y<<<1, LT, 0, st>>>(m.mask, m.n_total, y, sc);
    return hipGetLastError();
}

hipError_t launch_logit_init(const Mat& m, double b0, double* eta, DevScalars* sc, hipStream_t st) {
    k_logit_init<<<grid_of(m.n_total), 256, 0, st>>>(m.mask, m.n_total, b0, eta, sc);
    return hipGetLastError();
}

hipError_t launch_logit_resid(const Mat& m, const double* y, const double* eta, double* g, double* r0, hipStream_t st) {
    k_logit_resid<<<grid_of(m.n_total), 256, 0, st>>>(m.mask, m.n_total, y, eta, g, r0);
    return hipGetLastError();
}

hipError_t launch_logit_center(const Mat& m, double* r0, double* r0c, DevScalars* sc, hipStream_t st) {
    k_logit_center<<<grid_of(m.n_total), 256, 0, st>>>(m.mask, m.n_total, r0, r0c, sc);
    k_logit_b0<<<1, 1, 0, st>>>(sc);
    return hipGetLastError();
}

hipError_t launch_logit_eta(const Mat& m, const double* r0c, const double* r, double* eta, const DevScalars* sc,
                            hipStream_t st) {
    k_logit_eta<<<grid_of(m.n_total), 256, 0, st>>>(m.mask, m.n_total, r0c, r, eta, sc);
    return hipGetLastError();
}

hipError_t launch_logit_loss(const Mat& m, const double* y, const double* eta, DevScalars* sc, hipStream_t st) {
    k_logit_loss<<<1, LT, 0, st>>>(m.mask, m.n_total, y, eta, sc);
    return hipGetLastError();
}

}  // namespace blk
