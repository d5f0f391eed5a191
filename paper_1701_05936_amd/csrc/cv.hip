// Cross-validation (Section 3.1.2: the folds are row subsets of one X; Section 5.2: the cross-validation
// curve with its standard errors): fold masks, held-out predictions of every fold's path on the original
// scale, and the reductions of the squared errors into the curve and per-fold errors.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace blk {

namespace {

constexpr int PT = 256;    // threads per workgroup of the prediction (one held-out row each)
constexpr int CV_KT = 32;  // lambda values per prediction workgroup (accumulators per thread)
constexpr int CV_JT = 64;  // coefficients staged in LDS per step (CV_JT x CV_KT)

// masks[f][i] = row i is in fold f's fit (fold_i >= 0 and fold_i != f), test[f][i] = fold_i == f,
// Y[f][i] = y_i, all_rows[i] = fold_i >= 0
__global__ void k_cv_setup(const int32_t* __restrict__ fold, const double* __restrict__ y, int64_t n_total,
                           int nfolds, uint8_t* __restrict__ masks, uint8_t* __restrict__ test,
                           double* __restrict__ Y, uint8_t* __restrict__ all_rows) {
    const int f = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_total; i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t g = fold[i];
        const int64_t fi = (int64_t)f * n_total + i;
        masks[fi] = (g >= 0 && g != f) ? 1 : 0;
        test[fi] = g == f ? 1 : 0;
        Y[fi] = y[i];
        if (f == 0) all_rows[i] = g >= 0 ? 1 : 0;
    }
}

// mark[f][j] = beta of fold f is nonzero at some lambda (beta is [nfolds][K][p])
__global__ void k_cv_union(const double* __restrict__ beta, int64_t p, int K, uint8_t* __restrict__ mark) {
    const int f = blockIdx.y;
    const double* bf = beta + (int64_t)f * K * p;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < p; j += (int64_t)gridDim.x * blockDim.x) {
        uint8_t o = 0;
        for (int k = 0; k < K && !o; ++k) o = bf[(int64_t)k * p + j] != 0.0;
        mark[(int64_t)f * p + j] = o;
    }
}

template <typename XT>
__device__ __forceinline__ double ld_elem(const XT* p) { return (double)*p; }

// y^_i(lambda_k) = icpt[f][k] + sum_{j in U_f} x_ij beta[f][k][j] / s[f][j] for the held-out rows of fold f
// (rows[f][0..rlens[f])), lambda values k0 .. k0 + CV_KT - 1 (blockIdx.z); also the squared error.
// The coefficients of CV_JT columns are staged in LDS on the original scale; each thread accumulates its
// row's CV_KT predictions in the columns' list order.
template <typename XT>
__global__ __launch_bounds__(PT) void k_cv_predict(const XT* __restrict__ X, int64_t ldx, int64_t n_total, int64_t p,
                                                   int K, const double* __restrict__ beta, const double* __restrict__ s,
                                                   const int32_t* __restrict__ ulist, const int64_t* __restrict__ ulens,
                                                   const int32_t* __restrict__ rows,
                                                   const int64_t* __restrict__ rlens, const double* __restrict__ icpt,
                                                   const double* __restrict__ y, double* __restrict__ pred,
                                                   double* __restrict__ loss) {
    __shared__ double coef[CV_JT][CV_KT];
    __shared__ int32_t cj[CV_JT];
    const int f = blockIdx.y;
    const int k0 = blockIdx.z * CV_KT;
    const int kn = K - k0 < CV_KT ? K - k0 : CV_KT;
    const int64_t nr = rlens[f];
    const int64_t t = (int64_t)blockIdx.x * PT + threadIdx.x;
    if ((int64_t)blockIdx.x * PT >= nr) return;   // the whole workgroup is past this fold's rows
    const bool live = t < nr;
    const int64_t i = live ? rows[(int64_t)f * n_total + t] : 0;
    const int64_t nu = ulens[f];
    const int32_t* ul = ulist + (int64_t)f * p;
    const double* bf = beta + (int64_t)f * K * p;
    const double* sf = s + (int64_t)f * p;
    double acc[CV_KT];
#pragma unroll
    for (int kk = 0; kk < CV_KT; ++kk) acc[kk] = 0.0;
    for (int64_t j0 = 0; j0 < nu; j0 += CV_JT) {
        const int jn = nu - j0 < CV_JT ? (int)(nu - j0) : CV_JT;
        __syncthreads();
        for (int idx = threadIdx.x; idx < CV_JT * CV_KT; idx += PT) {
            const int jj = idx / CV_KT, kk = idx % CV_KT;
            double v = 0.0;
            if (jj < jn && kk < kn) {
                const int32_t j = ul[j0 + jj];
                v = bf[(int64_t)(k0 + kk) * p + j] / sf[j];
            }
            coef[jj][kk] = v;
        }
        if (threadIdx.x < CV_JT) cj[threadIdx.x] = threadIdx.x < jn ? ul[j0 + threadIdx.x] : 0;
        __syncthreads();
        if (live) {
            for (int jj = 0; jj < jn; ++jj) {
                const double x = ld_elem(X + (int64_t)cj[jj] * ldx + i);
#pragma unroll
                for (int kk = 0; kk < CV_KT; ++kk) acc[kk] = fma(x, coef[jj][kk], acc[kk]);
            }
        }
    }
    if (!live) return;
    const double yi = y[i];
#pragma unroll
    for (int kk = 0; kk < CV_KT; ++kk) {
        if (kk < kn) {
            const int k = k0 + kk;
            const double v = icpt[(int64_t)f * K + k] + acc[kk];
            const double e = yi - v;
            pred[(int64_t)k * n_total + i] = v;
            loss[(int64_t)k * n_total + i] = e * e;
        }
    }
}

// fixed-order workgroup sum of one value per thread
__device__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int w = PT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// curve at lambda k (one workgroup each): mean of the squared errors over the rows in a fold and the
// standard error of that mean (sample SD / sqrt(N)), two passes
__global__ __launch_bounds__(PT) void k_cv_curve(const double* __restrict__ loss, const uint8_t* __restrict__ all_rows,
                                                 int64_t n_total, double* __restrict__ cve, double* __restrict__ cvse) {
    __shared__ double sh[PT];
    const int k = blockIdx.x;
    const double* L = loss + (int64_t)k * n_total;
    double s = 0.0, cnt = 0.0;
    for (int64_t i = threadIdx.x; i < n_total; i += PT)
        if (all_rows[i]) {
            s += L[i];
            cnt += 1.0;
        }
    const double N = block_sum(cnt, sh);
    const double mean = block_sum(s, sh) / N;
    double q = 0.0;
    for (int64_t i = threadIdx.x; i < n_total; i += PT)
        if (all_rows[i]) {
            const double d = L[i] - mean;
            q = fma(d, d, q);
        }
    const double ss = block_sum(q, sh);
    if (threadIdx.x == 0) {
        cve[k] = mean;
        cvse[k] = N > 1.0 ? sqrt(ss / (N - 1.0)) / sqrt(N) : 0.0;
    }
}

// mean squared error of fold f at lambda k (workgroup (k, f)) over the fold's rows
__global__ __launch_bounds__(PT) void k_cv_fold_err(const double* __restrict__ loss, const int32_t* __restrict__ rows,
                                                    const int64_t* __restrict__ rlens, int64_t n_total, int K,
                                                    double* __restrict__ ferr) {
    __shared__ double sh[PT];
    const int k = blockIdx.x, f = blockIdx.y;
    const double* L = loss + (int64_t)k * n_total;
    const int64_t nr = rlens[f];
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < nr; t += PT) s += L[rows[(int64_t)f * n_total + t]];
    const double tot = block_sum(s, sh);
    if (threadIdx.x == 0) ferr[(int64_t)f * K + k] = nr > 0 ? tot / (double)nr : 0.0;
}

int grid_of(int64_t work, int per, int maxb) {
    int64_t g = (work + per - 1) / per;
    if (g < 1) g = 1;
    if (g > maxb) g = maxb;
    return (int)g;
}

template <typename XT>
hipError_t predict_typed(const Mat& m, int nfolds, int K, int64_t max_rows, const double* beta, const double* s,
                         const int32_t* ulist, const int64_t* ulens, const int32_t* rows, const int64_t* rlens,
                         const double* icpt, const double* y, double* pred, double* loss, hipStream_t st) {
    dim3 grid((unsigned)((max_rows + PT - 1) / PT), (unsigned)nfolds, (unsigned)((K + CV_KT - 1) / CV_KT));
    k_cv_predict<XT><<<grid, PT, 0, st>>>((const XT*)m.X, m.ldx, m.n_total, m.p, K, beta, s, ulist, ulens, rows, rlens,
                                          icpt, y, pred, loss);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_cv_setup(const int32_t* fold, const double* y, int64_t n_total, int nfolds, uint8_t* masks,
                           uint8_t* test, double* Y, uint8_t* all_rows, hipStream_t st) {
    dim3 grid(grid_of(n_total, 256, 1024), nfolds);
    k_cv_setup<<<grid, 256, 0, st>>>(fold, y, n_total, nfolds, masks, test, Y, all_rows);
    return hipGetLastError();
}

hipError_t launch_cv_union(const double* beta, int64_t p, int K, int nfolds, uint8_t* mark, hipStream_t st) {
    dim3 grid(grid_of(p, 256, 1024), nfolds);
    k_cv_union<<<grid, 256, 0, st>>>(beta, p, K, mark);
    return hipGetLastError();
}

hipError_t launch_cv_predict(const Mat& m, int nfolds, int K, int64_t max_rows, const double* beta, const double* s,
                             const int32_t* ulist, const int64_t* ulens, const int32_t* rows, const int64_t* rlens,
                             const double* icpt, const double* y, double* pred, double* loss, hipStream_t st) {
    if (max_rows <= 0 || K <= 0) return hipSuccess;
    switch (m.xtype) {
        case 0: return predict_typed<double>(m, nfolds, K, max_rows, beta, s, ulist, ulens, rows, rlens, icpt, y, pred,
                                             loss, st);
        case 1: return predict_typed<float>(m, nfolds, K, max_rows, beta, s, ulist, ulens, rows, rlens, icpt, y, pred,
                                            loss, st);
        default: return predict_typed<int8_t>(m, nfolds, K, max_rows, beta, s, ulist, ulens, rows, rlens, icpt, y,
                                              pred, loss, st);
    }
}

hipError_t launch_cv_reduce(const double* loss, const uint8_t* all_rows, const int32_t* rows, const int64_t* rlens,
                            int64_t n_total, int K, int nfolds, double* cve, double* cvse, double* ferr,
                            hipStream_t st) {
    k_cv_curve<<<K, PT, 0, st>>>(loss, all_rows, n_total, cve, cvse);
    k_cv_fold_err<<<dim3(K, nfolds), PT, 0, st>>>(loss, rows, rlens, n_total, K, ferr);
    return hipGetLastError();
}

}  // namespace blk
