// Host driver of K-fold cross-validation: the full-data path sets the grid, one batched call fits every
// fold on it (row masks, X shared), then the held-out predictions and their squared errors are reduced
// on the device into the cross-validation curve.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.h"

using namespace blk;
using namespace blapi;

extern "C" bl_status bl_cv_fit(bl_ctx ctx, const bl_matrix* X, const bl_cv* cv, const bl_path_opts* opts,
                               bl_cv_result* res) {
    const auto t_start = std::chrono::steady_clock::now();
    bl_status s = check_ctx(ctx);
    if (s) return s;
    Mat m;
    if ((s = check_matrix(ctx, X, &m))) return s;
    if (!cv || !opts || !res) return fail(ctx, BL_ERR_INVALID, "cv/opts/res must be non-NULL");
    res->k_done = 0;
    if (m.mask) return fail(ctx, BL_ERR_INVALID, "cross-validation chooses rows by fold (X->row_mask must be NULL)");
    if (m.xtype != BL_X_F64 && m.xtype != BL_X_F32)
        return fail(ctx, BL_ERR_UNSUPPORTED, "cross-validation: X must be f32 or f64 (the batched form)");
    const int F = cv->nfolds;
    if (F < 2 || F > BNP) return fail(ctx, BL_ERR_INVALID, "nfolds must be in 2..%d", BNP);
    if (!cv->fold || !cv->y) return fail(ctx, BL_ERR_INVALID, "fold and y must be non-NULL");
    const int K = opts->nlambda;
    if (K < 1) return fail(ctx, BL_ERR_INVALID, "nlambda must be >= 1");
    if (opts->rule == BL_SCREEN_LEARNED || opts->k_start != 0 || opts->precision != BL_PREC_FP64)
        return fail(ctx, BL_ERR_UNSUPPORTED, "cross-validation: no learned rule, resume or precision form");
    const int64_t nt = m.n_total, p = m.p;
    hipStream_t st = ctx->stream;

    // the folds, checked on the host
    std::vector<int32_t> hf(nt);
    HIPCHK(hipMemcpyAsync(hf.data(), cv->fold, nt * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    std::vector<int64_t> cnt(F, 0);
    int64_t N = 0;
    for (int64_t i = 0; i < nt; ++i) {
        const int32_t g = hf[i];
        if (g < -1 || g >= F) return fail(ctx, BL_ERR_INVALID, "fold[%lld] = %d outside -1..%d", (long long)i, g, F - 1);
        if (g >= 0) {
            ++cnt[g];
            ++N;
        }
    }
    for (int f = 0; f < F; ++f)
        if (cnt[f] == 0) return fail(ctx, BL_ERR_INVALID, "fold %d has no rows", f);
    const int64_t max_rows = *std::max_element(cnt.begin(), cnt.end());

    uint8_t *masks, *test, *all_rows, *mark, *want;
    double *Y, *fbeta, *pred, *loss, *icpt, *outv;
    int32_t *rows, *ulist;
    int64_t *rlens, *ulens;
    void* cmp;
    ENSURE(CV_MASKS, (size_t)F * nt, masks);
    ENSURE(CV_TEST, (size_t)F * nt, test);
    ENSURE(CV_Y, (size_t)F * nt * 8, Y);
    ENSURE(CV_ALL, (size_t)nt, all_rows);
    ENSURE(CV_ROWS, (size_t)F * nt * 4, rows);
    ENSURE(CV_RLENS, (size_t)BNP * 8, rlens);
    ENSURE(CV_MARK, (size_t)F * p, mark);
    ENSURE(CV_ULIST, (size_t)F * p * 4, ulist);
    ENSURE(CV_ULENS, (size_t)BNP * 8, ulens);
    ENSURE(CV_WANT, (size_t)BNP, want);
    ENSURE(CV_CMP, std::max(b_compact_scratch_bytes(p), b_compact_scratch_bytes(nt)), cmp);
    if (res->fold_beta) fbeta = res->fold_beta; else ENSURE(CV_FBETA, (size_t)F * K * p * 8, fbeta);
    if (res->pred) pred = res->pred; else ENSURE(CV_PRED, (size_t)K * nt * 8, pred);
    ENSURE(CV_LOSS, (size_t)K * nt * 8, loss);
    ENSURE(CV_ICPT, (size_t)F * K * 8, icpt);
    ENSURE(CV_OUT, (size_t)(2 + F) * K * 8, outv);
    HIPCHK(launch_cv_setup(cv->fold, cv->y, nt, F, masks, test, Y, all_rows, st));
    HIPCHK(launch_fill_u8(want, 0, BNP, st));
    HIPCHK(launch_fill_u8(want, 1, F, st));

    // the full-data path (rows in some fold) and its grid
    std::vector<double> lam(K);
    {
        bl_matrix Xa = *X;
        Xa.row_mask = all_rows;
        bl_path_opts o = *opts;
        o.r_out = nullptr;
        bl_path_result pr{};
        pr.beta = res->beta;
        pr.lambda = lam.data();
        s = bl_fit_path(ctx, &Xa, cv->y, &o, &pr);
        if (s) return s;
    }
    if (res->lambda) std::memcpy(res->lambda, lam.data(), K * sizeof(double));

    // every fold over that grid in one batched call
    std::vector<double> h_icpt((size_t)F * K);
    {
        bl_batch bt{};
        bt.nprob = F;
        bt.Y = Y;
        bt.masks = masks;
        bl_path_opts o = *opts;
        o.lambda = lam.data();
        o.r_out = nullptr;
        bl_batch_result br{};
        br.beta = fbeta;
        br.intercept = h_icpt.data();
        s = bl_fit_path_batch(ctx, X, &bt, &o, &br);
        if (s) return s;
        if (br.k_done != K) return fail(ctx, BL_ERR_NOT_CONVERGED, "fold paths stopped at lambda index %d", br.k_done);
    }
    // each fold's column scales stay in the batched call's scratch, problem-major [F x p]
    const double* fscale = (const double*)ctx->bufs[BB_S].p;
    HIPCHK(hipMemcpyAsync(icpt, h_icpt.data(), h_icpt.size() * 8, hipMemcpyHostToDevice, st));

    // held-out predictions over the columns each fold ever uses, and their squared errors
    HIPCHK(launch_cv_union(fbeta, p, K, F, mark, st));
    HIPCHK(launch_b_compact(mark, p, F, want, ulist, ulens, cmp, st));
    HIPCHK(launch_b_compact(test, nt, F, want, rows, rlens, cmp, st));
    HIPCHK(launch_fill_f64(pred, 0.0, (int64_t)K * nt, st));
    HIPCHK(launch_fill_f64(loss, 0.0, (int64_t)K * nt, st));
    HIPCHK(launch_cv_predict(m, F, K, max_rows, fbeta, fscale, ulist, ulens, rows, rlens, icpt, cv->y, pred, loss, st));
    HIPCHK(launch_cv_reduce(loss, all_rows, rows, rlens, nt, K, F, outv, outv + K, outv + 2 * K, st));
    std::vector<double> h((size_t)(2 + F) * K);
    HIPCHK(hipMemcpyAsync(h.data(), outv, h.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const double* cve = h.data();
    const double* cvse = h.data() + K;
    if (res->cve) std::memcpy(res->cve, cve, K * sizeof(double));
    if (res->cvse) std::memcpy(res->cvse, cvse, K * sizeof(double));
    if (res->fold_err) std::memcpy(res->fold_err, h.data() + 2 * K, (size_t)F * K * sizeof(double));
    // lambda.min: the first smallest error; the one-standard-error choice: the largest lambda whose error is
    // within one standard error of that minimum
    int kmin = 0;
    for (int k = 1; k < K; ++k)
        if (cve[k] < cve[kmin]) kmin = k;
    int k1 = kmin;
    for (int k = 0; k <= kmin; ++k)
        if (cve[k] <= cve[kmin] + cvse[kmin]) {
            k1 = k;
            break;
        }
    res->k_min = kmin;
    res->k_1se = k1;
    res->lambda_min = lam[kmin];
    res->lambda_1se = lam[k1];
    res->n_rows = N;
    res->k_done = K;
    res->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return BL_OK;
}
