// Host side of the screening network: inference, loss + gradient, and Adam training with the steps of an
// epoch replayed from a captured HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "ctx.h"

using namespace blk;
using namespace blapi;

namespace {

constexpr int HIST_BINS = 4096;

uint64_t splitmix(uint64_t& s) {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

bl_status check_records(bl_ctx ctx, const float* feat, int64_t m, const float* params) {
    if (!feat || !params) return fail(ctx, BL_ERR_INVALID, "feat/params must be non-NULL");
    if (m < 1 || m >= ((int64_t)1 << 31)) return fail(ctx, BL_ERR_INVALID, "m must be in [1, 2^31)");
    return BL_OK;
}

}  // namespace

extern "C" {

bl_status bl_mlp_forward(bl_ctx ctx, const float* feat, int64_t m, const float* params, float* prob) {
    bl_status s = check_ctx(ctx);
    if (s) return s;
    if ((s = check_records(ctx, feat, m, params))) return s;
    if (!prob) return fail(ctx, BL_ERR_INVALID, "prob is NULL");
    HIPCHK(launch_mlp_fwd(feat, m, params, prob, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return BL_OK;
}

bl_status bl_mlp_loss_grad(bl_ctx ctx, const float* feat, const float* label, int64_t m, const float* params,
                           float* grad, double* loss) {
    bl_status s = check_ctx(ctx);
    if (s) return s;
    if ((s = check_records(ctx, feat, m, params))) return s;
    if (!label || !grad) return fail(ctx, BL_ERR_INVALID, "label/grad must be non-NULL");
    const int nblk = mlp_grad_blocks(m);
    float* part;
    double *lossp, *lossh;
    ENSURE(M_PART, (size_t)nblk * MLP_NPARAMS * 4, part);
    ENSURE(M_LOSSP, (size_t)nblk * 8, lossp);
    ENSURE(M_LOSSH, 8, lossh);
    hipStream_t st = ctx->stream;
    HIPCHK(launch_mlp_grad(feat, label, m, m, 1, nullptr, nullptr, params, part, lossp, st));
    HIPCHK(launch_mlp_adam(part, nblk, lossp, nullptr, nullptr, nullptr, nullptr, m, m, 1, 0.0, 0.0, 0.0, 0.0, 0, grad,
                           lossh, st));
    double L = 0.0;
    HIPCHK(hipMemcpyAsync(&L, lossh, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (loss) *loss = L;
    return BL_OK;
}

bl_status bl_mlp_train(bl_ctx ctx, const float* feat, const float* label, int64_t m, float* params,
                       const bl_mlp_train_opts* opts, bl_mlp_train_result* res) {
    const auto t0 = std::chrono::steady_clock::now();
    bl_status s = check_ctx(ctx);
    if (s) return s;
    if ((s = check_records(ctx, feat, m, params))) return s;
    if (!label || !opts || !res) return fail(ctx, BL_ERR_INVALID, "label/opts/res must be non-NULL");
    if (opts->epochs < 1 || opts->batch < 128 || opts->batch % 128 != 0)
        return fail(ctx, BL_ERR_INVALID, "epochs >= 1 and batch a positive multiple of 128 are required");
    if (!(opts->lr > 0.0) || !(opts->beta1 >= 0.0 && opts->beta1 < 1.0) || !(opts->beta2 >= 0.0 && opts->beta2 < 1.0) ||
        !(opts->eps > 0.0) || !(opts->target_recall > 0.0 && opts->target_recall <= 1.0))
        return fail(ctx, BL_ERR_INVALID, "lr > 0, 0 <= beta1, beta2 < 1, eps > 0, 0 < target_recall <= 1 required");
    const int64_t batch = std::min<int64_t>(opts->batch, (m + 127) / 128 * 128);
    const int64_t nb = (m + batch - 1) / batch;
    const int64_t total = nb * opts->epochs;
    const int nblk = mlp_grad_blocks(batch);
    float *part, *mom, *vel, *prob;
    double *lossp, *lossh;
    int64_t *step, *perm;
    uint32_t* hist;
    ENSURE(M_PART, (size_t)nblk * MLP_NPARAMS * 4, part);
    ENSURE(M_LOSSP, (size_t)nblk * 8, lossp);
    ENSURE(M_MOM, MLP_NPARAMS * 4, mom);
    ENSURE(M_VEL, MLP_NPARAMS * 4, vel);
    ENSURE(M_STEP, 8, step);
    ENSURE(M_PERM, (size_t)opts->epochs * 16, perm);
    ENSURE(M_LOSSH, (size_t)total * 8, lossh);
    ENSURE(M_PROB, (size_t)m * 4, prob);
    ENSURE(M_HIST, 2 * HIST_BINS * 4, hist);
    if (!ctx->aux) HIPCHK(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
    hipStream_t st = ctx->aux;
    HIPCHK(hipStreamSynchronize(ctx->stream));

    // record order of each epoch: t -> (a t + c) mod m with gcd(a, m) = 1 (a permutation of 0..m-1)
    std::vector<int64_t> hperm((size_t)opts->epochs * 2);
    uint64_t sd = opts->seed;
    for (int e = 0; e < opts->epochs; ++e) {
        int64_t a = 1;
        if (m > 2) {
            do {
                a = (int64_t)(splitmix(sd) % (uint64_t)(m - 1)) + 1;
            } while (std::gcd(a, m) != 1);
        }
        hperm[2 * e] = a;
        hperm[2 * e + 1] = (int64_t)(splitmix(sd) % (uint64_t)m);
    }
    HIPCHK(hipMemcpyAsync(perm, hperm.data(), hperm.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(step, 0, 8, st));
    HIPCHK(hipMemsetAsync(mom, 0, MLP_NPARAMS * 4, st));
    HIPCHK(hipMemsetAsync(vel, 0, MLP_NPARAMS * 4, st));
    HIPCHK(hipStreamSynchronize(st));

    auto one_step = [&]() -> hipError_t {
        hipError_t e = launch_mlp_grad(feat, label, m, batch, nb, perm, step, params, part, lossp, st);
        if (e == hipSuccess)
            e = launch_mlp_adam(part, nblk, lossp, params, mom, vel, step, m, batch, nb, opts->lr, opts->beta1,
                                opts->beta2, opts->eps, 1, nullptr, lossh, st);
        if (e == hipSuccess) e = launch_step_inc(step, st);
        return e;
    };
    // a graph of G consecutive steps (kernels read the step counter from device memory)
    const int64_t G = std::min<int64_t>(nb, 64);
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    hipError_t ce = hipSuccess;
    for (int64_t g = 0; g < G && ce == hipSuccess; ++g) ce = one_step();
    const hipError_t ee = hipStreamEndCapture(st, &graph);
    if (ce != hipSuccess || ee != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return fail(ctx, BL_ERR_DEVICE, "capturing the training steps: %s",
                    hipGetErrorString(ce != hipSuccess ? ce : ee));
    }
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipGraphDestroy(graph);
        return fail(ctx, BL_ERR_DEVICE, "hipGraphInstantiate failed");
    }
    bl_status out = BL_OK;
    int64_t done = 0;
    while (done + G <= total) {
        if (hipGraphLaunch(exec, st) != hipSuccess) {
            out = fail(ctx, BL_ERR_DEVICE, "hipGraphLaunch failed");
            break;
        }
        done += G;
    }
    while (out == BL_OK && done < total) {
        if (one_step() != hipSuccess) out = fail(ctx, BL_ERR_DEVICE, "training step launch failed");
        ++done;
    }
    (void)hipStreamSynchronize(st);
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    if (out != BL_OK) return out;

    // losses, then the threshold from the scores of the positive records
    std::vector<double> hl((size_t)total);
    HIPCHK(hipMemcpyAsync(hl.data(), lossh, hl.size() * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemsetAsync(hist, 0, 2 * HIST_BINS * 4, st));
    HIPCHK(launch_mlp_fwd(feat, m, params, prob, st));
    HIPCHK(launch_mlp_hist(prob, label, m, HIST_BINS, hist, st));
    std::vector<uint32_t> hh(2 * HIST_BINS);
    HIPCHK(hipMemcpyAsync(hh.data(), hist, hh.size() * 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    double first = 0.0, last = 0.0;
    for (int64_t t = 0; t < nb; ++t) {
        first += hl[(size_t)t];
        last += hl[(size_t)(total - nb + t)];
    }
    res->loss_first = first / (double)nb;
    res->loss_last = last / (double)nb;
    res->steps = total;
    const double npos = std::accumulate(hh.begin() + HIST_BINS, hh.end(), 0.0);
    const double nneg = std::accumulate(hh.begin(), hh.begin() + HIST_BINS, 0.0);
    int cut = 0;  // largest bin b with (positives in bins >= b) >= target * npos
    double cum = 0.0;
    for (int b = HIST_BINS - 1; b >= 0; --b) {
        cum += hh[HIST_BINS + b];
        if (npos > 0.0 && cum >= opts->target_recall * npos) {
            cut = b;
            break;
        }
    }
    double pos_above = 0.0, neg_above = 0.0;
    for (int b = cut; b < HIST_BINS; ++b) {
        pos_above += hh[HIST_BINS + b];
        neg_above += hh[b];
    }
    res->tau = (double)cut / HIST_BINS;
    res->recall = npos > 0.0 ? pos_above / npos : 1.0;
    res->neg_pass = nneg > 0.0 ? neg_above / nneg : 0.0;
    res->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return BL_OK;
}

}  // extern "C"
