// Host driver of the batched form (bl_fit_path_batch): all problems advance through
// their lambda grids in lockstep; one host synchronization per CD + check round.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "ctx.h"

using namespace blk;
using namespace blapi;

namespace {

// distinct row masks up to which the column statistics take one pass of X per mask rather than the two mask
// scans on the matrix cores (a pass of the statistics kernel is HBM-bound; the two scans take about six of
// its passes with 64 problems)
constexpr int BATCH_STATS_PASSES = 4;

bl_status bpool_reserve(bl_ctx ctx, int nprob, int64_t need, const std::vector<int64_t>& sizes) {
    if (need <= ctx->bpool_cap && nprob <= ctx->bpool_np) return BL_OK;
    int64_t cap = need <= ctx->bpool_cap ? ctx->bpool_cap : std::max<int64_t>({need, ctx->bpool_cap * 2, 256});
    cap = (cap + 63) / 64 * 64;
    double* g = nullptr;
    if (hipMalloc(&g, (size_t)nprob * cap * cap * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, BL_ERR_NOMEM, "batched Gram pools of %lld features do not fit", (long long)cap);
    }
    for (int b = 0; b < nprob && b < ctx->bpool_np && ctx->bgpool; ++b) {
        if (sizes[b] <= 0) continue;
        const hipError_t e = hipMemcpy2DAsync(g + (size_t)b * cap * cap, cap * sizeof(double),
                                              ctx->bgpool + (size_t)b * ctx->bpool_cap * ctx->bpool_cap,
                                              ctx->bpool_cap * sizeof(double), sizes[b] * sizeof(double), sizes[b],
                                              hipMemcpyDeviceToDevice, ctx->stream);
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(ctx->stream);
            (void)hipFree(g);
            return fail(ctx, BL_ERR_DEVICE, "Gram pool copy: %s", hipGetErrorString(e));
        }
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (ctx->bgpool) (void)hipFree(ctx->bgpool);
    ctx->bgpool = g;
    ctx->bpool_cap = cap;
    ctx->bpool_np = nprob;
    return BL_OK;
}

// Pick the variant of the shared scan for this shape (workgroup width, register prefetch): time each
// candidate on up to 32,768 columns (raw products against the row masks) and keep the fastest.  Every candidate computes each
// column's products in the same order, so the choice never changes results.
// The tuning cache file named by the environment variable BL_AUTOTUNE_CACHE (when set): one line per shape,
// "bscan <arch> <xtype> <n_total> <p> <variant>"; a shape found there is not timed again, a new one is appended.
static std::string tune_key(bl_ctx ctx, const Mat& m) {
    hipDeviceProp_t prop{};
    std::string arch = hipGetDeviceProperties(&prop, ctx->device) == hipSuccess ? prop.gcnArchName : "unknown";
    for (char& ch : arch)
        if (ch == ' ') ch = '_';
    char buf[160];
    std::snprintf(buf, sizeof(buf), "bscan %s %d %lld %lld", arch.c_str(), m.xtype, (long long)m.n_total,
                  (long long)m.p);
    return buf;
}

static int tune_cache_lookup(const std::string& key) {
    const char* path = std::getenv("BL_AUTOTUNE_CACHE");
    if (!path || !*path) return -1;
    FILE* f = std::fopen(path, "r");
    if (!f) return -1;
    char line[256];
    int found = -1;
    while (std::fgets(line, sizeof(line), f)) {
        const size_t kl = key.size();
        if (std::strncmp(line, key.c_str(), kl) == 0 && line[kl] == ' ') {
            const int v = std::atoi(line + kl + 1);
            if (v >= 0 && v < BSCAN_VARIANTS) found = v;   // the last entry for the shape wins
        }
    }
    std::fclose(f);
    return found;
}

static void tune_cache_store(const std::string& key, int v) {
    const char* path = std::getenv("BL_AUTOTUNE_CACHE");
    if (!path || !*path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;   // the cache is an optimization: an unwritable file only costs the timing next time
    std::fprintf(f, "%s %d\n", key.c_str(), v);
    std::fclose(f);
}

bl_status tune_bscan(bl_ctx ctx, const Mat& m, const double* B, int nprob, BatchScalars* bs, double* part,
                     double* out) {
    if (ctx->bscan_n == m.n_total && ctx->bscan_p == m.p && ctx->bscan_x == m.xtype) return BL_OK;
    const std::string key = tune_key(ctx, m);
    const int cached = tune_cache_lookup(key);
    if (cached >= 0) {
        ctx->bscan_n = m.n_total;
        ctx->bscan_p = m.p;
        ctx->bscan_x = m.xtype;
        ctx->bscan_waves = cached;
        return BL_OK;
    }
    hipStream_t st = ctx->stream;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(ctx, BL_ERR_DEVICE, "hipEventCreate failed");
    }
    const int64_t cols = m.p < 32768 ? m.p : 32768;
    float best = 1e30f;
    int pick = 1;
    bl_status s = BL_OK;
    for (int w = 0; w < BSCAN_VARIANTS; ++w) {
        hipError_t e = launch_bscan(m, 0, nullptr, nullptr, cols, B, nprob, bs, nullptr, nullptr, nullptr, part, out, st, w);
        if (e == hipSuccess) e = hipEventRecord(e0, st);
        for (int r = 0; r < 2 && e == hipSuccess; ++r)
            e = launch_bscan(m, 0, nullptr, nullptr, cols, B, nprob, bs, nullptr, nullptr, nullptr, part, out, st, w);
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            s = fail(ctx, BL_ERR_DEVICE, "scan tuning: %s", hipGetErrorString(e));
            break;
        }
        if (ms < best) {
            best = ms;
            pick = w;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != BL_OK) return s;
    ctx->bscan_n = m.n_total;
    ctx->bscan_p = m.p;
    ctx->bscan_x = m.xtype;
    ctx->bscan_waves = pick;
    tune_cache_store(key, pick);
    return BL_OK;
}

struct GraphSet {
    hipGraphExec_t x[2] = {nullptr, nullptr};
    ~GraphSet() {
        for (auto& g : x)
            if (g) (void)hipGraphExecDestroy(g);
    }
};

}  // namespace

extern "C" bl_status bl_fit_path_batch(bl_ctx ctx, const bl_matrix* X, const bl_batch* bt, const bl_path_opts* opts,
                                       bl_batch_result* res) {
    const auto t_start = std::chrono::steady_clock::now();
    bl_status s = check_ctx(ctx);
    if (s) return s;
    Mat m;
    if ((s = check_matrix(ctx, X, &m))) return s;
    if (!bt || !opts || !res) return fail(ctx, BL_ERR_INVALID, "batch/opts/res must be non-NULL");
    res->k_done = 0;
    if (m.mask) return fail(ctx, BL_ERR_INVALID, "batched form: rows are chosen per problem (X->row_mask must be NULL)");
    if (m.xtype != BL_X_F64 && m.xtype != BL_X_F32) return fail(ctx, BL_ERR_UNSUPPORTED, "batched form: X must be f32 or f64");
    const int NB = bt->nprob;
    if (NB < 1 || NB > BNP) return fail(ctx, BL_ERR_INVALID, "nprob must be in 1..%d", BNP);
    if (!bt->Y) return fail(ctx, BL_ERR_INVALID, "Y is NULL");
    const int K = opts->nlambda;
    if (K < 1) return fail(ctx, BL_ERR_INVALID, "nlambda must be >= 1");
    const bool user_grid = opts->lambda != nullptr;   // one grid shared by every problem (cross-validation)
    if (user_grid) {
        for (int k = 0; k < K; ++k) {
            if (!(std::isfinite(opts->lambda[k]) && opts->lambda[k] > 0.0))
                return fail(ctx, BL_ERR_INVALID, "user lambda[%d] must be finite and > 0", k);
            if (k > 0 && !(opts->lambda[k] <= opts->lambda[k - 1]))
                return fail(ctx, BL_ERR_INVALID, "user lambda must be non-increasing");
        }
    } else if (K > 1 && !(opts->lambda_min_ratio > 0.0 && opts->lambda_min_ratio < 1.0)) {
        return fail(ctx, BL_ERR_INVALID, "lambda_min_ratio must be in (0, 1)");
    }
    if (opts->rule < BL_SCREEN_NONE || opts->rule > BL_SCREEN_ACTIVE) return fail(ctx, BL_ERR_INVALID, "unknown rule");
    if (opts->rule == BL_SCREEN_LEARNED) return fail(ctx, BL_ERR_UNSUPPORTED, "batched form: no learned rule");
    if (opts->k_start != 0) return fail(ctx, BL_ERR_UNSUPPORTED, "batched form: no resume (k_start must be 0)");
    if ((opts->alpha != 0.0 && opts->alpha != 1.0) || opts->penalty_factor)
        return fail(ctx, BL_ERR_UNSUPPORTED, "batched form: lasso only (no elastic net or penalty factors)");
    if (!(opts->tol > 0.0) || opts->max_sweeps < 1 || opts->max_rounds < 1)
        return fail(ctx, BL_ERR_INVALID, "tol > 0, max_sweeps >= 1 and max_rounds >= 1 are required");
    // check scans: FP64 matrix cores, or (f32 X) BF16 matrix cores with FP64 re-scans of the decisions in the band
    const bool bf = opts->precision == BL_PREC_BF16X3 || opts->precision == BL_PREC_BF16X2;
    const int pieces = opts->precision == BL_PREC_BF16X2 ? 2 : 3;
    if (opts->precision != BL_PREC_FP64 && !(bf && m.xtype == BL_X_F32))
        return fail(ctx, BL_ERR_UNSUPPORTED, "batched form: FP64 scans, or BF16X3 / BF16X2 scans of f32 X");
    // the active-set rule keeps only the previous active set: the strong rule with an infinite threshold
    const bool active_only = opts->rule == BL_SCREEN_ACTIVE;
    const bool bedpp = opts->rule == BL_SCREEN_BEDPP || opts->rule == BL_SCREEN_SSR_BEDPP || active_only;
    const bool ssr = opts->rule == BL_SCREEN_SSR || opts->rule == BL_SCREEN_SSR_BEDPP || active_only;
    const int64_t p = m.p, nt = m.n_total, npad = batch_pad(nt);
    const double es = (double)elem_bytes(m.xtype);
    hipStream_t st = ctx->stream;

    uint8_t *masks, *keep, *safe, *safen, *strong, *uni, *want, *want_all;
    double *Mb, *Yt, *R, *Bm, *S1, *S2, *c, *sd, *a, *bb, *z0, *z1, *lamg, *thrg, *beta, *g0, *b0, *b1, *GE = nullptr;
    int32_t *lT, *lE, *pos, *list, *lsafe;
    int64_t *lens, *lenT, *safecnt;
    BatchScalars* bs;
    LamStats* stats;
    void* cmp;
    const size_t P8 = (size_t)NB * p * 8, P1 = (size_t)NB * p, P4 = (size_t)NB * p * 4, RB = (size_t)npad * BNP * 8;
    if (bt->masks) masks = const_cast<uint8_t*>(bt->masks);
    else ENSURE(BB_MASKS, (size_t)NB * nt, masks);
    ENSURE(BB_MB, RB, Mb);
    ENSURE(BB_YT, RB, Yt);
    ENSURE(BB_R, RB, R);
    ENSURE(BB_B, RB, Bm);
    ENSURE(BB_S1, P8, S1);
    ENSURE(BB_S2, P8, S2);
    ENSURE(BB_C, P8, c);
    ENSURE(BB_S, P8, sd);
    ENSURE(BB_KEEP, P1, keep);
    ENSURE(BB_A, P8, a);
    ENSURE(BB_BB, P8, bb);
    ENSURE(BB_Z0, P8, z0);
    ENSURE(BB_Z1, P8, z1);
    ENSURE(BB_SAFE, P1, safe);
    ENSURE(BB_SAFEN, P1, safen);
    ENSURE(BB_STRONG, P1, strong);
    ENSURE(BB_UNION, p, uni);
    ENSURE(BB_LT, p * 4, lT);
    ENSURE(BB_LE, P4, lE);
    ENSURE(BB_LENS, (BNP + 8) * 8, lens);
    lenT = lens + BNP;
    ENSURE(BB_SAFECNT, BNP * 8, safecnt);
    ENSURE(BB_LSAFE, P4, lsafe);
    ENSURE(BB_LAM, (size_t)(K + 1) * BNP * 8, lamg);   // lamg[k*BNP + b] = lambda_k of problem b
    ENSURE(BB_THR, (size_t)K * BNP * 8, thrg);         // strong-rule thresholds 2 lambda_k - lambda_{k-1}
    ENSURE(BB_WANT, BNP, want);
    ENSURE(BB_WANTALL, BNP, want_all);
    ENSURE(BB_BS, BNP * sizeof(BatchScalars), bs);
    ENSURE(BB_BETA, P8, beta);
    ENSURE(BB_POS, P4, pos);
    ENSURE(BB_LIST, P4, list);
    ENSURE(BB_G0, P8, g0);
    ENSURE(BB_B0, P8, b0);
    ENSURE(BB_B1, P8, b1);
    ENSURE(BB_STATS, (size_t)NB * K * sizeof(LamStats), stats);
    ENSURE(BB_CMP, std::max(b_compact_scratch_bytes(p), compact_scratch_bytes(p)), cmp);
    double* bspart;   // rows of the shared scans' cut tiles
    ENSURE(BB_BSPART, bscan_part_bytes(), bspart);
    int64_t* kdev;   // lambda step counter read by the replayed screening graph
    ENSURE(BB_KDEV, 8, kdev);
    __bf16* Rp = nullptr;
    double* bfpart = nullptr;
    uint8_t* flag = nullptr;
    int32_t *lF = nullptr, *lU = nullptr;
    int64_t* lenF = lens + BNP + 2;
    int64_t* lenU = lens + BNP + 3;
    const double bf_rel = bf ? bscan_bf16_rel(nt, pieces) : 0.0;
    ENSURE(BB_LU, p * 4, lU);
    if (bf) {
        ENSURE(BB_RP, (size_t)bscan_bf16_pieces_bytes(nt, pieces), Rp);
        ENSURE(BB_BFPART, bscan_bf16_part_bytes(pieces), bfpart);
        ENSURE(BB_FLAG, p, flag);
        ENSURE(BB_LF, p * 4, lF);
    }

    // pinned host staging: every write to it is followed by a stream synchronization before the next one
    struct Pinned {
        uint8_t want[BNP];
        int64_t lens[BNP];
        int64_t lenT;
        int64_t lenF, lenU;   // BF16 form: flagged columns re-scanned, working-set union scanned exactly
        BatchScalars bs[BNP];
    };
    if (!ctx->bpinned && hipHostMalloc(&ctx->bpinned, sizeof(Pinned), hipHostMallocDefault) != hipSuccess) {
        ctx->bpinned = nullptr;
        (void)hipGetLastError();
        return fail(ctx, BL_ERR_NOMEM, "pinned staging allocation failed");
    }
    Pinned* hp = (Pinned*)ctx->bpinned;
    auto read_bs = [&]() -> bl_status {
        HIPCHK(hipMemcpyAsync(hp->bs, bs, NB * sizeof(BatchScalars), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        return BL_OK;
    };

    // ---- set-up: row masks, per-problem standardization, lambda_max, BEDPP inputs ----
    HIPCHK(hipMemsetAsync(bs, 0, BNP * sizeof(BatchScalars), st));
    HIPCHK(hipMemsetAsync(Yt, 0, RB, st));
    HIPCHK(hipMemsetAsync(R, 0, RB, st));
    HIPCHK(hipMemsetAsync(Bm, 0, RB, st));
    HIPCHK(hipMemsetAsync(want_all, 0, BNP, st));
    HIPCHK(launch_fill_u8(want_all, 1, NB, st));
    if (!bt->masks) HIPCHK(launch_fill_u8(masks, 1, (int64_t)NB * nt, st));
    HIPCHK(launch_b_masks(masks, nt, NB, Mb, st));
    HIPCHK(launch_b_center_y(masks, bt->Y, nt, NB, Yt, R, bs, st));
    if ((s = tune_bscan(ctx, m, Mb, NB, bs, bspart, S1))) return s;
    const int waves = ctx->bscan_waves;   // the variant picked for this shape
    res->scan_cols = bscan_variant_cols(waves);
    // Centers and scales depend on a problem's rows alone, so problems with the same mask (the responses of
    // one cross-validation fold) share them.  With few distinct masks each takes one pass of the column
    // statistics kernel and the other problems copy its results; otherwise the two mask scans X'M and
    // (X o X)'M run on the matrix cores for every problem at once.
    std::vector<int> rep(NB);
    std::vector<int64_t> rows(NB, nt);
    int U = 0;
    {
        std::vector<uint8_t> hm(bt->masks ? (size_t)NB * nt : 0);
        if (bt->masks) {
            HIPCHK(hipMemcpyAsync(hm.data(), masks, hm.size(), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
        }
        for (int b = 0; b < NB; ++b) {
            rep[b] = b;
            for (int u = 0; u < b && bt->masks; ++u)
                if (rep[u] == u && std::memcmp(&hm[(size_t)u * nt], &hm[(size_t)b * nt], (size_t)nt) == 0) {
                    rep[b] = u;
                    break;
                }
            if (!bt->masks && b > 0) rep[b] = 0;
            if (rep[b] != b) continue;
            ++U;
            if (bt->masks)
                rows[b] = nt - std::count(hm.begin() + (size_t)b * nt, hm.begin() + (size_t)(b + 1) * nt, (uint8_t)0);
        }
    }
    const bool by_mask = U <= BATCH_STATS_PASSES;
    prof_mark(ctx, 0);
    if (by_mask) {
        for (int b = 0; b < NB; ++b) {
            if (rep[b] != b) continue;
            Mat mb = m;
            mb.mask = bt->masks ? masks + (size_t)b * nt : nullptr;
            HIPCHK(launch_colstats(mb, c + (size_t)b * p, sd + (size_t)b * p, keep + (size_t)b * p, rows[b], st));
        }
    } else {
        HIPCHK(launch_bscan(m, 0, nullptr, nullptr, p, Mb, NB, bs, nullptr, nullptr, nullptr, bspart, S1, st, waves));
        HIPCHK(launch_bscan(m, 1, nullptr, nullptr, p, Mb, NB, bs, nullptr, nullptr, nullptr, bspart, S2, st, waves));
    }
    prof_mark(ctx, 1);
    if (by_mask) {
        for (int b = 0; b < NB; ++b) {
            if (rep[b] == b) continue;
            const size_t o = (size_t)b * p, ou = (size_t)rep[b] * p;
            HIPCHK(hipMemcpyAsync(c + o, c + ou, (size_t)p * 8, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(sd + o, sd + ou, (size_t)p * 8, hipMemcpyDeviceToDevice, st));
            HIPCHK(hipMemcpyAsync(keep + o, keep + ou, (size_t)p, hipMemcpyDeviceToDevice, st));
        }
    } else {
        HIPCHK(launch_b_stats(S1, S2, p, NB, bs, c, sd, keep, st));
    }
    HIPCHK(launch_b_sum_r(R, nt, NB, bs, st));
    prof_mark(ctx, 2);
    HIPCHK(launch_bscan(m, 2, nullptr, nullptr, p, Yt, NB, bs, c, sd, keep, bspart, a, st, waves));
    prof_mark(ctx, 3);
    HIPCHK(launch_b_argmax(a, keep, p, NB, bs, st));
    if ((s = read_bs())) return s;
    prof_add(ctx, 0, BL_PROF_COLSTATS, (by_mask ? (double)U : 2.0) * p * nt * es);
    prof_add(ctx, 2, BL_PROF_SETUP, (double)p * nt * es + (double)nt * NB * 8.0, 2.0 * p * nt * NB, (double)p);
    std::vector<double> lmax(NB);
    for (int b = 0; b < NB; ++b) {
        const BatchScalars& h = hp->bs[b];
        if (h.n_rows < 1) return fail(ctx, BL_ERR_INVALID, "problem %d: its mask selects no rows", b);
        if (!std::isfinite(h.y_mean) || !std::isfinite(h.yy)) return fail(ctx, BL_ERR_INVALID, "problem %d: y has NaN or Inf", b);
        if (h.jstar < 0) return fail(ctx, BL_ERR_INVALID, "problem %d: no column is kept (all constant)", b);
        if (!std::isfinite(h.lmax)) return fail(ctx, BL_ERR_INVALID, "problem %d: X or y has NaN or Inf", b);
        if (!(h.lmax > 0.0)) return fail(ctx, BL_ERR_INVALID, "problem %d: lambda_max is 0 (y constant on its rows)", b);
        lmax[b] = h.lmax;
    }
    if (bedpp) {
        HIPCHK(launch_b_std_column(m, masks, NB, bs, c, sd, Bm, st));
        HIPCHK(launch_b_sum_r(Bm, nt, NB, bs, st));   // the mode-2 scan subtracts c_j * (sum of the right-hand side)
        prof_mark(ctx, 2);
        HIPCHK(launch_bscan(m, 2, nullptr, nullptr, p, Bm, NB, bs, c, sd, keep, bspart, bb, st, waves));
        prof_mark(ctx, 3);
        HIPCHK(launch_b_sum_r(R, nt, NB, bs, st));    // back to the residual's sum and ||y~||^2
        HIPCHK(hipStreamSynchronize(st));
        prof_add(ctx, 2, BL_PROF_SETUP, (double)p * nt * es + (double)nt * NB * 8.0, 2.0 * p * nt * NB, (double)p);
    }
    // lambda grids (own lambda_max per problem) and strong-rule thresholds, resident on the device
    std::vector<double> lam((size_t)NB * K), lg((size_t)(K + 1) * BNP, 0.0), tg((size_t)K * BNP, 0.0);
    for (int b = 0; b < NB; ++b)
        for (int k = 0; k < K; ++k)
            lam[(size_t)b * K + k] = user_grid ? opts->lambda[k]
                                   : (K == 1 ? lmax[b] : lmax[b] * std::pow(opts->lambda_min_ratio, (double)k / (K - 1)));
    for (int k = 0; k <= K; ++k)   // row K repeats row K-1: the last step's "next" safe set is its own
        for (int b = 0; b < NB; ++b) {
            lg[(size_t)k * BNP + b] = lam[(size_t)b * K + (k < K ? k : K - 1)];
            if (k == K) continue;
            // the strong rule's previous lambda before the grid's first point is lambda_max (z there is a)
            tg[(size_t)k * BNP + b] = active_only ? INFINITY
                                      : 2.0 * lam[(size_t)b * K + k] - (k > 0 ? lam[(size_t)b * K + k - 1] : lmax[b]);
        }
    HIPCHK(hipMemcpyAsync(lamg, lg.data(), lg.size() * 8, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(thrg, tg.data(), tg.size() * 8, hipMemcpyHostToDevice, st));
    if (res->lambda) std::memcpy(res->lambda, lam.data(), lam.size() * sizeof(double));

    HIPCHK(launch_fill_f64(beta, 0.0, (int64_t)NB * p, st));
    HIPCHK(launch_fill_u8((uint8_t*)pos, 0xff, (int64_t)P4, st));
    HIPCHK(hipMemsetAsync(lens, 0, (BNP + 8) * 8, st));
    std::vector<int64_t> pool_size(NB, 0);
    std::vector<int32_t> h_sweeps((size_t)NB * K, 0), h_rounds((size_t)NB * K, 0);
    std::vector<int64_t> h_viol((size_t)NB * K, 0);
    int64_t ge_cap = 0;  // per-problem stride of the working-set Gram buffer (elements)
    // z of every problem at its previous lambda: at step k it is in z1 for odd k, z0 for even k.  With the
    // grid from each problem's lambda_max the path starts at step 1 from z = a (copied to z1); a shared
    // user grid starts at step 0 (beta = 0 for problems whose lambda_max is at most lambda_0), z = a in z0
    const int k_first = user_grid ? 0 : 1;
    double* zprev = k_first ? z1 : z0;
    double* zcur = k_first ? z0 : z1;
    HIPCHK(hipMemcpyAsync(zprev, a, P8, hipMemcpyDeviceToDevice, st));
    bl_status final_status = BL_OK;

    // Screening of a lambda step: S_k per problem and its size, the scan list (union over problems of
    // S_{k+1}; of S_k at the last step, whose row K of the grid repeats K-1) and the working sets E_k.
    // With kd the step comes from the device counter (graph replays), otherwise from k.
    auto screen_step = [&](hipStream_t s2, const int64_t* kd, int k, const double* zp) -> hipError_t {
        const int ko = kd ? 0 : k;
        hipError_t e = launch_b_bedpp(p, NB, a, bb, keep, bedpp, bs, lamg, ko, kd, safe, s2);
        if (e == hipSuccess) e = launch_b_compact(safe, p, NB, want_all, lsafe, safecnt, cmp, s2);
        if (e == hipSuccess) e = launch_b_bedpp(p, NB, a, bb, keep, bedpp, bs, lamg, ko + 1, kd, safen, s2);
        if (e == hipSuccess) e = launch_b_union(p, NB, safen, uni, s2);
        if (e == hipSuccess) e = launch_compact(uni, p, lT, lenT, cmp, s2);
        if (e == hipSuccess) e = launch_b_ssr(p, NB, safe, beta, zp, ssr, thrg, ko, kd, want_all, strong, s2);
        if (e == hipSuccess) e = launch_b_compact(strong, p, NB, want_all, lE, lens, cmp, s2);
        return e;
    };
    GraphSet graphs;
    const bool use_graph = !(bt->flags & BL_BATCH_EAGER) && K > 2;
    if (use_graph) {
        if (!ctx->aux) HIPCHK(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
        for (int par = 0; par < 2; ++par) {
            hipGraph_t g = nullptr;
            HIPCHK(hipStreamBeginCapture(ctx->aux, hipStreamCaptureModeThreadLocal));
            const hipError_t ce = screen_step(ctx->aux, kdev, 0, par ? z1 : z0);
            const hipError_t ee = hipStreamEndCapture(ctx->aux, &g);
            hipError_t ie = hipSuccess;
            if (ce == hipSuccess && ee == hipSuccess) ie = hipGraphInstantiate(&graphs.x[par], g, nullptr, nullptr, 0);
            if (g) (void)hipGraphDestroy(g);
            if (ce != hipSuccess || ee != hipSuccess || ie != hipSuccess) {
                (void)hipGetLastError();
                return fail(ctx, BL_ERR_DEVICE, "capturing the screening step: %s",
                            hipGetErrorString(ce != hipSuccess ? ce : (ee != hipSuccess ? ee : ie)));
            }
        }
    }
    HIPCHK(hipMemsetAsync(kdev, 0, 8, st));
    if (k_first == 1) {
        HIPCHK(launch_b_kinc(kdev, st));   // the counter holds the step being screened: 1
        // lambda index 0 is lambda_max of every problem: beta = 0
        HIPCHK(launch_b_bedpp(p, NB, a, bb, keep, bedpp, bs, lamg, 0, nullptr, safe, st));
        HIPCHK(launch_b_compact(safe, p, NB, want_all, lsafe, safecnt, cmp, st));
        HIPCHK(launch_b_record(lE, lens, p, NB, beta, c, sd, bs, lamg, stats, 0, K, safecnt, st));
        if (res->beta)
            HIPCHK(hipMemcpy2DAsync(res->beta, (size_t)K * p * 8, beta, p * 8, p * 8, NB, hipMemcpyDeviceToDevice, st));
        res->k_done = 1;
    }

    for (int k = k_first; k < K; ++k) {
        const double* lam_k = lamg + (size_t)k * BNP;
        if (use_graph) HIPCHK(hipGraphLaunch(graphs.x[k & 1], st));
        else HIPCHK(screen_step(st, nullptr, k, zprev));
        std::vector<uint8_t> act(NB, 1);
        std::vector<int> rounds(NB, 0);
        const uint8_t* wv = want_all;
        for (int it = 0;; ++it) {
            // working-set sizes and new pool members of the problems still solving
            HIPCHK(hipMemcpyAsync(hp->lens, lens, NB * 8, hipMemcpyDeviceToHost, st));
            HIPCHK(launch_b_pool_add(lE, lens, p, NB, wv, pos, list, bs, st));
            if ((s = read_bs())) return s;
            int64_t max_m = 0, max_P = 0, max_N = 0;
            for (int b = 0; b < NB; ++b) {
                if (!act[b]) continue;
                if (hp->lens[b] > BCD_MAX)
                    return fail(ctx, BL_ERR_UNSUPPORTED, "problem %d: working set of %lld features exceeds %d", b,
                                (long long)hp->lens[b], BCD_MAX);
                max_m = std::max(max_m, hp->lens[b]);
                max_P = std::max(max_P, pool_size[b] + hp->bs[b].n_new);
                max_N = std::max(max_N, hp->bs[b].n_new);
            }
            if ((s = bpool_reserve(ctx, NB, max_P, pool_size))) return s;
            prof_mark(ctx, 4);
            HIPCHK(launch_b_gram_update(m, masks, NB, list, bs, c, sd, ctx->bgpool, ctx->bpool_cap, max_P, max_N, wv, st));
            HIPCHK(launch_b_commit(NB, wv, bs, st));
            prof_mark(ctx, 5);
            for (int b = 0; b < NB; ++b)
                if (act[b]) pool_size[b] += hp->bs[b].n_new;
            if (max_m * max_m > ge_cap) ge_cap = std::max<int64_t>(max_m * max_m, 2 * ge_cap);
            ENSURE(BB_GE, (size_t)NB * std::max<int64_t>(ge_cap, 1) * 8, GE);
            {
                // every solve starts from FP64 gradients of its working set taken by one scan of the union of the
                // working sets, split over row ranges (a short list): the same values whichever form the check
                // scans take, so the BF16 form's solves see the FP64 form's inputs
                HIPCHK(launch_b_union(p, NB, strong, uni, st));
                HIPCHK(launch_compact(uni, p, lU, lenU, cmp, st));
                HIPCHK(hipMemcpyAsync(&hp->lenU, lenU, 8, hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                double* part;
                ENSURE(BB_PART, bscan_split_part_bytes(nt, hp->lenU), part);
                prof_mark(ctx, 8);
                HIPCHK(launch_bscan_split(m, lU, hp->lenU, R, NB, bs, c, sd, keep, part, it == 0 ? zprev : zcur, st));
                prof_mark(ctx, 9);
            }
            HIPCHK(launch_b_gather(lE, lens, p, NB, wv, pos, ctx->bgpool, ctx->bpool_cap, it == 0 ? zprev : zcur, beta,
                                   GE, ge_cap, g0, b0, max_m, st));
            prof_mark(ctx, 6);
            HIPCHK(launch_b_gcd(lE, lens, p, NB, wv, GE, ge_cap, g0, b0, b1, beta, lam_k, opts->tol, opts->max_sweeps, bs,
                                st));
            prof_mark(ctx, 7);
            HIPCHK(launch_b_r_update(m, masks, lE, lens, NB, wv, b0, b1, c, sd, R, st));
            HIPCHK(launch_b_sum_r(R, nt, NB, bs, st));
            // post-convergence scan of every problem over the union list, then each problem's check
            if (!bf) {
                prof_mark(ctx, 2);
                HIPCHK(launch_bscan(m, 2, lT, lenT, 0, R, NB, bs, c, sd, keep, bspart, zcur, st, waves));
                prof_mark(ctx, 3);
            } else {
                HIPCHK(launch_b_r_pieces(R, nt, NB, pieces, Rp, st));
                prof_mark(ctx, 2);
                HIPCHK(launch_bscan_bf16(m, lT, lenT, 0, pieces, Rp, NB, bs, c, sd, keep, bfpart, zcur, st));
                prof_mark(ctx, 3);
                // decisions within the bound of a threshold (this check, the next strong rule) are re-taken on
                // the FP64 scan of those columns
                prof_mark(ctx, 0);
                HIPCHK(launch_fill_u8(flag, 0, p, st));
                HIPCHK(launch_b_band(lT, lenT, p, NB, zcur, c, sd, keep, bs, lam_k,
                                     (ssr && k + 1 < K) ? thrg + (size_t)(k + 1) * BNP : nullptr, bf_rel, flag, st));
                HIPCHK(launch_compact(flag, p, lF, lenF, cmp, st));
                HIPCHK(hipMemcpyAsync(&hp->lenF, lenF, 8, hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                double* part;
                ENSURE(BB_PART, bscan_split_part_bytes(nt, hp->lenF), part);
                HIPCHK(launch_bscan_split(m, lF, hp->lenF, R, NB, bs, c, sd, keep, part, zcur, st));
                prof_mark(ctx, 1);
            }
            if (ssr) HIPCHK(launch_b_viol(lT, lenT, p, NB, zcur, safe, strong, lam_k, wv, bs, st));
            HIPCHK(hipMemcpyAsync(&hp->lenT, lenT, 8, hipMemcpyDeviceToHost, st));
            if ((s = read_bs())) return s;
            prof_add(ctx, 4, BL_PROF_GRAM, (double)max_N * (double)max_P * nt * es);
            double cd_bytes = 0.0, cd_updates = 0.0;
            for (int b = 0; b < NB; ++b)
                if (act[b]) {
                    cd_bytes += (double)hp->bs[b].sweeps * hp->lens[b] * hp->lens[b] * 8.0;
                    cd_updates += (double)hp->bs[b].sweeps * hp->lens[b];
                }
            prof_add(ctx, 6, BL_PROF_CD, cd_bytes, 0.0, cd_updates);
            prof_add(ctx, 2, BL_PROF_BSCAN, (double)hp->lenT * nt * es + (double)nt * NB * (bf ? 2.0 * pieces : 8.0),
                     2.0 * hp->lenT * nt * NB, (double)hp->lenT);
            // the FP64 scans of the working sets' union and (BF16 form) of the columns in the band
            prof_add(ctx, 8, BL_PROF_RECHECK, (double)hp->lenU * nt * es, 0.0, (double)hp->lenU);
            if (bf) prof_add(ctx, 0, BL_PROF_RECHECK, (double)hp->lenF * nt * es, 0.0, (double)hp->lenF);
            bool any = false;
            for (int b = 0; b < NB; ++b) {
                if (!act[b]) continue;
                const BatchScalars& h = hp->bs[b];
                h_sweeps[(size_t)b * K + k] += h.sweeps;
                h_viol[(size_t)b * K + k] += h.n_viol;
                rounds[b] += 1;
                if (h.status != 0 && final_status == BL_OK)
                    final_status = fail(ctx, BL_ERR_NOT_CONVERGED, "problem %d: CD did not converge at lambda index %d", b, k);
                act[b] = (h.n_viol > 0 && h.status == 0) ? 1 : 0;
                if (act[b] && rounds[b] >= opts->max_rounds && final_status == BL_OK) {
                    final_status = fail(ctx, BL_ERR_NOT_CONVERGED, "problem %d: check rounds exhausted at lambda index %d", b, k);
                    act[b] = 0;
                }
                any = any || act[b];
            }
            if (final_status != BL_OK || !any) break;
            // problems with violators solve again over their grown working sets
            std::memset(hp->want, 0, BNP);
            for (int b = 0; b < NB; ++b) hp->want[b] = act[b];
            HIPCHK(hipMemcpyAsync(want, hp->want, BNP, hipMemcpyHostToDevice, st));
            wv = want;
            HIPCHK(launch_b_compact(strong, p, NB, wv, lE, lens, cmp, st));
        }
        if (final_status != BL_OK) break;
        for (int b = 0; b < NB; ++b) h_rounds[(size_t)b * K + k] = rounds[b];
        HIPCHK(launch_b_record(lE, lens, p, NB, beta, c, sd, bs, lam_k, stats, k, K, safecnt, st));
        if (res->beta)
            HIPCHK(hipMemcpy2DAsync(res->beta + (size_t)k * p, (size_t)K * p * 8, beta, p * 8, p * 8, NB,
                                    hipMemcpyDeviceToDevice, st));
        HIPCHK(launch_b_kinc(kdev, st));
        res->k_done = k + 1;
        zprev = zcur;
        zcur = (zcur == z0) ? z1 : z0;
    }
    std::vector<LamStats> hs((size_t)NB * K);
    HIPCHK(hipMemcpyAsync(hs.data(), stats, hs.size() * sizeof(LamStats), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int b = 0; b < NB; ++b) {
        for (int k = 0; k < res->k_done; ++k) {
            const size_t q = (size_t)b * K + k;
            if (res->intercept) res->intercept[q] = hs[q].intercept;
            if (res->rss) res->rss[q] = hs[q].rss;
            if (res->obj) res->obj[q] = hs[q].obj;
            if (res->n_active) res->n_active[q] = hs[q].n_active;
            if (res->n_strong) res->n_strong[q] = hs[q].n_strong;
            if (res->n_safe) res->n_safe[q] = hs[q].n_safe;
            if (res->sweeps) res->sweeps[q] = h_sweeps[q];
            if (res->rounds) res->rounds[q] = h_rounds[q];
            if (res->n_viol) res->n_viol[q] = h_viol[q];
        }
    }
    res->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return final_status;
}
