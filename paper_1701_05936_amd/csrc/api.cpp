// C ABI of libbl.so: argument validation, device scratch, and the host-side
// driver of the lasso path (one stream, one host synchronization per
// CD + check round).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <algorithm>
#include <cstring>
#include <vector>

#include "ctx.h"

using namespace blk;
using namespace blapi;



namespace blapi {

bl_status fail(bl_ctx c, bl_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    return st;
}

// Device scratch owned by the context; grown on demand, freed by bl_destroy.
bl_status ensure(bl_ctx ctx, int id, size_t bytes, void** out) {
    if ((int)ctx->bufs.size() <= id) ctx->bufs.resize(B_COUNT);
    DevBuf& b = ctx->bufs[id];
    if (bytes == 0) bytes = 8;
    if (b.cap < bytes) {
        if (b.p) (void)hipFree(b.p);
        b.p = nullptr;
        b.cap = 0;
        if (hipMalloc(&b.p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(ctx, BL_ERR_NOMEM, "device scratch allocation of %zu bytes failed", bytes);
        }
        b.cap = bytes;
    }
    *out = b.p;
    return BL_OK;
}

int elem_bytes(int xtype) { return xtype == BL_X_F64 ? 8 : (xtype == BL_X_F32 ? 4 : 1); }

bl_status check_ctx(bl_ctx ctx) {
    if (!ctx) return BL_ERR_INVALID;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, BL_ERR_DEVICE, "hipSetDevice failed");
    return BL_OK;
}

bl_status check_matrix(bl_ctx ctx, const bl_matrix* X, Mat* m) {
    if (!X) return fail(ctx, BL_ERR_INVALID, "X is NULL");
    if (!X->X) return fail(ctx, BL_ERR_INVALID, "X->X is NULL");
    if (X->xtype != BL_X_F64 && X->xtype != BL_X_F32 && X->xtype != BL_X_I8)
        return fail(ctx, BL_ERR_INVALID, "unknown xtype %d", X->xtype);
    if (X->n_total < 1) return fail(ctx, BL_ERR_INVALID, "n_total must be >= 1 (got %lld)", (long long)X->n_total);
    if (X->p < 1) return fail(ctx, BL_ERR_INVALID, "p must be >= 1 (got %lld)", (long long)X->p);
    if (X->p > 2147483647LL) return fail(ctx, BL_ERR_UNSUPPORTED, "p above 2^31-1");
    if (X->n_total > 2147483647LL) return fail(ctx, BL_ERR_UNSUPPORTED, "n_total above 2^31-1");
    if (X->ldx < X->n_total) return fail(ctx, BL_ERR_INVALID, "ldx < n_total");
    m->X = X->X;
    m->xtype = X->xtype;
    m->n_total = X->n_total;
    m->p = X->p;
    m->ldx = X->ldx;
    m->mask = X->row_mask;
    return BL_OK;
}

}  // namespace blapi

namespace {

using namespace blapi;

// rows in the fit (synchronous)
bl_status rows_in_fit(bl_ctx ctx, const Mat& m, int64_t* n) {
    if (!m.mask) {
        *n = m.n_total;
        return BL_OK;
    }
    HIPCHK(launch_count_rows(m, &ctx->sc->n_rows, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->sc_host, ctx->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    *n = ctx->sc_host->n_rows;
    if (*n < 1) return fail(ctx, BL_ERR_INVALID, "row_mask selects no rows");
    return BL_OK;
}

bl_status set_n_rows(bl_ctx ctx, int64_t n) {
    HIPCHK(hipMemcpyAsync(&ctx->sc->n_rows, &n, sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return BL_OK;
}

bl_status read_scalars(bl_ctx ctx) {
    HIPCHK(hipMemcpyAsync(ctx->sc_host, ctx->sc, sizeof(DevScalars), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return BL_OK;
}

}  // namespace

namespace blapi {

// kernel timing: record an event pair around a launch when profiling is on
void prof_mark(bl_ctx ctx, int slot) {
    if (ctx->prof) (void)hipEventRecord(ctx->ev[slot], ctx->stream);
}
// after the stream has been synchronized: add the pair (slot, slot+1) to kernel `which`
void prof_add(bl_ctx ctx, int slot, int which, double bytes, double flops, double units) {
    if (!ctx->prof) return;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, ctx->ev[slot], ctx->ev[slot + 1]) == hipSuccess) {
        ctx->kp[which].launches += 1;
        ctx->kp[which].total_ms += ms;
        ctx->kp[which].bytes += bytes;
        ctx->kp[which].flops += flops;
        ctx->kp[which].units += units;
    }
}

}  // namespace blapi

namespace {

using namespace blapi;

// ---- Gram pool -------------------------------------------------------------------------------------
bl_status pool_reset(bl_ctx ctx, int64_t p) {
    int32_t *pos, *list;
    ENSURE(B_POOLPOS, p * 4, pos);
    ENSURE(B_POOLLIST, p * 4, list);
    HIPCHK(launch_fill_u8((uint8_t*)pos, 0xff, p * 4, ctx->stream));  // every slot = -1
    ctx->pool_size = 0;
    return BL_OK;
}

bl_status pool_reserve(bl_ctx ctx, int64_t need) {
    if (need <= ctx->pool_cap) return BL_OK;
    int64_t cap = ctx->pool_cap * 2;
    if (cap < need) cap = need;
    if (cap < 1024) cap = 1024;
    cap = (cap + 63) / 64 * 64;
    double* g = nullptr;
    if (hipMalloc(&g, (size_t)cap * cap * sizeof(double)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(ctx, BL_ERR_NOMEM, "Gram pool of %lld features does not fit", (long long)cap);
    }
    if (ctx->gpool && ctx->pool_size > 0)
        HIPCHK(hipMemcpy2DAsync(g, cap * sizeof(double), ctx->gpool, ctx->pool_cap * sizeof(double),
                                ctx->pool_size * sizeof(double), ctx->pool_size, hipMemcpyDeviceToDevice,
                                ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (ctx->gpool) (void)hipFree(ctx->gpool);
    ctx->gpool = g;
    ctx->pool_cap = cap;
    return BL_OK;
}

// X as the path reads it: resident in HBM (m.X a device pointer), or in host memory (host = true), streamed
// to the device in panels of panel_cols columns (column-major, so a panel is one contiguous copy).
struct XAccess {
    Mat m;
    bool host = false;
    int64_t panel_cols = 0;
    bl_host_stream* hs = nullptr;   // streaming counters (host X)
};

size_t x_es(const Mat& m) { return (size_t)elem_bytes(m.xtype); }

// the two panel buffers, their events and the copy stream (all library-owned, default priority)
bl_status panels_ready(bl_ctx ctx, const XAccess& xa) {
    const size_t bytes = (size_t)xa.panel_cols * (size_t)xa.m.ldx * x_es(xa.m);
    if (ctx->panel_cap < bytes) {
        for (int b = 0; b < 2; ++b) {
            if (ctx->panel[b]) (void)hipFree(ctx->panel[b]);
            ctx->panel[b] = nullptr;
        }
        ctx->panel_cap = 0;
        HIPCHK(hipStreamSynchronize(ctx->stream));
        ctx->panel_used[0] = ctx->panel_used[1] = false;
        for (int b = 0; b < 2; ++b)
            if (hipMalloc(&ctx->panel[b], bytes) != hipSuccess) {
                (void)hipGetLastError();
                return fail(ctx, BL_ERR_NOMEM, "panel buffers of %zu bytes do not fit", bytes);
            }
        ctx->panel_cap = bytes;
    }
    for (int b = 0; b < 2; ++b) {
        if (!ctx->ev_copy[b]) HIPCHK(hipEventCreateWithFlags(&ctx->ev_copy[b], hipEventDisableTiming));
        if (!ctx->ev_free[b]) HIPCHK(hipEventCreateWithFlags(&ctx->ev_free[b], hipEventDisableTiming));
    }
    if (!ctx->aux) HIPCHK(hipStreamCreateWithFlags(&ctx->aux, hipStreamNonBlocking));
    return BL_OK;
}

// Stream the panels holding the columns [j0, j1) of each listed range, two in flight: panel i is copied on
// the aux stream into buffer i mod 2 once the main stream has finished with that buffer, and the main
// stream runs fn(panel device pointer, j0, j1) after the copy.  fn enqueues its kernels on ctx->stream.
template <typename Fn>
bl_status stream_panels(bl_ctx ctx, const XAccess& xa, const std::vector<std::pair<int64_t, int64_t>>& ranges, Fn fn) {
    bl_status s;
    if ((s = panels_ready(ctx, xa))) return s;
    const size_t col_bytes = (size_t)xa.m.ldx * x_es(xa.m);
    bool* used = ctx->panel_used;   // across calls: a buffer may still be read by the last call's kernels
    for (size_t i = 0; i < ranges.size(); ++i) {
        const int b = (int)(i & 1);
        const int64_t j0 = ranges[i].first, j1 = ranges[i].second;
        if (used[b]) HIPCHK(hipStreamWaitEvent(ctx->aux, ctx->ev_free[b], 0));
        const size_t bytes = (size_t)(j1 - j0) * col_bytes;
        HIPCHK(hipMemcpyAsync(ctx->panel[b], (const char*)xa.m.X + (size_t)j0 * col_bytes, bytes, hipMemcpyHostToDevice,
                              ctx->aux));
        HIPCHK(hipEventRecord(ctx->ev_copy[b], ctx->aux));
        HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_copy[b], 0));
        if ((s = fn(ctx->panel[b], j0, j1))) return s;
        HIPCHK(hipEventRecord(ctx->ev_free[b], ctx->stream));
        used[b] = true;
        if (xa.hs) {
            xa.hs->panels_streamed += 1;
            xa.hs->bytes_streamed += (double)bytes;
        }
    }
    return BL_OK;
}

// every panel of X
std::vector<std::pair<int64_t, int64_t>> all_panels(const XAccess& xa) {
    std::vector<std::pair<int64_t, int64_t>> out;
    for (int64_t j0 = 0; j0 < xa.m.p; j0 += xa.panel_cols) out.emplace_back(j0, std::min(xa.m.p, j0 + xa.panel_cols));
    return out;
}

// column statistics of every column
bl_status x_colstats(bl_ctx ctx, const XAccess& xa, double* c, double* sd, uint8_t* keep, int64_t n) {
    if (!xa.host) {
        HIPCHK(launch_colstats(xa.m, c, sd, keep, n, ctx->stream));
        return BL_OK;
    }
    return stream_panels(ctx, xa, all_panels(xa), [&](void* buf, int64_t j0, int64_t j1) -> bl_status {
        Mat pm = xa.m;
        pm.X = buf;
        pm.p = j1 - j0;
        HIPCHK(launch_colstats(pm, c + j0, sd + j0, keep + j0, n, ctx->stream));
        return BL_OK;
    });
}

// identity column list 0..p-1 (device), for scans of every column of a panel
bl_status ident_list(bl_ctx ctx, int64_t p, int32_t** out) {
    DevBuf& b = ctx->bufs[H_IDENT];
    const bool fresh = b.cap < (size_t)p * 4;
    int32_t* id;
    ENSURE(H_IDENT, p * 4, id);
    if (fresh || ctx->ident_len < p) {
        std::vector<int32_t> h(p);
        for (int64_t j = 0; j < p; ++j) h[j] = (int32_t)j;
        HIPCHK(hipMemcpyAsync(id, h.data(), p * 4, hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(hipStreamSynchronize(ctx->stream));
        ctx->ident_len = p;
    }
    *out = id;
    return BL_OK;
}

// the scan of ScanArgs a (kernels.hip) over X wherever it lives.  Host X: the listed columns' panels only
// (BEDPP survivors steer which panels move); each panel's launch reads the columns through a pointer
// offset so that global column indices address the panel buffer.
bl_status x_scan(bl_ctx ctx, const XAccess& xa, const ScanArgs& a) {
    hipStream_t st = ctx->stream;
    if (!xa.host) {
        HIPCHK(launch_scan(xa.m, a, st));
        return BL_OK;
    }
    const int64_t p = xa.m.p;
    std::vector<int32_t> hl;
    const int32_t* cols = a.cols;
    int64_t len = a.len_host;
    bl_status s;
    if (cols) {
        if (a.len_dev) {
            HIPCHK(hipMemcpyAsync(&ctx->sc_host->stage, a.len_dev, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            len = ctx->sc_host->stage;
        }
        hl.resize((size_t)std::max<int64_t>(len, 1));
        if (len > 0) {
            HIPCHK(hipMemcpyAsync(hl.data(), cols, len * 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
        }
    } else {
        int32_t* id;
        if ((s = ident_list(ctx, p, &id))) return s;
        cols = id;
    }
    // the panels that hold listed columns (lists are ascending), with the list range of each
    std::vector<std::pair<int64_t, int64_t>> ranges;
    std::vector<std::pair<int64_t, int64_t>> spans;
    int64_t t = 0;
    for (int64_t j0 = 0; j0 < p && t < len; j0 += xa.panel_cols) {
        const int64_t j1 = std::min(p, j0 + xa.panel_cols);
        const int64_t t0 = t;
        if (a.cols) {
            while (t < len && hl[t] < j1) ++t;
        } else {
            t = std::min(len, j1);
        }
        if (t > t0) {
            ranges.emplace_back(j0, j1);
            spans.emplace_back(t0, t);
        }
    }
    if (xa.hs) xa.hs->panels_skipped += (p + xa.panel_cols - 1) / xa.panel_cols - (int64_t)ranges.size();
    size_t k = 0;
    s = stream_panels(ctx, xa, ranges, [&](void* buf, int64_t j0, int64_t j1) -> bl_status {
        (void)j1;
        Mat pm = xa.m;
        pm.X = (const char*)buf - (ptrdiff_t)((size_t)j0 * (size_t)xa.m.ldx * x_es(xa.m));
        ScanArgs pa = a;
        pa.cols = cols + spans[k].first;
        pa.len_dev = nullptr;
        pa.len_host = spans[k].second - spans[k].first;
        pa.len_out = nullptr;
        ++k;
        HIPCHK(launch_scan(pm, pa, ctx->stream));
        return BL_OK;
    });
    if (s) return s;
    if (a.len_out) {
        ctx->sc_host->stage = len;
        HIPCHK(hipMemcpyAsync(a.len_out, &ctx->sc_host->stage, sizeof(int64_t), hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    return BL_OK;
}

// v = standardized column j (fitted rows) wherever X lives
bl_status x_std_column(bl_ctx ctx, const XAccess& xa, int64_t j, const double* c, const double* sd, double* v) {
    if (!xa.host) {
        HIPCHK(launch_std_column(xa.m, j, c, sd, v, ctx->stream));
        return BL_OK;
    }
    void* col;
    const size_t cb = (size_t)xa.m.ldx * x_es(xa.m);
    ENSURE(H_COL, cb, col);
    HIPCHK(hipMemcpyAsync(col, (const char*)xa.m.X + (size_t)j * cb, cb, hipMemcpyHostToDevice, ctx->stream));
    Mat pm = xa.m;
    pm.X = col;
    pm.p = 1;
    HIPCHK(launch_std_column(pm, 0, c + j, sd + j, v, ctx->stream));
    if (xa.hs) xa.hs->bytes_streamed += (double)cb;
    return BL_OK;
}

// Cyclic CD at lambda over set[0..m) (length also at *len_dev), warm-started from beta and r.
// z[j] must hold x~_j' r / n at the current r for every j of the set.  Updates beta, r,
// sc->sum_r, sc->rss and sc->round.{sweeps, status, cd_len}.
// Host X: the device cache of the pool features' columns (pool order), grown keeping its contents.
// The column bytes are those of the current X: a cache laid out for another X is rebuilt (the pool, which the
// cache follows, starts empty on every path).
bl_status xcache_reserve(bl_ctx ctx, const XAccess& xa, int64_t need) {
    const size_t cb = (size_t)xa.m.ldx * x_es(xa.m);
    const bool same = cb == ctx->xcache_cb;
    if (need <= ctx->xcache_cap && same) return BL_OK;
    const int64_t keep = same ? ctx->pool_size : 0;
    int64_t cap = std::max<int64_t>({need, same ? 2 * ctx->xcache_cap : 0, 256});
    void* nb = nullptr;
    double *nc = nullptr, *ns = nullptr;
    if (hipMalloc(&nb, (size_t)cap * cb) != hipSuccess || hipMalloc((void**)&nc, (size_t)cap * 8) != hipSuccess ||
        hipMalloc((void**)&ns, (size_t)cap * 8) != hipSuccess) {
        (void)hipGetLastError();
        if (nb) (void)hipFree(nb);
        if (nc) (void)hipFree(nc);
        return fail(ctx, BL_ERR_NOMEM, "device cache of %lld columns does not fit", (long long)cap);
    }
    if (keep > 0) {
        HIPCHK(hipMemcpyAsync(nb, ctx->xcache, (size_t)keep * cb, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(nc, ctx->xcache_c, (size_t)keep * 8, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(ns, ctx->xcache_s, (size_t)keep * 8, hipMemcpyDeviceToDevice, ctx->stream));
    }
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (ctx->xcache) (void)hipFree(ctx->xcache);
    if (ctx->xcache_c) (void)hipFree(ctx->xcache_c);
    if (ctx->xcache_s) (void)hipFree(ctx->xcache_s);
    ctx->xcache = nb;
    ctx->xcache_c = nc;
    ctx->xcache_s = ns;
    ctx->xcache_cap = cap;
    ctx->xcache_cb = cb;
    return BL_OK;
}

bl_status solve_set(bl_ctx ctx, const XAccess& xa, const int32_t* set, const int64_t* len_dev, int64_t m,
                    const double* z, double* beta, double* r, const double* c, const double* s, double n_rows,
                    double lam, double tol, int max_sweeps, double alpha = 1.0, const double* w = nullptr) {
    const Mat& mt = xa.m;
    hipStream_t st = ctx->stream;
    const double es = (double)elem_bytes(mt.xtype);
    const bool enet = alpha < 1.0 || w != nullptr;
    // covariance form up to cov_max features; the multi-workgroup solve only with every workgroup resident
    // and one threshold for every coordinate, else the single-workgroup solve (its gradient lives in LDS:
    // GCD_MAX features) or the residual form
    int H = gcd_multi_helpers(m, ctx->cd_helpers);
    const bool multi_ok = H <= ctx->cd_helpers && w == nullptr;
    const bool cov = m <= ctx->cov_max && (multi_ok || m <= GCD_MAX);
    if (!multi_ok) H = 0;
    ctx->last_residual = !cov;
    if (!cov && xa.host)
        return fail(ctx, BL_ERR_UNSUPPORTED, "X in host memory: working set of %lld features above the covariance "
                    "solve's limits", (long long)m);
    if (!cov) {
        if (!cd_supported(mt.n_total))
            return fail(ctx, BL_ERR_UNSUPPORTED, "working set of %lld features with n_total %lld is too large",
                        (long long)m, (long long)mt.n_total);
        CdArgs ca{};
        ca.set = set;
        ca.len_host = m;
        ca.c = c;
        ca.s = s;
        ca.lam = lam;
        ca.beta = beta;
        ca.r = r;
        ca.tol = tol;
        ca.max_sweeps = max_sweeps;
        ca.sc = ctx->sc;
        ca.alpha = alpha;
        ca.w = w;
        prof_mark(ctx, 0);
        HIPCHK(launch_cd(mt, ca, st));
        prof_mark(ctx, 1);
        return BL_OK;
    }
    int32_t *pos, *list;
    double *GE, *g0, *b0, *b1, *part;
    ENSURE(B_POOLPOS, mt.p * 4, pos);
    ENSURE(B_POOLLIST, mt.p * 4, list);
    ENSURE(B_GE, (size_t)(m > 0 ? m : 1) * (m > 0 ? m : 1) * 8, GE);
    ENSURE(B_G0, (m + 1) * 8, g0);
    ENSURE(B_B0, (m + 1) * 8, b0);
    ENSURE(B_B1, (m + 1) * 8, b1);
    ENSURE(B_RUPART, r_update_scratch_bytes(mt.n_total, m), part);
    prof_mark(ctx, 4);
    HIPCHK(launch_pool_add(set, len_dev, m, pos, list, ctx->pool_size, &ctx->sc->n_new, st));
    HIPCHK(hipMemcpyAsync(&ctx->sc_host->n_new, &ctx->sc->n_new, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    const int64_t n_new = ctx->sc_host->n_new;
    bl_status s_;
    if ((s_ = pool_reserve(ctx, ctx->pool_size + n_new))) return s_;
    // the residual update below reads X through (Mat, set, c, s); with X in host memory those are the cache
    Mat xm = mt;
    const int32_t* xset = set;
    const double *xc = c, *xs = s;
    if (!xa.host) {
        HIPCHK(launch_gram_update(mt, list, ctx->pool_size + n_new, ctx->pool_size, n_new, c, s, n_rows, ctx->gpool,
                                  ctx->pool_cap, st));
    } else {
        // copy the new pool features' columns into the cache (pool order) with their statistics, then
        // take the Gram entries from the cache in pool order: the same tiles over the same columns
        if ((s_ = xcache_reserve(ctx, xa, ctx->pool_size + n_new))) return s_;
        double* cc = ctx->xcache_c;
        double* scc = ctx->xcache_s;
        int32_t *id, *setc;
        ENSURE(H_SETC, (size_t)(m + 1) * 4, setc);
        const size_t cb = (size_t)mt.ldx * x_es(mt);
        if (n_new > 0) {
            std::vector<int32_t> hj(n_new);
            HIPCHK(hipMemcpyAsync(hj.data(), list + ctx->pool_size, n_new * 4, hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            for (int64_t t = 0; t < n_new; ++t)
                HIPCHK(hipMemcpyAsync((char*)ctx->xcache + (size_t)(ctx->pool_size + t) * cb,
                                      (const char*)mt.X + (size_t)hj[t] * cb, (size_t)mt.n_total * x_es(mt),
                                      hipMemcpyHostToDevice, st));
            if (xa.hs) xa.hs->bytes_streamed += (double)n_new * (double)mt.n_total * (double)x_es(mt);
            HIPCHK(launch_gather_start(list + ctx->pool_size, n_new, c, s, cc + ctx->pool_size, scc + ctx->pool_size,
                                       st));
        }
        bl_status si;
        if ((si = ident_list(ctx, std::max<int64_t>(ctx->xcache_cap, 1), &id))) return si;
        xm.X = ctx->xcache;
        xm.p = ctx->xcache_cap;
        HIPCHK(launch_gram_update(xm, id, ctx->pool_size + n_new, ctx->pool_size, n_new, cc, scc, n_rows, ctx->gpool,
                                  ctx->pool_cap, st));
        HIPCHK(launch_map_pos(set, m, pos, setc, st));
        xset = setc;
        xc = cc;
        xs = scc;
    }
    const double gram_bytes = (double)(ctx->pool_size + 2 * n_new) * mt.n_total * es + (double)m * m * 8.0;
    ctx->pool_size += n_new;
    HIPCHK(launch_gather_gram(set, m, pos, ctx->gpool, ctx->pool_cap, GE, st));
    HIPCHK(launch_gather_start(set, m, z, beta, g0, b0, st));
    // the elastic net solved as a lasso in gamma = q beta with a unit-diagonal Gram (launch_enet_scale)
    double* lamv = nullptr;
    double lam_solve = lam;
    if (enet) {
        if (w) ENSURE(B_LAMV, (m + 1) * 8, lamv);
        HIPCHK(launch_enet_scale(set, m, w, lam, alpha, GE, g0, b0, lamv, st));
        if (!w) lam_solve = lam * alpha / std::sqrt(1.0 + lam * (1.0 - alpha));
    }
    prof_mark(ctx, 5);
    if (H > 0) {
        // leader + helper workgroups; g0 holds the working gradient, b1 the working coefficients
        double* dl;
        uint32_t* sy;
        const size_t words = gcd_multi_sync_words(H);
        ENSURE(B_DELTA, (size_t)2 * (m + 64) * 8, dl);
        ENSURE(B_SYNC, words * 4, sy);
        HIPCHK(launch_copy_f64(b0, b1, m, st));
        HIPCHK(hipMemsetAsync(sy, 0, words * 4, st));
        GcdMultiArgs ma{};
        ma.G = GE;
        ma.m = m;
        ma.g = g0;
        ma.b = b1;
        ma.delta = dl;
        ma.sync = sy;
        ma.H = H;
        ma.spin_limit = 2000000u;  // about two seconds of polling per wait
        ma.lam = lam_solve;
        ma.tol = tol;
        ma.max_sweeps = max_sweeps;
        ma.sc = ctx->sc;
        prof_mark(ctx, 0);
        HIPCHK(launch_gcd_multi(ma, st));
        prof_mark(ctx, 1);
        HIPCHK(launch_scatter_beta(set, m, b1, beta, st));
    } else {
        GcdArgs ga{};
        ga.G = GE;
        ga.m = m;
        ga.g0 = g0;
        ga.b0 = b0;
        ga.b1 = b1;
        ga.set = set;
        ga.beta = beta;
        ga.lam = lam_solve;
        ga.lamv = lamv;
        ga.tol = tol;
        ga.max_sweeps = max_sweeps;
        ga.sc = ctx->sc;
        prof_mark(ctx, 0);
        HIPCHK(launch_gcd(ga, st));
        prof_mark(ctx, 1);
    }
    if (enet) HIPCHK(launch_enet_unscale(set, m, w, lam, alpha, b0, b1, beta, st));
    prof_mark(ctx, 6);
    HIPCHK(launch_r_update(xm, xset, m, b0, b1, xc, xs, part, r, st));
    HIPCHK(launch_sum_r(mt, r, ctx->sc, true, st));
    prof_mark(ctx, 7);
    ctx->pend_gram_bytes = gram_bytes;
    ctx->pend_ru_bytes = (double)m * mt.n_total * es;
    return BL_OK;
}

// Active-set cycling (the descent iterates over the nonzero coefficients of the working set, Section 3.1.1):
// solve on A = {j in E : beta_j != 0} (E's order) until a sweep over A changes no coefficient by tol or more,
// then sweep E once from its gradient at the current residual; stop when that sweep changes no coefficient by
// tol or more (the plain solve's stopping rule), else take the new A and repeat.  Working sets below
// ctx->cycle_min are solved by one plain solve.  Each part is a solve_set; their sweeps add up (an A-sweep
// counts as a sweep) and their totals go to sc->round.  *cycled tells the caller that the CD, Gram and
// residual-update timings were recorded here, part by part.
bl_status solve_ws(bl_ctx ctx, const XAccess& xa, const int32_t* set, const int64_t* len_dev, int64_t m,
                   const double* z, double* beta, double* r, const double* c, const double* s, const uint8_t* keep,
                   double n_rows, double lam, double tol, int max_sweeps, double alpha, const double* w, void* scr,
                   bool* cycled) {
    *cycled = false;
    if (m < ctx->cycle_min || max_sweeps < 2)
        return solve_set(ctx, xa, set, len_dev, m, z, beta, r, c, s, n_rows, lam, tol, max_sweeps, alpha, w);
    *cycled = true;
    const Mat& mt = xa.m;
    const int64_t p = mt.p;
    hipStream_t st = ctx->stream;
    const double col_bytes = (double)mt.n_total * elem_bytes(mt.xtype);
    uint8_t* fl;
    int32_t* lA;
    int64_t* lenA;
    double* zc;
    ENSURE(B_CYCF, (size_t)p, fl);
    ENSURE(B_CYCL, (size_t)p * 4, lA);
    ENSURE(B_CYCN, 8, lenA);
    ENSURE(B_ZCYC, (size_t)p * 8, zc);
    // the round's figures of one part, and its timings
    auto part_done = [&](int64_t mp, RoundInfo* ri) -> bl_status {
        HIPCHK(hipMemcpyAsync(&ctx->sc_host->round, &ctx->sc->round, sizeof(RoundInfo), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        *ri = ctx->sc_host->round;
        if (ctx->last_residual) {
            prof_add(ctx, 0, BL_PROF_CD, (double)ri->sweeps * mp * col_bytes, 0.0, (double)ri->sweeps * mp);
        } else {
            prof_add(ctx, 0, BL_PROF_CD, (double)ri->sweeps * (double)mp * (double)mp * 8.0, 0.0,
                     (double)ri->sweeps * mp);
            prof_add(ctx, 4, BL_PROF_GRAM, ctx->pend_gram_bytes);
            prof_add(ctx, 6, BL_PROF_RUPDATE, ctx->pend_ru_bytes);
        }
        return BL_OK;
    };
    // gradient of the listed columns at the current residual into zc
    auto grad = [&](const int32_t* cols, const int64_t* len) -> bl_status {
        ScanArgs ga{};
        ga.cols = cols;
        ga.len_dev = len;
        ga.r = r;
        ga.sc = ctx->sc;
        ga.c = c;
        ga.s = s;
        ga.keep = keep;
        ga.z = zc;
        return x_scan(ctx, xa, ga);
    };
    int sweeps = 0, status = 1;
    bl_status st_;
    RoundInfo ri{};
    const double* zA = z;   // the caller's gradient holds at the current residual for the first part
    for (int cyc = 0;; ++cyc) {
        HIPCHK(launch_fill_u8(fl, 0, p, st));
        HIPCHK(launch_mark_nonzero(set, len_dev, m, beta, fl, st));
        HIPCHK(launch_compact(fl, p, lA, lenA, scr, st));
        HIPCHK(hipMemcpyAsync(&ctx->sc_host->stage, lenA, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        const int64_t mA = ctx->sc_host->stage;
        const int budget = max_sweeps - sweeps - 1;   // one sweep is kept for E
        if (mA > 0 && mA < m && budget >= 1) {
            if (cyc > 0) {
                if ((st_ = grad(lA, lenA))) return st_;
                zA = zc;
            }
            if ((st_ = solve_set(ctx, xa, lA, lenA, mA, zA, beta, r, c, s, n_rows, lam, tol, budget, alpha, w)))
                return st_;
            if ((st_ = part_done(mA, &ri))) return st_;
            sweeps += ri.sweeps;
            if (ri.status == 2) {
                status = 2;
                break;
            }
        }
        // one sweep over E
        if ((st_ = grad(set, len_dev))) return st_;
        if ((st_ = solve_set(ctx, xa, set, len_dev, m, zc, beta, r, c, s, n_rows, lam, tol, 1, alpha, w))) return st_;
        if ((st_ = part_done(m, &ri))) return st_;
        sweeps += ri.sweeps;
        if (ri.status != 1) {
            status = ri.status;   // 0: the sweep over E changed nothing by tol; 2: device error
            break;
        }
        if (sweeps >= max_sweeps) break;
        zA = nullptr;
    }
    HIPCHK(launch_set_round(ctx->sc, sweeps, status, (int32_t)m, st));
    return BL_OK;
}

double bedpp_rhs(double lmax, double lam, double v) {
    double slack = v - lmax * lmax;
    if (slack < 0.0) slack = 0.0;
    return 2.0 * lam * lmax - (lmax - lam) * std::sqrt(slack);
}

}  // namespace

extern "C" {

bl_status bl_create(bl_ctx* out, int device, void* hip_stream) {
    if (!out) return BL_ERR_INVALID;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return BL_ERR_DEVICE;
    if (device < 0 || device >= ndev) return BL_ERR_INVALID;
    if (hipSetDevice(device) != hipSuccess) return BL_ERR_DEVICE;
    bl_ctx c = new bl_ctx_s();
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->bufs.resize(B_COUNT);
    if (hipMalloc(&c->sc, sizeof(DevScalars)) != hipSuccess ||
        hipHostMalloc((void**)&c->sc_host, sizeof(DevScalars), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        bl_destroy(c);
        return BL_ERR_NOMEM;
    }
    std::memset(c->sc_host, 0, sizeof(DevScalars));
    // every workgroup of the multi-workgroup solve waits on the others, so all of them must be resident
    c->cd_resident = gcd_multi_resident();
    c->cd_helpers = std::min(255, std::max(0, c->cd_resident - 1));
    c->cov_max = gram_cd_max();
    // this GPU's copy of the allocation-free check's array (an error surfaces when that entry point is called)
    (void)noalloc_setup(device);
    *out = c;
    return BL_OK;
}

bl_status bl_get_limits(bl_ctx ctx, bl_limits* out) {
    if (!ctx) return BL_ERR_INVALID;
    if (!out) return fail(ctx, BL_ERR_INVALID, "out is NULL");
    out->cov_max = ctx->cov_max;
    out->cd_helpers = ctx->cd_helpers;
    out->resident = ctx->cd_resident;
    out->cycle_min = ctx->cycle_min == INT64_MAX ? -1 : ctx->cycle_min;
    return BL_OK;
}

bl_status bl_set_limits(bl_ctx ctx, const bl_limits* in) {
    if (!ctx) return BL_ERR_INVALID;
    if (!in) return fail(ctx, BL_ERR_INVALID, "in is NULL");
    if (in->cov_max < 0) return fail(ctx, BL_ERR_INVALID, "cov_max must be >= 0");
    if (in->cd_helpers < -1 || in->cd_helpers > 255 || in->cd_helpers > ctx->cd_resident - 1)
        return fail(ctx, BL_ERR_INVALID, "cd_helpers must be -1 or in 0..%d (resident workgroups - 1, at most 255)",
                    std::min(255, std::max(0, ctx->cd_resident - 1)));
    if (in->cycle_min < -1) return fail(ctx, BL_ERR_INVALID, "cycle_min must be -1, 0 or positive");
    if (in->cov_max > 0) ctx->cov_max = in->cov_max;
    if (in->cd_helpers >= 0) ctx->cd_helpers = in->cd_helpers;
    if (in->cycle_min > 0) ctx->cycle_min = in->cycle_min;
    if (in->cycle_min == -1) ctx->cycle_min = INT64_MAX;
    return BL_OK;
}

void bl_destroy(bl_ctx c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    else (void)hipDeviceSynchronize();
    for (auto& b : c->bufs)
        if (b.p) (void)hipFree(b.p);
    for (auto& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    for (int b = 0; b < 2; ++b) {
        if (c->panel[b]) (void)hipFree(c->panel[b]);
        if (c->ev_copy[b]) (void)hipEventDestroy(c->ev_copy[b]);
        if (c->ev_free[b]) (void)hipEventDestroy(c->ev_free[b]);
    }
    if (c->xcache) (void)hipFree(c->xcache);
    if (c->xcache_c) (void)hipFree(c->xcache_c);
    if (c->xcache_s) (void)hipFree(c->xcache_s);
    if (c->gpool) (void)hipFree(c->gpool);
    if (c->bgpool) (void)hipFree(c->bgpool);
    if (c->bpinned) (void)hipHostFree(c->bpinned);
    if (c->aux) (void)hipStreamDestroy(c->aux);
    if (c->sc) (void)hipFree(c->sc);
    if (c->sc_host) (void)hipHostFree(c->sc_host);
    delete c;
}

const char* bl_last_error(bl_ctx c) { return c ? c->err.c_str() : "null context"; }

bl_status bl_profile(bl_ctx ctx, int enable) {
    bl_status s = check_ctx(ctx);
    if (s) return s;
    if (enable) {
        for (auto& e : ctx->ev)
            if (!e) HIPCHK(hipEventCreate(&e));
    }
    ctx->prof = enable != 0;
    for (auto& k : ctx->kp) k = bl_kernel_profile{0, 0.0, 0.0, 0.0, 0.0};
    return BL_OK;
}

bl_status bl_profile_get(bl_ctx ctx, int kernel, bl_kernel_profile* out) {
    if (!ctx) return BL_ERR_INVALID;
    if (kernel < 0 || kernel >= BL_PROF_COUNT || !out) return fail(ctx, BL_ERR_INVALID, "bad kernel id or NULL out");
    *out = ctx->kp[kernel];
    return BL_OK;
}

bl_status bl_device_info(bl_ctx ctx, int* n_cu, char* name, int name_len) {
    bl_status s = check_ctx(ctx);
    if (s) return s;
    hipDeviceProp_t prop;
    HIPCHK(hipGetDeviceProperties(&prop, ctx->device));
    if (n_cu) *n_cu = prop.multiProcessorCount;
    if (name && name_len > 0) {
        std::snprintf(name, (size_t)name_len, "%s (%s)", prop.name, prop.gcnArchName);
    }
    return BL_OK;
}

bl_status bl_standardize(bl_ctx ctx, const bl_matrix* X, double* center, double* scale, uint8_t* keep,
                         int64_t* n_rows) {
    bl_status s = check_ctx(ctx);
    if (s) return s;
    Mat m;
    if ((s = check_matrix(ctx, X, &m))) return s;
    if (!center || !scale || !keep) return fail(ctx, BL_ERR_INVALID, "center/scale/keep must be non-NULL");
    int64_t n;
    if ((s = rows_in_fit(ctx, m, &n))) return s;
    HIPCHK(launch_colstats(m, center, scale, keep, n, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (n_rows) *n_rows = n;
    return BL_OK;
}

bl_status bl_lambda_max(bl_ctx ctx, const bl_matrix* X, const double* center, const double* scale,
                        const uint8_t* keep, const double* y, double* ytilde, double* a, double* y_mean,
                        double* lambda_max, int64_t* jstar) {
    bl_status s = check_ctx(ctx);
    if (s) return s;
    Mat m;
    if ((s = check_matrix(ctx, X, &m))) return s;
    if (!center || !scale || !keep || !y || !ytilde || !a)
        return fail(ctx, BL_ERR_INVALID, "array arguments must be non-NULL");
    int64_t n;
    if ((s = rows_in_fit(ctx, m, &n))) return s;
    double* pv;
    int64_t* pi;
    ENSURE(B_ARGV, 256 * sizeof(double), pv);
    ENSURE(B_ARGI, 256 * sizeof(int64_t), pi);
    HIPCHK(launch_center_y(m, y, ytilde, nullptr, ctx->sc, ctx->stream));
    HIPCHK(launch_sum_r(m, ytilde, ctx->sc, false, ctx->stream));
    ScanArgs sa{};
    sa.cols = nullptr;
    sa.len_dev = nullptr;
    sa.len_host = m.p;
    sa.r = ytilde;
    sa.sc = ctx->sc;
    sa.c = center;
    sa.s = scale;
    sa.keep = keep;
    sa.z = a;
    HIPCHK(launch_scan(m, sa, ctx->stream));
    HIPCHK(launch_argmax_abs(a, keep, m.p, pv, pi, ctx->sc, ctx->stream));
    if ((s = read_scalars(ctx))) return s;
    const DevScalars& h = *ctx->sc_host;
    if (!std::isfinite(h.y_mean) || !std::isfinite(h.yy)) return fail(ctx, BL_ERR_INVALID, "y has NaN or Inf");
    if (h.jstar < 0) return fail(ctx, BL_ERR_INVALID, "no column is kept (all constant)");
    if (!std::isfinite(h.lmax)) return fail(ctx, BL_ERR_INVALID, "X or y has NaN or Inf (lambda_max not finite)");
    if (y_mean) *y_mean = h.y_mean;
    if (lambda_max) *lambda_max = h.lmax;
    if (jstar) *jstar = h.jstar;
    return BL_OK;
}

bl_status bl_bedpp_setup(bl_ctx ctx, const bl_matrix* X, const double* center, const double* scale,
                         const uint8_t* keep, const double* ytilde, int64_t jstar, double* b, double* v) {
    bl_status s = check_ctx(ctx);
    if (s) return s;
    Mat m;
    if ((s = check_matrix(ctx, X, &m))) return s;
    if (!center || !scale || !keep || !ytilde || !b) return fail(ctx, BL_ERR_INVALID, "array arguments must be non-NULL");
    if (jstar < 0 || jstar >= m.p) return fail(ctx, BL_ERR_INVALID, "jstar out of range");
    int64_t n;
    if ((s = rows_in_fit(ctx, m, &n))) return s;
    if ((s = set_n_rows(ctx, n))) return s;
    double* xs;
    ENSURE(B_XS, m.n_total * sizeof(double), xs);
    HIPCHK(launch_sum_r(m, ytilde, ctx->sc, true, ctx->stream));  // rss = ||y~||^2
    HIPCHK(launch_std_column(m, jstar, center, scale, xs, ctx->stream));
    HIPCHK(launch_sum_r(m, xs, ctx->sc, false, ctx->stream));
    ScanArgs sa{};
    sa.len_host = m.p;
    sa.r = xs;
    sa.sc = ctx->sc;
    sa.c = center;
    sa.s = scale;
    sa.keep = keep;
    sa.z = b;
    HIPCHK(launch_scan(m, sa, ctx->stream));
    if ((s = read_scalars(ctx))) return s;
    if (v) *v = ctx->sc_host->rss / (double)n;
    return BL_OK;
}

bl_status bl_screen(bl_ctx ctx, const bl_screen_state* st, double lambda_k, double lambda_prev, const double* z_prev,
                    uint8_t* safe, uint8_t* strong, int64_t* n_safe, int64_t* n_strong) {
    bl_status s = check_ctx(ctx);
    if (s) return s;
    if (!st || !safe || !strong) return fail(ctx, BL_ERR_INVALID, "state/safe/strong must be non-NULL");
    if (st->p < 1 || st->p > 2147483647LL) return fail(ctx, BL_ERR_INVALID, "bad p");
    if (!st->keep) return fail(ctx, BL_ERR_INVALID, "keep must be non-NULL");
    const int rule = st->rule;
    if (rule == BL_SCREEN_LEARNED)
        return fail(ctx, BL_ERR_UNSUPPORTED, "the learned rule needs the path's z history: it runs inside bl_fit_path");
    if (rule < BL_SCREEN_NONE || rule > BL_SCREEN_ACTIVE) return fail(ctx, BL_ERR_INVALID, "unknown rule");
    const bool active_only = rule == BL_SCREEN_ACTIVE;
    const bool bedpp = rule == BL_SCREEN_BEDPP || rule == BL_SCREEN_SSR_BEDPP || active_only;
    const bool ssr = rule == BL_SCREEN_SSR || rule == BL_SCREEN_SSR_BEDPP;
    if (bedpp && (!st->a || !st->b)) return fail(ctx, BL_ERR_INVALID, "BEDPP needs a and b");
    if (ssr && !z_prev) return fail(ctx, BL_ERR_INVALID, "strong rule needs z_prev");
    if (active_only && !st->active) return fail(ctx, BL_ERR_INVALID, "the active-set rule needs the active mask");
    if (!(std::isfinite(lambda_k) && lambda_k > 0.0)) return fail(ctx, BL_ERR_INVALID, "lambda_k must be finite and > 0");
    if (ssr && !(std::isfinite(lambda_prev) && lambda_prev >= lambda_k))
        return fail(ctx, BL_ERR_INVALID, "lambda_prev must be finite and >= lambda_k");
    if (bedpp && !(std::isfinite(st->lambda_max) && st->lambda_max > 0.0 && std::isfinite(st->v)))
        return fail(ctx, BL_ERR_INVALID, "bad lambda_max or v");
    const int64_t p = st->p;
    const double rhs = bedpp ? bedpp_rhs(st->lambda_max, lambda_k, st->v) : 0.0;
    const double sgn = st->sign_star < 0 ? -1.0 : 1.0;
    HIPCHK(launch_bedpp(p, st->a, st->b, st->keep, bedpp, st->lambda_max, sgn, lambda_k, rhs, safe, ctx->stream));
    // the active-set rule: the strong rule's test with an infinite threshold keeps the active features only
    HIPCHK(launch_ssr(p, safe, st->active, nullptr, active_only ? nullptr : z_prev, ssr || active_only,
                      active_only ? INFINITY : 2.0 * lambda_k - lambda_prev, strong, ctx->stream));
    void* scr;
    int32_t* lst;
    int64_t* lens;
    ENSURE(B_CMP, compact_scratch_bytes(p), scr);
    ENSURE(B_LT, p * sizeof(int32_t), lst);
    ENSURE(B_LENS, 8 * sizeof(int64_t), lens);
    HIPCHK(launch_compact(safe, p, lst, lens + 0, scr, ctx->stream));
    HIPCHK(launch_compact(strong, p, lst, lens + 1, scr, ctx->stream));
    int64_t h[2];
    HIPCHK(hipMemcpyAsync(h, lens, 2 * sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (n_safe) *n_safe = h[0];
    if (n_strong) *n_strong = h[1];
    return BL_OK;
}

bl_status bl_cd_solve(bl_ctx ctx, const bl_matrix* X, const double* center, const double* scale, double lambda,
                      const int32_t* set, int64_t set_len, double* beta, double* r, double tol, int32_t max_sweeps,
                      int32_t* sweeps) {
    bl_status s = check_ctx(ctx);
    if (s) return s;
    Mat m;
    if ((s = check_matrix(ctx, X, &m))) return s;
    if (!center || !scale || !beta || !r) return fail(ctx, BL_ERR_INVALID, "array arguments must be non-NULL");
    if (set_len < 0 || set_len > m.p) return fail(ctx, BL_ERR_INVALID, "set_len out of range");
    if (set_len > 0 && !set) return fail(ctx, BL_ERR_INVALID, "set is NULL");
    if (!(std::isfinite(lambda) && lambda >= 0.0)) return fail(ctx, BL_ERR_INVALID, "lambda must be finite and >= 0");
    if (!(tol > 0.0) || max_sweeps < 1) return fail(ctx, BL_ERR_INVALID, "tol must be > 0 and max_sweeps >= 1");
    int64_t n;
    if ((s = rows_in_fit(ctx, m, &n))) return s;
    if ((s = set_n_rows(ctx, n))) return s;
    double* zs;
    ENSURE(B_ZS, m.p * 8, zs);
    HIPCHK(launch_sum_r(m, r, ctx->sc, false, ctx->stream));
    if (set_len > 0) {
        ScanArgs sa{};
        sa.cols = set;
        sa.len_host = set_len;
        sa.r = r;
        sa.sc = ctx->sc;
        sa.c = center;
        sa.s = scale;
        sa.z = zs;
        HIPCHK(launch_scan(m, sa, ctx->stream));
    }
    if ((s = pool_reset(ctx, m.p))) return s;
    XAccess xa;
    xa.m = m;
    if ((s = solve_set(ctx, xa, set, nullptr, set_len, zs, beta, r, center, scale, (double)n, lambda, tol,
                       max_sweeps)))
        return s;
    if ((s = read_scalars(ctx))) return s;
    if (sweeps) *sweeps = ctx->sc_host->round.sweeps;
    if (ctx->sc_host->round.status == 2)
        return fail(ctx, BL_ERR_DEVICE, "coordinate descent workgroups timed out waiting for each other");
    if (ctx->sc_host->round.status != 0)
        return fail(ctx, BL_ERR_NOT_CONVERGED, "coordinate descent did not converge in %d sweeps", max_sweeps);
    return BL_OK;
}

bl_status bl_kkt_check(bl_ctx ctx, const bl_matrix* X, const double* center, const double* scale, const double* r,
                       double lambda, const int32_t* check_set, int64_t len, const uint8_t* exclude, double* z,
                       int32_t* violators, int64_t* n_viol) {
    bl_status s = check_ctx(ctx);
    if (s) return s;
    Mat m;
    if ((s = check_matrix(ctx, X, &m))) return s;
    if (!center || !scale || !r || !z || !violators) return fail(ctx, BL_ERR_INVALID, "array arguments must be non-NULL");
    if (len < 0 || len > m.p) return fail(ctx, BL_ERR_INVALID, "len out of range");
    if (len > 0 && !check_set) return fail(ctx, BL_ERR_INVALID, "check_set is NULL");
    if (!(std::isfinite(lambda) && lambda >= 0.0)) return fail(ctx, BL_ERR_INVALID, "lambda must be finite and >= 0");
    int64_t n;
    if ((s = rows_in_fit(ctx, m, &n))) return s;
    if ((s = set_n_rows(ctx, n))) return s;
    uint8_t* mark;
    void* scr;
    int64_t* lens;
    ENSURE(B_MARK, m.p, mark);
    ENSURE(B_CMP, compact_scratch_bytes(m.p), scr);
    ENSURE(B_LENS, 8 * sizeof(int64_t), lens);
    HIPCHK(launch_fill_u8(mark, 0, m.p, ctx->stream));
    HIPCHK(hipMemsetAsync(&ctx->sc->round, 0, sizeof(RoundInfo), ctx->stream));
    HIPCHK(launch_sum_r(m, r, ctx->sc, false, ctx->stream));
    if (len > 0) {
        ScanArgs sa{};
        sa.cols = check_set;
        sa.len_host = len;
        sa.r = r;
        sa.sc = ctx->sc;
        sa.c = center;
        sa.s = scale;
        sa.keep = nullptr;
        sa.z = z;
        sa.check = true;
        sa.lam = lambda;
        sa.in_s = nullptr;
        sa.excl = exclude;
        sa.mark = mark;
        sa.nviol = &ctx->sc->round.n_viol;
        HIPCHK(launch_scan(m, sa, ctx->stream));
    }
    HIPCHK(launch_compact(mark, m.p, violators, lens, scr, ctx->stream));
    int64_t nv = 0;
    HIPCHK(hipMemcpyAsync(&nv, lens, sizeof(int64_t), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (n_viol) *n_viol = nv;
    return BL_OK;
}

bl_status bl_scan(bl_ctx ctx, const bl_matrix* X, const double* center, const double* scale, const double* r,
                  const int32_t* cols, int64_t len, int32_t precision, double* z, double* err) {
    bl_status s = check_ctx(ctx);
    if (s) return s;
    Mat m;
    if ((s = check_matrix(ctx, X, &m))) return s;
    if (!center || !scale || !r || !z) return fail(ctx, BL_ERR_INVALID, "array arguments must be non-NULL");
    if (len < 0 || len > m.p) return fail(ctx, BL_ERR_INVALID, "len out of range");
    if (len > 0 && !cols) return fail(ctx, BL_ERR_INVALID, "cols is NULL");
    if (precision != BL_PREC_FP64 && precision != BL_PREC_BF16X3 && precision != BL_PREC_I8X4 &&
        precision != BL_PREC_BF16X2)
        return fail(ctx, BL_ERR_INVALID, "unknown precision");
    if (precision == BL_PREC_BF16X2) return fail(ctx, BL_ERR_UNSUPPORTED, "BF16X2 scans are the batched form's");
    if (precision != BL_PREC_FP64 && !lowp_supported(m))
        return fail(ctx, BL_ERR_UNSUPPORTED, "matrix-core scans need int8 X with 16-byte aligned columns");
    int64_t n;
    if ((s = rows_in_fit(ctx, m, &n))) return s;
    if ((s = set_n_rows(ctx, n))) return s;
    hipStream_t st = ctx->stream;
    HIPCHK(launch_sum_r(m, r, ctx->sc, true, st));
    if (len > 0) {
        if (precision == BL_PREC_FP64) {
            ScanArgs sa{};
            sa.cols = cols;
            sa.len_host = len;
            sa.r = r;
            sa.sc = ctx->sc;
            sa.c = center;
            sa.s = scale;
            sa.z = z;
            HIPCHK(launch_scan(m, sa, st));
        } else {
            const bool i8 = precision == BL_PREC_I8X4;
            void* pieces;
            int64_t* lens;
            ENSURE(B_PIECES, lowp_piece_bytes(m.n_total), pieces);
            ENSURE(B_LENS, 8 * sizeof(int64_t), lens);
            if (i8) {
                HIPCHK(launch_r_pieces_i8(r, m.n_total, (int8_t*)pieces, ctx->sc, st));
                HIPCHK(launch_scan_i8(m, (const int8_t*)pieces, cols, nullptr, len, ctx->sc, center, scale, nullptr, z,
                                      st));
            } else {
                HIPCHK(launch_r_pieces(r, m.n_total, (__bf16*)pieces, st));
                HIPCHK(launch_scan_bf16(m, (const __bf16*)pieces, cols, nullptr, len, ctx->sc, center, scale, nullptr,
                                        z, st));
            }
            if (err) {
                ctx->sc_host->stage = len;
                HIPCHK(hipMemcpyAsync(lens + 5, &ctx->sc_host->stage, sizeof(int64_t), hipMemcpyHostToDevice, st));
                HIPCHK(launch_band(cols, lens + 5, z, center, scale, ctx->sc, -1.0, nullptr, nullptr, -1.0, nullptr,
                                   err, m.p, i8, st));
            }
        }
    }
    HIPCHK(hipStreamSynchronize(st));
    return BL_OK;
}

}  // extern "C"

namespace {

// Logistic safe rule: the |a_j| threshold of the gap-safe sphere around the dual point known at lambda_max
// (beta = 0, b0 = logit(y-bar)); G is that point's duality gap at lambda, in closed form over the n1 ones.
double logit_entropy(double t) {
    const double a = t > 0.0 ? t * std::log(t) : 0.0;
    const double b = t < 1.0 ? (1.0 - t) * std::log(1.0 - t) : 0.0;
    return a + b;
}

double logit_safe_threshold(double n, double n1, double lmax, double lam) {
    const double yb = n1 / n, n0 = n - n1;
    const double P = -(n1 * std::log(yb) + n0 * std::log(1.0 - yb));
    const double rho = std::min(1.0, lam / lmax);
    const double D = -(n1 * logit_entropy(1.0 - rho * (1.0 - yb)) + n0 * logit_entropy(rho * yb));
    const double G = std::max(0.0, P - D);
    return lmax * (1.0 - std::sqrt(G / (2.0 * n)) / lam);
}

// The logistic lasso path (family BL_FAMILY_BINOMIAL; include/bl.h states the model and the rules).
bl_status fit_logistic(bl_ctx ctx, const XAccess& xa, const double* y, const bl_path_opts* opts,
                       bl_path_result* res) {
    auto t_start = std::chrono::steady_clock::now();
    bl_status s;
    const Mat& m = xa.m;
    if (!y || !opts || !res) return fail(ctx, BL_ERR_INVALID, "y/opts/res must be non-NULL");
    res->k_done = 0;
    res->n_recorded = 0;
    const int K = opts->nlambda;
    if (K < 1) return fail(ctx, BL_ERR_INVALID, "nlambda must be >= 1");
    if (!opts->lambda && !(opts->lambda_min_ratio > 0.0 && opts->lambda_min_ratio < 1.0) && K > 1)
        return fail(ctx, BL_ERR_INVALID, "lambda_min_ratio must be in (0, 1)");
    if (opts->lambda)
        for (int k = 0; k < K; ++k) {
            if (!(std::isfinite(opts->lambda[k]) && opts->lambda[k] > 0.0))
                return fail(ctx, BL_ERR_INVALID, "user lambda[%d] must be finite and > 0", k);
            if (k > 0 && !(opts->lambda[k] <= opts->lambda[k - 1]))
                return fail(ctx, BL_ERR_INVALID, "user lambda must be non-increasing");
        }
    if (opts->rule < BL_SCREEN_NONE || opts->rule > BL_SCREEN_ACTIVE) return fail(ctx, BL_ERR_INVALID, "unknown rule");
    if (!(opts->tol > 0.0) || opts->max_sweeps < 1 || opts->max_rounds < 1)
        return fail(ctx, BL_ERR_INVALID, "tol > 0, max_sweeps >= 1 and max_rounds >= 1 are required");
    if (opts->rule == BL_SCREEN_LEARNED || opts->precision != BL_PREC_FP64 || opts->k_start != 0 ||
        opts->rec_cap > 0 || (opts->alpha != 0.0 && opts->alpha != 1.0) || opts->penalty_factor)
        return fail(ctx, BL_ERR_UNSUPPORTED, "logistic regression: FP64 scans, lasso penalty, no learned rule, resume "
                    "or training records");
    const bool active_only = opts->rule == BL_SCREEN_ACTIVE;
    const bool safe_rule = opts->rule == BL_SCREEN_BEDPP || opts->rule == BL_SCREEN_SSR_BEDPP || active_only;
    const bool ssr = opts->rule == BL_SCREEN_SSR || opts->rule == BL_SCREEN_SSR_BEDPP;
    const bool check = ssr || active_only;
    const int64_t p = m.p, nt = m.n_total;
    hipStream_t st = ctx->stream;

    double *yt, *r, *r0c, *g, *eta, *a, *z0, *z1, *zs, *beta, *c, *sc_, *pv;
    uint8_t *s0, *s1, *strong, *keep;
    int32_t *lT, *lE;
    int64_t *lens, *pi;
    LamStats* stats;
    void* scr;
    ENSURE(B_YT, nt * 8, yt);
    ENSURE(B_R, nt * 8, r);
    ENSURE(L_R0C, nt * 8, r0c);
    ENSURE(L_G, nt * 8, g);
    ENSURE(L_ETA, nt * 8, eta);
    ENSURE(B_A, p * 8, a);
    ENSURE(B_Z0, p * 8, z0);
    ENSURE(B_Z1, p * 8, z1);
    ENSURE(B_ZS, p * 8, zs);
    ENSURE(B_BETA, p * 8, beta);
    ENSURE(B_S0, p, s0);
    ENSURE(B_S1, p, s1);
    ENSURE(B_E, p, strong);
    ENSURE(B_LT, p * 4, lT);
    ENSURE(B_LE, p * 4, lE);
    ENSURE(B_LENS, 8 * 8, lens);
    ENSURE(B_STATS, (size_t)K * sizeof(LamStats), stats);
    ENSURE(B_CMP, compact_scratch_bytes(p), scr);
    ENSURE(B_ARGV, 256 * 8, pv);
    ENSURE(B_ARGI, 256 * 8, pi);
    if (res->center) c = res->center; else ENSURE(B_C, p * 8, c);
    if (res->scale) sc_ = res->scale; else ENSURE(B_S, p * 8, sc_);
    if (res->keep) keep = res->keep; else ENSURE(B_KEEP, p, keep);

    if ((s = pool_reset(ctx, p))) return s;
    int64_t n;
    if ((s = rows_in_fit(ctx, m, &n))) return s;
    if ((s = set_n_rows(ctx, n))) return s;
    const double es = (double)elem_bytes(m.xtype);
    const double col_bytes = (double)nt * es;
    HIPCHK(launch_logit_check_y(m, y, ctx->sc, st));
    if ((s = read_scalars(ctx))) return s;
    const double n1 = ctx->sc_host->lg_n1;
    if (ctx->sc_host->lg_bad > 0.0) return fail(ctx, BL_ERR_INVALID, "logistic regression: y must be 0 or 1 on the fitted rows");
    if (n1 < 1.0 || n1 > (double)n - 1.0) return fail(ctx, BL_ERR_INVALID, "logistic regression: y is constant on the fitted rows");
    prof_mark(ctx, 0);
    if ((s = x_colstats(ctx, xa, c, sc_, keep, n))) return s;
    prof_mark(ctx, 1);
    // a_j = x~_j'(y - y-bar) / n and lambda_max
    HIPCHK(launch_center_y(m, y, yt, nullptr, ctx->sc, st));
    HIPCHK(launch_sum_r(m, yt, ctx->sc, false, st));
    ScanArgs sa{};
    sa.len_host = p;
    sa.r = yt;
    sa.sc = ctx->sc;
    sa.c = c;
    sa.s = sc_;
    sa.keep = keep;
    sa.z = a;
    prof_mark(ctx, 2);
    if ((s = x_scan(ctx, xa, sa))) return s;
    prof_mark(ctx, 3);
    HIPCHK(launch_argmax_abs(a, keep, p, pv, pi, ctx->sc, st));
    if ((s = read_scalars(ctx))) return s;
    prof_add(ctx, 0, BL_PROF_COLSTATS, (double)p * col_bytes);
    prof_add(ctx, 2, BL_PROF_SCAN, (double)p * col_bytes + nt * 8.0, 0.0, (double)p);
    const double ybar = ctx->sc_host->y_mean, lmax = ctx->sc_host->lmax;
    if (ctx->sc_host->jstar < 0) return fail(ctx, BL_ERR_INVALID, "no column is kept (all constant)");
    if (!std::isfinite(lmax) || !(lmax > 0.0)) return fail(ctx, BL_ERR_INVALID, "X has NaN or Inf, or lambda_max is 0");
    std::vector<double> lam(K);
    for (int k = 0; k < K; ++k)
        lam[k] = opts->lambda ? opts->lambda[k]
                              : (K == 1 ? lmax : lmax * std::pow(opts->lambda_min_ratio, (double)k / (double)(K - 1)));
    if (res->lambda)
        for (int k = 0; k < K; ++k) res->lambda[k] = lam[k];
    res->y_mean = ybar;
    res->lambda_max = lmax;
    res->jstar = ctx->sc_host->jstar;

    // beta = 0 with the intercept logit(y-bar) solves every lambda >= lambda_max
    HIPCHK(launch_fill_f64(beta, 0.0, p, st));
    HIPCHK(launch_logit_init(m, std::log(ybar / (1.0 - ybar)), eta, ctx->sc, st));
    HIPCHK(hipMemsetAsync(lens, 0, 8 * 8, st));
    std::vector<int32_t> h_sweeps(K, 0), h_rounds(K, 0);
    std::vector<int64_t> h_viol(K, 0);
    // safe[j] at lambda: kept and, with the safe rule, |a_j| at or above the sphere's threshold
    auto safe_at = [&](double l, uint8_t* out) -> hipError_t {
        return launch_ssr(p, keep, nullptr, nullptr, a, safe_rule, safe_rule ? logit_safe_threshold((double)n, n1, lmax, l)
                                                                              : 0.0, out, st);
    };
    uint8_t* safe_cur = s0;
    uint8_t* safe_next = s1;
    double* zprev = a;
    double* zcur = z0;
    int64_t* len_cur = lens + 1;
    int64_t* len_next = lens + 2;
    bl_status final_status = BL_OK;
    int k_first = 0;
    if (lam[0] >= lmax) {
        HIPCHK(safe_at(lam[0], safe_cur));
        HIPCHK(launch_compact(safe_cur, p, lT, len_cur, scr, st));
        HIPCHK(launch_logit_loss(m, y, eta, ctx->sc, st));
        HIPCHK(launch_record(nullptr, lens + 3, len_cur, lens + 3, beta, c, sc_, ctx->sc, lam[0], stats + 0, st));
        if (res->beta) HIPCHK(hipMemcpyAsync(res->beta, beta, p * 8, hipMemcpyDeviceToDevice, st));
        k_first = 1;
    }
    for (int k = k_first; k < K; ++k) {
        const double lk = lam[k];
        const double lprev = k > 0 ? lam[k - 1] : lmax;
        HIPCHK(safe_at(lk, safe_cur));
        HIPCHK(launch_compact(safe_cur, p, lT, len_cur, scr, st));
        uint8_t* scan_mask = safe_cur;
        if (k + 1 < K) {
            HIPCHK(safe_at(lam[k + 1], safe_next));
            scan_mask = safe_next;
        }
        HIPCHK(launch_compact(scan_mask, p, lT, len_next, scr, st));
        HIPCHK(launch_ssr(p, safe_cur, nullptr, beta, zprev, check, active_only ? INFINITY : 2.0 * lk - lprev, strong,
                          st));
        HIPCHK(launch_compact(strong, p, lE, lens + 0, scr, st));
        int rounds = 0, sweeps_total = 0;
        int64_t viol_total = 0;
        for (;;) {
            HIPCHK(hipMemcpyAsync(&ctx->sc_host->n_new, lens + 0, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            const int64_t m_len = ctx->sc_host->n_new;
            // majorize-minimize steps over the working set
            for (int it = 0;; ++it) {
                HIPCHK(launch_logit_resid(m, y, eta, g, r, st));   // r = 4 (y - pi)
                HIPCHK(launch_sum_r(m, r, ctx->sc, false, st));
                HIPCHK(launch_logit_center(m, r, r0c, ctx->sc, st));   // intercept step, r centered, copy in r0c
                HIPCHK(launch_sum_r(m, r, ctx->sc, false, st));
                ScanArgs ga{};
                ga.cols = lE;
                ga.len_dev = lens + 0;
                ga.r = r;
                ga.sc = ctx->sc;
                ga.c = c;
                ga.s = sc_;
                ga.keep = keep;
                ga.z = zs;
                if ((s = x_scan(ctx, xa, ga))) return s;
                if ((s = solve_set(ctx, xa, lE, lens + 0, m_len, zs, beta, r, c, sc_, (double)n, 4.0 * lk, opts->tol,
                                   opts->max_sweeps)))
                    return s;
                HIPCHK(launch_logit_eta(m, r0c, r, eta, ctx->sc, st));
                if ((s = read_scalars(ctx))) return s;
                const RoundInfo ri = ctx->sc_host->round;
                sweeps_total += ri.sweeps;
                if (ri.status == 2) {
                    final_status = fail(ctx, BL_ERR_DEVICE, "CD workgroups timed out waiting for each other at lambda index %d", k);
                    break;
                }
                if (ri.status != 0) {
                    final_status = fail(ctx, BL_ERR_NOT_CONVERGED, "CD did not converge at lambda index %d", k);
                    break;
                }
                // a step that moved no coefficient (intercept included) by tol ends the solve
                if (ri.sweeps <= 1 && std::fabs(ctx->sc_host->lg_db0) < opts->tol) break;
                if (it + 1 >= opts->max_sweeps) {
                    final_status = fail(ctx, BL_ERR_NOT_CONVERGED, "majorization steps exhausted at lambda index %d", k);
                    break;
                }
            }
            if (final_status != BL_OK) break;
            // the check: z = x~'(y - pi)/n over S_{k+1}, violators in S_k outside the working set
            HIPCHK(launch_logit_resid(m, y, eta, g, nullptr, st));
            HIPCHK(launch_sum_r(m, g, ctx->sc, false, st));
            HIPCHK(hipMemsetAsync(&ctx->sc->round.n_viol, 0, sizeof(uint32_t), st));
            ScanArgs ka{};
            ka.cols = lT;
            ka.len_dev = len_next;
            ka.r = g;
            ka.sc = ctx->sc;
            ka.c = c;
            ka.s = sc_;
            ka.keep = keep;
            ka.z = zcur;
            ka.check = check;
            ka.lam = lk;
            ka.in_s = safe_cur;
            ka.excl = strong;
            ka.mark = strong;
            ka.nviol = &ctx->sc->round.n_viol;
            ka.len_out = &ctx->sc->round.scan_len;
            prof_mark(ctx, 2);
            if ((s = x_scan(ctx, xa, ka))) return s;
            prof_mark(ctx, 3);
            if ((s = read_scalars(ctx))) return s;
            prof_add(ctx, 2, BL_PROF_SCAN, (double)ctx->sc_host->round.scan_len * col_bytes + nt * 8.0, 0.0,
                     (double)ctx->sc_host->round.scan_len);
            ++rounds;
            const uint32_t nv = ctx->sc_host->round.n_viol;
            viol_total += nv;
            if (nv == 0) break;
            if (rounds >= opts->max_rounds) {
                final_status = fail(ctx, BL_ERR_NOT_CONVERGED, "check rounds exhausted at lambda index %d", k);
                break;
            }
            HIPCHK(launch_compact(strong, p, lE, lens + 0, scr, st));
        }
        if (final_status != BL_OK) break;
        h_sweeps[k] = sweeps_total;
        h_rounds[k] = rounds;
        h_viol[k] = viol_total;
        HIPCHK(launch_logit_loss(m, y, eta, ctx->sc, st));
        HIPCHK(launch_record(lE, lens + 0, len_cur, len_next, beta, c, sc_, ctx->sc, lk, stats + k, st));
        if (res->beta) HIPCHK(hipMemcpyAsync(res->beta + (size_t)k * p, beta, p * 8, hipMemcpyDeviceToDevice, st));
        res->k_done = k + 1;
        zprev = zcur;
        zcur = (zcur == z0) ? z1 : z0;
    }
    if (k_first == 1 && res->k_done < 1) res->k_done = 1;
    std::vector<LamStats> hs(K);
    HIPCHK(hipMemcpyAsync(hs.data(), stats, (size_t)K * sizeof(LamStats), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int k = 0; k < res->k_done; ++k) {
        if (res->intercept) res->intercept[k] = hs[k].intercept;
        if (res->rss) res->rss[k] = hs[k].rss;
        if (res->obj) res->obj[k] = hs[k].obj;
        if (res->n_active) res->n_active[k] = hs[k].n_active;
        if (res->sweeps) res->sweeps[k] = h_sweeps[k];
        if (res->rounds) res->rounds[k] = h_rounds[k];
        if (res->n_viol) res->n_viol[k] = h_viol[k];
        if (res->n_scanned) res->n_scanned[k] = hs[k].n_scan * h_rounds[k];
        if (res->n_recheck) res->n_recheck[k] = 0;
        if (res->n_safe) res->n_safe[k] = hs[k].n_safe;
        if (res->n_strong) res->n_strong[k] = hs[k].n_strong;
    }
    if (opts->r_out) HIPCHK(hipMemcpyAsync(opts->r_out, g, nt * 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    res->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return final_status;
}

// The path over X wherever it lives (XAccess): bl_fit_path (X in HBM) and bl_fit_path_host (X in host memory).
bl_status fit_path_impl(bl_ctx ctx, const XAccess& xa, const double* y, const bl_path_opts* opts,
                        bl_path_result* res) {
    if (opts && opts->family == BL_FAMILY_BINOMIAL) return fit_logistic(ctx, xa, y, opts, res);
    if (opts && opts->family != BL_FAMILY_GAUSSIAN) return fail(ctx, BL_ERR_INVALID, "unknown family %d", opts->family);
    auto t_start = std::chrono::steady_clock::now();
    bl_status s;
    const Mat& m = xa.m;
    if (!y || !opts || !res) return fail(ctx, BL_ERR_INVALID, "y/opts/res must be non-NULL");
    res->k_done = 0;
    const int K = opts->nlambda;
    if (K < 1) return fail(ctx, BL_ERR_INVALID, "nlambda must be >= 1");
    if (!opts->lambda && !(opts->lambda_min_ratio > 0.0 && opts->lambda_min_ratio < 1.0) && K > 1)
        return fail(ctx, BL_ERR_INVALID, "lambda_min_ratio must be in (0, 1)");
    if (opts->lambda) {
        for (int k = 0; k < K; ++k) {
            if (!(std::isfinite(opts->lambda[k]) && opts->lambda[k] > 0.0))
                return fail(ctx, BL_ERR_INVALID, "user lambda[%d] must be finite and > 0", k);
            if (k > 0 && !(opts->lambda[k] <= opts->lambda[k - 1]))
                return fail(ctx, BL_ERR_INVALID, "user lambda must be non-increasing");
        }
    }
    if (opts->rule < BL_SCREEN_NONE || opts->rule > BL_SCREEN_ACTIVE) return fail(ctx, BL_ERR_INVALID, "unknown rule");
    if (!(opts->tol > 0.0) || opts->max_sweeps < 1 || opts->max_rounds < 1)
        return fail(ctx, BL_ERR_INVALID, "tol > 0, max_sweeps >= 1 and max_rounds >= 1 are required");
    const bool learned = opts->rule == BL_SCREEN_LEARNED;
    const bool active_only = opts->rule == BL_SCREEN_ACTIVE;
    // elastic net and penalty factors; BEDPP is a lasso rule and stays off for them
    const double alpha = opts->alpha == 0.0 ? 1.0 : opts->alpha;
    if (!(alpha > 0.0 && alpha <= 1.0)) return fail(ctx, BL_ERR_INVALID, "alpha must be in (0, 1]");
    const double* pf = opts->penalty_factor;
    const bool enet = alpha < 1.0 || pf != nullptr;
    if (enet && (learned || opts->precision != BL_PREC_FP64))
        return fail(ctx, BL_ERR_UNSUPPORTED, "elastic net / penalty factors: FP64 scans and no learned rule");
    const bool bedpp =
        !enet && (opts->rule == BL_SCREEN_BEDPP || opts->rule == BL_SCREEN_SSR_BEDPP || learned || active_only);
    const bool ssr = opts->rule == BL_SCREEN_SSR || opts->rule == BL_SCREEN_SSR_BEDPP || learned;
    const bool check = ssr || active_only;   // rules with a post-convergence check
    const int k_start = opts->k_start;
    if (k_start < 0 || k_start >= K) return fail(ctx, BL_ERR_INVALID, "k_start must be in 0..nlambda-1");
    if (k_start > 0 && !opts->beta_init) return fail(ctx, BL_ERR_INVALID, "k_start > 0 needs beta_init");
    if (learned && (!opts->mlp || !(opts->mlp_tau >= 0.0 && opts->mlp_tau < 1.0)))
        return fail(ctx, BL_ERR_INVALID, "the learned rule needs opts->mlp and 0 <= mlp_tau < 1");
    const bool recording = opts->rec_cap > 0;
    if (recording && (!opts->rec_feat || !opts->rec_label))
        return fail(ctx, BL_ERR_INVALID, "rec_cap > 0 needs rec_feat and rec_label");
    if (recording && !ssr) return fail(ctx, BL_ERR_INVALID, "training records need a rule with the strong rule");
    res->n_recorded = 0;
    const bool history = learned || recording;
    if (k_start > 0 && history)
        return fail(ctx, BL_ERR_UNSUPPORTED, "resuming needs no z history: not with the learned rule or training records");
    const float tau_logit = learned && opts->mlp_tau > 0.0 ? (float)std::log(opts->mlp_tau / (1.0 - opts->mlp_tau))
                                                           : -INFINITY;
    if (opts->precision != BL_PREC_FP64 && opts->precision != BL_PREC_BF16X3 && opts->precision != BL_PREC_I8X4 &&
        opts->precision != BL_PREC_BF16X2)
        return fail(ctx, BL_ERR_INVALID, "unknown precision");
    if (opts->precision == BL_PREC_BF16X2)
        return fail(ctx, BL_ERR_UNSUPPORTED, "BF16X2 scans are the batched form's");
    const bool lowp = opts->precision != BL_PREC_FP64;
    const bool i8 = opts->precision == BL_PREC_I8X4;
    if (lowp && !lowp_supported(m))
        return fail(ctx, BL_ERR_UNSUPPORTED, "matrix-core scans need int8 X with 16-byte aligned columns");
    const int64_t p = m.p, nt = m.n_total;
    hipStream_t st = ctx->stream;
    if (pf) {
        std::vector<double> hw(p);
        HIPCHK(hipMemcpyAsync(hw.data(), pf, p * 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        for (int64_t j = 0; j < p; ++j)
            if (!(std::isfinite(hw[j]) && hw[j] > 0.0))
                return fail(ctx, BL_ERR_INVALID, "penalty_factor[%lld] must be finite and > 0", (long long)j);
    }

    double *yt, *r, *xs, *a, *b, *z0, *z1, *beta, *c, *sc_, *pv;
    uint8_t *s0, *s1, *strong, *keep;
    int32_t *lT, *lE;
    int64_t *lens, *pi;
    LamStats* stats;
    void* scr;
    ENSURE(B_YT, nt * 8, yt);
    ENSURE(B_R, nt * 8, r);
    ENSURE(B_XS, nt * 8, xs);
    ENSURE(B_A, p * 8, a);
    ENSURE(B_B, p * 8, b);
    ENSURE(B_Z0, p * 8, z0);
    ENSURE(B_Z1, p * 8, z1);
    ENSURE(B_BETA, p * 8, beta);
    ENSURE(B_S0, p, s0);
    ENSURE(B_S1, p, s1);
    ENSURE(B_E, p, strong);
    ENSURE(B_LT, p * 4, lT);
    ENSURE(B_LE, p * 4, lE);
    ENSURE(B_LENS, 8 * 8, lens);
    ENSURE(B_STATS, (size_t)K * sizeof(LamStats), stats);
    ENSURE(B_CMP, compact_scratch_bytes(p), scr);
    ENSURE(B_ARGV, 256 * 8, pv);
    ENSURE(B_ARGI, 256 * 8, pi);
    if (res->center) c = res->center; else ENSURE(B_C, p * 8, c);
    if (res->scale) sc_ = res->scale; else ENSURE(B_S, p * 8, sc_);
    if (res->keep) keep = res->keep; else ENSURE(B_KEEP, p, keep);
    float* zh = nullptr;          // |z|/lambda at the last three lambda values, slot k mod 3
    uint8_t* cand = nullptr;      // strong-rule candidates outside the previous active set
    int32_t* lC = nullptr;
    int64_t* recn = nullptr;
    if (history) {
        ENSURE(B_ZH, (size_t)3 * p * 4, zh);
        ENSURE(B_RECN, 8, recn);
    }
    if (recording) {
        ENSURE(B_CAND, p, cand);
        ENSURE(B_LC, p * 4, lC);
    }
    void* pieces = nullptr;
    uint8_t* flag = nullptr;
    int32_t* lB = nullptr;
    if (lowp) {
        ENSURE(B_PIECES, lowp_piece_bytes(nt), pieces);
        ENSURE(B_MARK, p, flag);
        ENSURE(B_LB, p * 4, lB);
    }

    if ((s = pool_reset(ctx, p))) return s;
    // standardize, lambda_max, BEDPP inputs
    int64_t n;
    if ((s = rows_in_fit(ctx, m, &n))) return s;
    if ((s = set_n_rows(ctx, n))) return s;
    const double es = (double)elem_bytes(m.xtype);
    const double col_bytes = (double)nt * es;
    prof_mark(ctx, 0);
    if ((s = x_colstats(ctx, xa, c, sc_, keep, n))) return s;
    prof_mark(ctx, 1);
    HIPCHK(launch_center_y(m, y, yt, r, ctx->sc, st));
    HIPCHK(launch_sum_r(m, yt, ctx->sc, true, st));
    ScanArgs sa{};
    sa.len_host = p;
    sa.r = yt;
    sa.sc = ctx->sc;
    sa.c = c;
    sa.s = sc_;
    sa.keep = keep;
    sa.z = a;
    prof_mark(ctx, 2);
    if ((s = x_scan(ctx, xa, sa))) return s;
    prof_mark(ctx, 3);
    HIPCHK(launch_argmax_abs(a, keep, p, pv, pi, ctx->sc, st));
    if ((s = read_scalars(ctx))) return s;
    prof_add(ctx, 0, BL_PROF_COLSTATS, (double)p * col_bytes);
    // the set-up scans are FP64 scans; in the precision form they are kept apart from its BF16 check scans
    const int setup_slot = lowp ? BL_PROF_SETUP : BL_PROF_SCAN;
    prof_add(ctx, 2, setup_slot, (double)p * col_bytes + nt * 8.0, 0.0, (double)p);
    const double ybar = ctx->sc_host->y_mean, yy = ctx->sc_host->yy;
    double lmax = ctx->sc_host->lmax;
    const int64_t jstar = ctx->sc_host->jstar;
    if (enet && jstar >= 0) {
        // lambda_max of the elastic net: the largest |a_j| / (alpha w_j) over kept columns
        double* lt;
        ENSURE(B_LMT, p * 8, lt);
        HIPCHK(launch_enet_lmax_terms(a, pf, alpha, p, lt, st));
        HIPCHK(launch_argmax_abs(lt, keep, p, pv, pi, ctx->sc, st));
        if ((s = read_scalars(ctx))) return s;
        lmax = ctx->sc_host->lmax;
    }
    if (!std::isfinite(ybar) || !std::isfinite(yy)) return fail(ctx, BL_ERR_INVALID, "y has NaN or Inf");
    if (jstar < 0) return fail(ctx, BL_ERR_INVALID, "no column is kept (all constant)");
    if (!std::isfinite(lmax)) return fail(ctx, BL_ERR_INVALID, "X or y has NaN or Inf");
    if (!(lmax > 0.0)) return fail(ctx, BL_ERR_INVALID, "lambda_max is 0 (y is constant on the fitted rows)");
    const double v = yy / (double)n;
    double sgn = 1.0;
    {
        HIPCHK(hipMemcpyAsync(&ctx->sc_host->rss, a + jstar, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        sgn = ctx->sc_host->rss < 0 ? -1.0 : 1.0;
    }
    if (bedpp) {
        if ((s = x_std_column(ctx, xa, jstar, c, sc_, xs))) return s;
        HIPCHK(launch_sum_r(m, xs, ctx->sc, false, st));
        sa.r = xs;
        sa.z = b;
        prof_mark(ctx, 2);
        if ((s = x_scan(ctx, xa, sa))) return s;
        prof_mark(ctx, 3);
        HIPCHK(hipStreamSynchronize(st));
        prof_add(ctx, 2, setup_slot, (double)p * col_bytes + nt * 8.0, 0.0, (double)p);
    }
    std::vector<double> lam(K);
    if (opts->lambda) {
        for (int k = 0; k < K; ++k) lam[k] = opts->lambda[k];
    } else {
        for (int k = 0; k < K; ++k)
            lam[k] = K == 1 ? lmax : lmax * std::pow(opts->lambda_min_ratio, (double)k / (double)(K - 1));
    }
    if (res->lambda)
        for (int k = 0; k < K; ++k) res->lambda[k] = lam[k];
    res->y_mean = ybar;
    res->lambda_max = lmax;
    res->jstar = jstar;

    // k = 0: beta = 0 when lambda_0 >= lambda_max (the grid's first point); a user grid may start lower
    HIPCHK(launch_fill_f64(beta, 0.0, p, st));
    HIPCHK(launch_sum_r(m, r, ctx->sc, true, st));
    // lens: [0] = |E|, [1],[2] = |S| slots, [3] = zero
    HIPCHK(hipMemsetAsync(lens, 0, 8 * 8, st));
    std::vector<int32_t> h_sweeps(K, 0), h_rounds(K, 0);
    std::vector<int64_t> h_viol(K, 0), h_recheck(K, 0);

    uint8_t* safe_cur = s0;
    uint8_t* safe_next = s1;
    double* zprev = a;       // z at the previous lambda (a at lambda_max)
    double* zcur = z0;
    double* zspare = z1;
    int64_t* len_cur = lens + 1;
    int64_t* len_next = lens + 2;
    bl_status final_status = BL_OK;

    // S_0 and its size
    HIPCHK(launch_bedpp(p, a, b, keep, bedpp, lmax, sgn, lam[0], bedpp_rhs(lmax, lam[0], v), safe_cur, st));
    HIPCHK(launch_compact(safe_cur, p, lT, len_cur, scr, st));
    int k_first = 0;
    if (history) {
        HIPCHK(launch_fill_u8((uint8_t*)zh, 0, (int64_t)3 * p * 4, st));
        HIPCHK(hipMemsetAsync(recn, 0, 8, st));
    }
    if (k_start > 0) {
        // resume at lambda_{k_start} from beta(lambda_{k_start - 1}) and its residual
        HIPCHK(hipMemcpyAsync(beta, opts->beta_init, p * 8, hipMemcpyDeviceToDevice, st));
        if (opts->r_init) {
            HIPCHK(hipMemcpyAsync(r, opts->r_init, nt * 8, hipMemcpyDeviceToDevice, st));
        } else if (xa.host) {
            return fail(ctx, BL_ERR_UNSUPPORTED, "X in host memory: resuming needs r_init");
        } else {
            // r = y~ - X~ beta over the nonzero coefficients (the strong-rule test with an infinite
            // threshold keeps the kept features with beta_j != 0)
            HIPCHK(launch_ssr(p, keep, nullptr, beta, nullptr, true, INFINITY, strong, st));
            HIPCHK(launch_compact(strong, p, lE, lens + 0, scr, st));
            HIPCHK(hipMemcpyAsync(&ctx->sc_host->n_new, lens + 0, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            const int64_t mz = ctx->sc_host->n_new;
            if (mz > 0) {
                double *g0, *b0, *b1, *part;
                ENSURE(B_G0, (mz + 1) * 8, g0);
                ENSURE(B_B0, (mz + 1) * 8, b0);
                ENSURE(B_B1, (mz + 1) * 8, b1);
                ENSURE(B_RUPART, r_update_scratch_bytes(nt, mz), part);
                HIPCHK(launch_gather_start(lE, mz, beta, beta, g0, b1, st));
                HIPCHK(launch_fill_f64(b0, 0.0, mz, st));
                HIPCHK(launch_r_update(m, lE, mz, b0, b1, c, sc_, part, r, st));
            }
        }
        HIPCHK(launch_sum_r(m, r, ctx->sc, true, st));
        // z at lambda_{k_start - 1} over S_{k_start}: the strong rule's input, as the uninterrupted path's
        // check scan at that lambda left it
        const double lr = lam[k_start];
        HIPCHK(launch_bedpp(p, a, b, keep, bedpp, lmax, sgn, lr, bedpp_rhs(lmax, lr, v), safe_next, st));
        HIPCHK(launch_compact(safe_next, p, lT, len_next, scr, st));
        ScanArgs za{};
        za.cols = lT;
        za.len_dev = len_next;
        za.r = r;
        za.sc = ctx->sc;
        za.c = c;
        za.s = sc_;
        za.keep = keep;
        za.z = z1;
        if ((s = x_scan(ctx, xa, za))) return s;
        zprev = z1;
        zcur = z0;
        k_first = k_start;
    } else if (lam[0] >= lmax) {
        HIPCHK(launch_record(nullptr, lens + 3, len_cur, lens + 3, beta, c, sc_, ctx->sc, lam[0], stats + 0, st));
        if (res->beta) HIPCHK(hipMemcpyAsync(res->beta, beta, p * 8, hipMemcpyDeviceToDevice, st));
        if (history) HIPCHK(launch_zhist_keep(keep, p, a, lam[0], zh, st));   // z at lambda_max is a
        k_first = 1;
    }
    const int k_row0 = k_start;   // first row of results this call writes
    for (int k = k_first; k < K; ++k) {
        const double lk = lam[k];
        const double lprev = k > 0 ? lam[k - 1] : lmax;
        // S_k (current) and S_{k+1} (scanned, feeds the strong rule at k+1)
        HIPCHK(launch_bedpp(p, a, b, keep, bedpp, lmax, sgn, lk, bedpp_rhs(lmax, lk, v), safe_cur, st));
        HIPCHK(launch_compact(safe_cur, p, lT, len_cur, scr, st));
        uint8_t* scan_mask = safe_cur;
        if (k + 1 < K) {
            const double ln = lam[k + 1];
            HIPCHK(launch_bedpp(p, a, b, keep, bedpp, lmax, sgn, ln, bedpp_rhs(lmax, ln, v), safe_next, st));
            scan_mask = safe_next;
        }
        HIPCHK(launch_compact(scan_mask, p, lT, len_next, scr, st));
        // working set E_k
        HIPCHK(launch_ssr(p, safe_cur, nullptr, beta, zprev, check, active_only ? INFINITY : (2.0 * lk - lprev) * alpha,
                          strong, st, pf));
        const int s1 = (k + 2) % 3, s2 = (k + 1) % 3, s3 = k % 3;   // slots of lambda_{k-1}, _{k-2}, _{k-3}
        if (history && k >= 3)
            HIPCHK(launch_learned(strong, beta, zh, p, s1, s2, s3, (float)(lk / lam[k - 1]), opts->mlp, tau_logit,
                                  learned ? 1 : 0, cand, st));
        HIPCHK(launch_compact(strong, p, lE, lens + 0, scr, st));
        int rounds = 0;
        int64_t viol_total = 0;
        int sweeps_total = 0;
        int64_t recheck_total = 0;
        for (;;) {
            HIPCHK(hipMemcpyAsync(&ctx->sc_host->n_new, lens + 0, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            const int64_t m_len = ctx->sc_host->n_new;
            double* zsrc = rounds == 0 ? zprev : zcur;
            if (lowp && m_len > 0) {
                // the solve starts from the exact gradient of its working set
                ScanArgs ea{};
                ea.cols = lE;
                ea.len_dev = lens + 0;
                ea.r = r;
                ea.sc = ctx->sc;
                ea.c = c;
                ea.s = sc_;
                ea.keep = keep;
                ea.z = zsrc;
                HIPCHK(launch_scan(m, ea, st));
                recheck_total += m_len;
            }
            bool cycled = false;
            if ((s = solve_ws(ctx, xa, lE, lens + 0, m_len, zsrc, beta, r, c, sc_, keep, (double)n, lk, opts->tol,
                              opts->max_sweeps, alpha, pf, scr, &cycled)))
                return s;
            HIPCHK(hipMemsetAsync(&ctx->sc->round.n_viol, 0, sizeof(uint32_t), st));
            if (!lowp) {
                ScanArgs ka{};
                ka.cols = lT;
                ka.len_dev = len_next;
                ka.r = r;
                ka.sc = ctx->sc;
                ka.c = c;
                ka.s = sc_;
                ka.keep = keep;
                ka.z = zcur;
                ka.check = check;
                ka.lam = lk * alpha;   // the check threshold lambda_k alpha w_j
                ka.w = pf;
                ka.in_s = safe_cur;
                ka.excl = strong;
                ka.mark = strong;
                ka.nviol = &ctx->sc->round.n_viol;
                ka.len_out = &ctx->sc->round.scan_len;
                prof_mark(ctx, 2);
                if ((s = x_scan(ctx, xa, ka))) return s;
                prof_mark(ctx, 3);
            } else {
                // matrix-core scan, then exact FP64 re-scans of the values near a threshold
                if (i8) {
                    HIPCHK(launch_r_pieces_i8(r, nt, (int8_t*)pieces, ctx->sc, st));
                    prof_mark(ctx, 2);
                    HIPCHK(launch_scan_i8(m, (const int8_t*)pieces, lT, len_next, 0, ctx->sc, c, sc_, keep, zcur, st));
                    prof_mark(ctx, 3);
                } else {
                    HIPCHK(launch_r_pieces(r, nt, (__bf16*)pieces, st));
                    prof_mark(ctx, 2);
                    HIPCHK(launch_scan_bf16(m, (const __bf16*)pieces, lT, len_next, 0, ctx->sc, c, sc_, keep, zcur,
                                            st));
                    prof_mark(ctx, 3);
                }
                prof_mark(ctx, 8);
                HIPCHK(hipMemcpyAsync(&ctx->sc->round.scan_len, len_next, sizeof(int64_t), hipMemcpyDeviceToDevice, st));
                HIPCHK(launch_fill_u8(flag, 0, p, st));
                const double thr2 = (ssr && k + 1 < K) ? 2.0 * lam[k + 1] - lk : -1.0;
                HIPCHK(launch_band(lT, len_next, zcur, c, sc_, ctx->sc, check ? lk : -1.0, safe_cur, strong, thr2, flag,
                                   nullptr, p, i8, st));
                HIPCHK(launch_compact(flag, p, lB, lens + 4, scr, st));
                ScanArgs ba{};
                ba.cols = lB;
                ba.len_dev = lens + 4;
                ba.r = r;
                ba.sc = ctx->sc;
                ba.c = c;
                ba.s = sc_;
                ba.keep = keep;
                ba.z = zcur;
                HIPCHK(launch_scan(m, ba, st));
                if (check) HIPCHK(launch_viol(lT, len_next, zcur, safe_cur, strong, lk, &ctx->sc->round.n_viol, p, st));
                prof_mark(ctx, 9);
                HIPCHK(hipMemcpyAsync(&ctx->sc_host->stage, lens + 4, sizeof(int64_t), hipMemcpyDeviceToHost, st));
            }
            HIPCHK(hipMemcpyAsync(&ctx->sc_host->round, &ctx->sc->round, sizeof(RoundInfo), hipMemcpyDeviceToHost, st));
            HIPCHK(hipStreamSynchronize(st));
            const RoundInfo ri = ctx->sc_host->round;
            if (cycled) {
                // recorded part by part in solve_ws
            } else if (ctx->last_residual) {
                prof_add(ctx, 0, BL_PROF_CD, (double)ri.sweeps * ri.cd_len * col_bytes, 0.0,
                         (double)ri.sweeps * ri.cd_len);
            } else {
                prof_add(ctx, 0, BL_PROF_CD, (double)ri.sweeps * (double)m_len * (double)m_len * 8.0, 0.0,
                         (double)ri.sweeps * (double)m_len);
                prof_add(ctx, 4, BL_PROF_GRAM, ctx->pend_gram_bytes);
                prof_add(ctx, 6, BL_PROF_RUPDATE, ctx->pend_ru_bytes);
            }
            prof_add(ctx, 2, BL_PROF_SCAN, (double)ri.scan_len * col_bytes + nt * 8.0, 0.0, (double)ri.scan_len);
            if (lowp) {
                const int64_t nb_ = ctx->sc_host->stage;
                recheck_total += nb_;
                prof_add(ctx, 8, BL_PROF_RECHECK, (double)nb_ * col_bytes);
            }
            ++rounds;
            sweeps_total += ri.sweeps;
            viol_total += ri.n_viol;
            if (ri.status == 2) {
                final_status = fail(ctx, BL_ERR_DEVICE, "CD workgroups timed out waiting for each other at lambda index %d", k);
                break;
            }
            if (ri.status != 0) {
                final_status = fail(ctx, BL_ERR_NOT_CONVERGED, "CD did not converge at lambda index %d", k);
                break;
            }
            if (ri.n_viol == 0) break;
            if (rounds >= opts->max_rounds) {
                final_status = fail(ctx, BL_ERR_NOT_CONVERGED, "check rounds exhausted at lambda index %d", k);
                break;
            }
            HIPCHK(launch_compact(strong, p, lE, lens + 0, scr, st));
        }
        if (final_status != BL_OK) break;
        h_sweeps[k] = sweeps_total;
        h_rounds[k] = rounds;
        h_viol[k] = viol_total;
        h_recheck[k] = recheck_total;
        HIPCHK(launch_record(lE, lens + 0, len_cur, len_next, beta, c, sc_, ctx->sc, lk, stats + k, st, alpha, pf));
        if (res->beta) HIPCHK(hipMemcpyAsync(res->beta + (size_t)k * p, beta, p * 8, hipMemcpyDeviceToDevice, st));
        if (recording && k >= 3) {
            HIPCHK(launch_compact(cand, p, lC, lens + 6, scr, st));
            HIPCHK(launch_rec_feat(lC, lens + 6, zh, p, s1, s2, s3, (float)(lk / lam[k - 1]), beta, opts->rec_cap,
                                   recn, opts->rec_feat, opts->rec_label, st));
        }
        if (history) {   // slot k mod 3 <- |z(lambda_k)| / lambda_k over the scanned columns
            float* slot = zh + (size_t)(k % 3) * p;
            HIPCHK(launch_fill_u8((uint8_t*)slot, 0, p * 4, st));
            HIPCHK(launch_zhist(lT, len_next, 0, zcur, lk, slot, p, st));
        }
        res->k_done = k + 1;
        // the scan at lambda_k is the strong-rule input at lambda_{k+1}
        zprev = zcur;
        zcur = (zcur == z0) ? z1 : z0;
        (void)zspare;
    }
    if (k_start == 0 && k_first == 1 && res->k_done < 1) res->k_done = 1;
    if (opts->r_out) HIPCHK(hipMemcpyAsync(opts->r_out, r, nt * 8, hipMemcpyDeviceToDevice, st));
    // results
    std::vector<LamStats> hs(K);
    HIPCHK(hipMemcpyAsync(hs.data(), stats, (size_t)K * sizeof(LamStats), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int k = k_row0; k < res->k_done; ++k) {
        if (res->intercept) res->intercept[k] = hs[k].intercept;
        if (res->rss) res->rss[k] = hs[k].rss;
        if (res->obj) res->obj[k] = hs[k].obj;
        if (res->n_active) res->n_active[k] = hs[k].n_active;
        if (res->sweeps) res->sweeps[k] = h_sweeps[k];
        if (res->rounds) res->rounds[k] = h_rounds[k];
        if (res->n_viol) res->n_viol[k] = h_viol[k];
        if (res->n_scanned) res->n_scanned[k] = hs[k].n_scan * h_rounds[k];
        if (res->n_recheck) res->n_recheck[k] = h_recheck[k];
        if (res->n_safe) res->n_safe[k] = hs[k].n_safe;
        if (res->n_strong) res->n_strong[k] = hs[k].n_strong;
    }
    if (recording) {
        HIPCHK(hipMemcpyAsync(&ctx->sc_host->stage, recn, 8, hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        res->n_recorded = ctx->sc_host->stage;
    }
    res->time_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
    return final_status;
}

}  // namespace

extern "C" {

bl_status bl_fit_path(bl_ctx ctx, const bl_matrix* X, const double* y, const bl_path_opts* opts,
                      bl_path_result* res) {
    bl_status s = check_ctx(ctx);
    if (s) return s;
    XAccess xa;
    if ((s = check_matrix(ctx, X, &xa.m))) return s;
    return fit_path_impl(ctx, xa, y, opts, res);
}

bl_status bl_fit_path_host(bl_ctx ctx, const bl_matrix* X, const double* y, const bl_path_opts* opts,
                           bl_host_stream* hs, bl_path_result* res) {
    bl_status s = check_ctx(ctx);
    if (s) return s;
    XAccess xa;
    if ((s = check_matrix(ctx, X, &xa.m))) return s;
    if (!opts || !res) return fail(ctx, BL_ERR_INVALID, "opts/res must be non-NULL");
    if (opts->precision != BL_PREC_FP64 || opts->rule == BL_SCREEN_LEARNED)
        return fail(ctx, BL_ERR_UNSUPPORTED, "X in host memory: FP64 scans and no learned rule");
    const size_t cb = (size_t)xa.m.ldx * (size_t)elem_bytes(xa.m.xtype);
    int64_t pc = hs && hs->panel_cols > 0 ? hs->panel_cols : (int64_t)std::max<size_t>(1, ((size_t)512 << 20) / cb);
    if (pc > xa.m.p) pc = xa.m.p;
    xa.host = true;
    xa.panel_cols = pc;
    xa.hs = hs;
    if (hs) {
        hs->panel_cols = pc;
        hs->panels_streamed = 0;
        hs->panels_skipped = 0;
        hs->bytes_streamed = 0.0;
    }
    // the context's Gram pool indexes the device cache of this X: start both empty
    return fit_path_impl(ctx, xa, y, opts, res);
}

}  // extern "C"
