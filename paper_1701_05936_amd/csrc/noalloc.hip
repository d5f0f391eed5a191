// bl_kkt_check_noalloc: the post-convergence check with no device allocation.  Its working memory is one
// file-scope device array per GPU; host code reaches it only through the address hipGetSymbolAddress
// returns for the current device, looked up once per device when a context is created on it.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "ctx.h"

using namespace blk;
using namespace blapi;

namespace {

// violator marks [BL_NOALLOC_MAX_P] | compaction counts | lengths
constexpr size_t NA_MARK = (size_t)BL_NOALLOC_MAX_P;
constexpr size_t NA_CMP_OFF = NA_MARK;
constexpr size_t NA_CMP = 8192;
constexpr size_t NA_LENS_OFF = NA_CMP_OFF + NA_CMP;
static_assert(BL_NOALLOC_BYTES >= NA_LENS_OFF + 64, "scratch array too small");

__device__ __align__(256) uint8_t scratch[BL_NOALLOC_BYTES];

constexpr int NA_MAX_DEV = 64;
std::mutex na_mu;
void* na_ptr[NA_MAX_DEV] = {};
hipError_t na_err[NA_MAX_DEV] = {};
bool na_done[NA_MAX_DEV] = {};

}  // namespace

namespace blapi {

// Once per device, with that device current: the device address of this GPU's copy of the array.
hipError_t noalloc_setup(int device) {
    if (device < 0 || device >= NA_MAX_DEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(na_mu);
    if (!na_done[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) (void)hipGetLastError();
        na_ptr[device] = e == hipSuccess ? p : nullptr;
        na_err[device] = e;
        na_done[device] = true;
    }
    return na_err[device];
}

}  // namespace blapi

extern "C" bl_status bl_kkt_check_noalloc(bl_ctx ctx, const bl_matrix* X, const double* center,
                                          const double* scale, const double* r, double lambda,
                                          const int32_t* check_set, int64_t len, const uint8_t* exclude, double* z,
                                          int32_t* violators, int64_t* n_viol) {
    bl_status s = check_ctx(ctx);
    if (s) return s;
    Mat m;
    if ((s = check_matrix(ctx, X, &m))) return s;
    if (!center || !scale || !r || !z || !violators) return fail(ctx, BL_ERR_INVALID, "array arguments must be non-NULL");
    if (m.p > BL_NOALLOC_MAX_P)
        return fail(ctx, BL_ERR_UNSUPPORTED, "p = %lld exceeds BL_NOALLOC_MAX_P = %d of the allocation-free check",
                    (long long)m.p, BL_NOALLOC_MAX_P);
    if (compact_scratch_bytes(m.p) > NA_CMP) return fail(ctx, BL_ERR_UNSUPPORTED, "compaction scratch too small");
    if (len < 0 || len > m.p) return fail(ctx, BL_ERR_INVALID, "len out of range");
    if (len > 0 && !check_set) return fail(ctx, BL_ERR_INVALID, "check_set is NULL");
    if (!(std::isfinite(lambda) && lambda >= 0.0)) return fail(ctx, BL_ERR_INVALID, "lambda must be finite and >= 0");
    const hipError_t se = noalloc_setup(ctx->device);
    if (se != hipSuccess)
        return fail(ctx, BL_ERR_DEVICE, "device address of the scratch array: %s", hipGetErrorString(se));
    uint8_t* base = (uint8_t*)na_ptr[ctx->device];
    uint8_t* mark = base;
    void* cmp = base + NA_CMP_OFF;
    int64_t* lens = (int64_t*)(base + NA_LENS_OFF);
    hipStream_t st = ctx->stream;
    // rows in the fit, into the context's scalars (allocated by bl_create)
    int64_t n = m.n_total;
    if (m.mask) {
        HIPCHK(launch_count_rows(m, &ctx->sc->n_rows, st));
        HIPCHK(hipMemcpyAsync(&ctx->sc_host->n_rows, &ctx->sc->n_rows, sizeof(int64_t), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        n = ctx->sc_host->n_rows;
        if (n < 1) return fail(ctx, BL_ERR_INVALID, "row_mask selects no rows");
    } else {
        ctx->sc_host->stage = n;
        HIPCHK(hipMemcpyAsync(&ctx->sc->n_rows, &ctx->sc_host->stage, sizeof(int64_t), hipMemcpyHostToDevice, st));
    }
    // the array keeps the last call's contents: clear what must start at zero, with fill kernels
    HIPCHK(launch_fill_u8(mark, 0, m.p, st));
    HIPCHK(launch_fill_u8((uint8_t*)&ctx->sc->round, 0, (int64_t)sizeof(RoundInfo), st));
    HIPCHK(launch_sum_r(m, r, ctx->sc, false, st));
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
        HIPCHK(launch_scan(m, sa, st));
    }
    HIPCHK(launch_compact(mark, m.p, violators, lens, cmp, st));
    HIPCHK(hipMemcpyAsync(&ctx->sc_host->stage, lens, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (n_viol) *n_viol = ctx->sc_host->stage;
    return BL_OK;
}
