// Context of libbl.so and helpers shared by the host-side drivers (api.cpp, api_batch.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "bl.h"
#include "internal.h"

struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
};

struct bl_ctx_s {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    blk::DevScalars* sc = nullptr;      // device
    blk::DevScalars* sc_host = nullptr; // pinned host mirror
    std::vector<DevBuf> bufs;
    // Gram pool of the covariance solve (features that have been in a working set)
    int64_t pool_size = 0;
    int64_t pool_cap = 0;
    double* gpool = nullptr;
    // Gram pools of the batched form (one per problem, common capacity)
    int64_t bpool_cap = 0;
    int bpool_np = 0;                    // problems the batched pools were allocated for
    double* bgpool = nullptr;
    void* bpinned = nullptr;            // pinned host staging of the batched driver
    hipStream_t aux = nullptr;          // library-owned stream for captured graphs
    // batched scan variant picked for the last shape (n_total, p, xtype)
    int64_t bscan_n = -1, bscan_p = -1;
    int bscan_x = -1, bscan_waves = 1;
    // limits of the coordinate-descent solve (bl_limits)
    int64_t cov_max = 0;                // largest working set of the covariance solve
    int cd_helpers = 0;                 // most helper workgroups of the multi-workgroup solve
    int cd_resident = 0;                // workgroups of that solve resident on the device at once
    int64_t cycle_min = INT64_MAX;      // working sets from this size on are solved by active-set cycling (off)
    bool last_residual = false;         // the last solve_set ran the residual-form solve
    // X in host memory: two device panel buffers streamed on `aux`, and the device cache of the columns
    // of the Gram pool's features
    void* panel[2] = {nullptr, nullptr};
    size_t panel_cap = 0;
    hipEvent_t ev_copy[2] = {}, ev_free[2] = {};
    bool panel_used[2] = {false, false};   // ev_free[b] marks the main stream's last use of panel b
    void* xcache = nullptr;
    double* xcache_c = nullptr;         // column centers and scales of the cached columns (pool order)
    double* xcache_s = nullptr;
    int64_t xcache_cap = 0;             // columns
    size_t xcache_cb = 0;               // bytes per cached column
    int64_t ident_len = 0;              // valid entries of the identity column list (H_IDENT)
    // kernel timing
    bool prof = false;
    hipEvent_t ev[10] = {};
    double pend_gram_bytes = 0.0, pend_ru_bytes = 0.0;  // bytes of the last solve, for the timing harvest
    bl_kernel_profile kp[BL_PROF_COUNT] = {};
};

namespace blapi {

enum BufId {
    B_CMP = 0, B_ARGV, B_ARGI, B_YT, B_R, B_XS, B_A, B_B, B_Z0, B_Z1, B_S0, B_S1, B_E, B_LT, B_LE, B_LENS,
    B_BETA, B_STATS, B_C, B_S, B_KEEP, B_MARK, B_POOLPOS, B_POOLLIST, B_GE, B_G0, B_B0, B_B1, B_RUPART, B_ZS,
    B_DELTA, B_SYNC, B_PIECES, B_LB,
    // batched form
    BB_MASKS, BB_MB, BB_Y, BB_YT, BB_R, BB_B, BB_S1, BB_S2, BB_C, BB_S, BB_KEEP, BB_A, BB_BB, BB_Z0, BB_Z1, BB_SAFE,
    BB_SAFEN, BB_STRONG, BB_UNION, BB_LT, BB_LE, BB_LENS, BB_LAM, BB_THR, BB_WANT, BB_BS, BB_BETA, BB_POS, BB_LIST,
    BB_GE, BB_G0, BB_B0, BB_B1, BB_STATS, BB_CMP, BB_LSAFE, BB_SAFECNT, BB_WANTALL,
    // learned form and its network
    B_ZH, B_CAND, B_RECN, B_LC, BB_KDEV, M_PART, M_LOSSP, M_MOM, M_VEL, M_STEP, M_PERM, M_LOSSH, M_PROB, M_HIST,
    // cross-validation
    CV_MASKS, CV_TEST, CV_Y, CV_ALL, CV_ROWS, CV_RLENS, CV_MARK, CV_ULIST, CV_ULENS, CV_FBETA, CV_PRED, CV_LOSS,
    CV_ICPT, CV_OUT, CV_CMP, CV_WANT, CV_LAM,
    // elastic net
    B_LAMV, B_PF, B_LMT,
    // X in host memory
    H_IDENT, H_SETC, H_COL,
    // logistic regression
    L_ETA, L_G, L_R0C,
    // batched BF16 scans
    BB_RP, BB_FLAG, BB_LF, BB_LU, BB_PART, BB_BFPART, BB_BSPART,
    // active-set cycling
    B_CYCF, B_CYCL, B_CYCN, B_ZCYC,
    B_COUNT
};

bl_status fail(bl_ctx c, bl_status st, const char* fmt, ...);
bl_status ensure(bl_ctx ctx, int id, size_t bytes, void** out);
int elem_bytes(int xtype);
bl_status check_ctx(bl_ctx ctx);
bl_status check_matrix(bl_ctx ctx, const bl_matrix* X, blk::Mat* m);
void prof_mark(bl_ctx ctx, int slot);
hipError_t noalloc_setup(int device);   // device address of the allocation-free check's array (noalloc.hip)
void prof_add(bl_ctx ctx, int slot, int which, double bytes, double flops = 0.0, double units = 0.0);

}  // namespace blapi

#define HIPCHK(expr)                                                                                        \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess) return blapi::fail(ctx, BL_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define ENSURE(id, bytes, ptr)                                                  \
    do {                                                                        \
        void* p_;                                                               \
        bl_status s_ = blapi::ensure(ctx, (id), (size_t)(bytes), &p_);          \
        if (s_ != BL_OK) return s_;                                             \
        (ptr) = (decltype(ptr))p_;                                              \
    } while (0)
