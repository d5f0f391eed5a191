/*
 * bl.h -- C ABI of the GPU pathwise-lasso library (libbl.so) for AMD CDNA4 (gfx950).
 *
 * The library computes the lasso solution path with implicit standardization,
 * hybrid safe-strong screening (BEDPP + sequential strong rule) and a
 * post-convergence check, as described by Zeng & Breheny, "The biglasso
 * Package" (arXiv:1701.05936), Sections 2.2 and 3.1.
 *
 * Problem (standardized scale; the paper standardizes X, Section 3.1):
 *   minimize over beta  Q(beta; lambda) = ||y~ - X~ beta||^2 / (2n) + lambda ||beta||_1
 *   x~_ij = (x_ij - c_j) / s_j   (c_j column mean, s_j column SD with divisor n, over the fitted rows)
 *   y~_i  = y_i - mean(y)        (the intercept is unpenalized)
 * z_j(r) = x~_j' r / n is the standardized correlation of column j with a residual r.
 *
 * General conventions
 *   - Every array argument is a DEVICE pointer unless the comment says "host".
 *     The caller allocates and owns every array.  Scalar outputs are host pointers.
 *   - X is column-major: element (i, j) at X[i + j*ldx], ldx >= n_total.
 *   - Vectors over rows (y, y~, r) have n_total entries.  Rows outside the fit
 *     (row_mask[i] == 0) must hold 0 in residual vectors; the library writes 0 there.
 *   - All work is enqueued on the context's HIP stream.  A call returns after
 *     its host-visible (scalar) outputs are available; device outputs are then
 *     also complete.
 *   - Errors are return codes; bl_last_error() gives the message.  Arguments
 *     are validated on the host before anything is launched.  On error, device
 *     outputs are unspecified (bl_fit_path: see k_done).
 *   - Calls on one context must not overlap (one host thread at a time).
 */
#ifndef BL_H
#define BL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bl_ctx_s* bl_ctx;

typedef enum {
    BL_OK = 0,
    BL_ERR_INVALID = 1,        /* bad argument (null pointer, size, NaN/Inf scalar, misaligned X ...) */
    BL_ERR_NOMEM = 2,          /* device scratch allocation failed                                     */
    BL_ERR_DEVICE = 3,         /* a HIP call failed                                                    */
    BL_ERR_NOT_CONVERGED = 4,  /* coordinate descent hit max_sweeps                                    */
    BL_ERR_UNSUPPORTED = 5     /* valid request outside what this build handles (e.g. n_total too big) */
} bl_status;

typedef enum {
    BL_X_F64 = 0,   /* double                                      */
    BL_X_F32 = 1,   /* float                                       */
    BL_X_I8 = 2     /* int8 codes (e.g. genotypes 0, 1, 2), exact   */
} bl_xtype;

typedef enum {
    BL_SCREEN_NONE = 0,       /* working set = every kept feature                                   */
    BL_SCREEN_SSR = 1,        /* sequential strong rule + check over all kept features              */
    BL_SCREEN_BEDPP = 2,      /* safe rule only: working set = BEDPP survivors, check over them     */
    BL_SCREEN_SSR_BEDPP = 3,  /* hybrid (default): strong rule and check restricted to BEDPP survivors */
    BL_SCREEN_LEARNED = 4,    /* hybrid + screening network: from the fourth lambda on, a strong-rule candidate
                                 outside the previous active set enters the working set only if the network
                                 scores it at or above opts->mlp_tau; the check over all BEDPP survivors is unchanged
                                 and adds every violator back, so the solution is the hybrid rule's       */
    BL_SCREEN_ACTIVE = 5      /* working set = previous active set (within the BEDPP survivors) only: no strong
                                 rule, so every feature that enters the path is found by the check over the
                                 BEDPP survivors and added back (Section 2.2: the check is what makes a
                                 heuristic screen exact).  Slow on purpose; it exercises the repair loop.  */
} bl_screen_rule;

/* Design matrix.  X must be 16-byte aligned when ldx*sizeof(element) is a multiple of 16;
 * otherwise the library uses element-wise loads (slower, still correct). */
typedef struct {
    const void* X;             /* device, column-major, n_total x p, leading dimension ldx        */
    int32_t xtype;             /* bl_xtype                                                        */
    int64_t n_total;           /* rows stored                                                     */
    int64_t p;                 /* columns                                                         */
    int64_t ldx;               /* leading dimension (elements), >= n_total                        */
    const uint8_t* row_mask;   /* device [n_total], 1 = row is in the fit; NULL = all rows.
                                  Cross-validation fits pass a mask instead of copying X (Section 3.1.2). */
} bl_matrix;

/* Create a context on `device` ordinal using `hip_stream` (hipStream_t; NULL = default stream). */
bl_status bl_create(bl_ctx* ctx, int device, void* hip_stream);
void bl_destroy(bl_ctx ctx);
const char* bl_last_error(bl_ctx ctx);
/* Number of compute units and the device name the context runs on (host outputs). */
bl_status bl_device_info(bl_ctx ctx, int* n_cu, char* name, int name_len);

/*
 * Size limits of the coordinate-descent solve (host struct, read and written by value).
 *   cov_max     largest working set solved in covariance form; larger sets run the residual-form
 *               solve.  Default 16,320; 0 keeps the current value.
 *   cd_helpers  most helper workgroups the multi-workgroup covariance solve may launch besides its
 *               leader.  Every workgroup of that solve must be resident at once, so bl_create sets
 *               it to (workgroups of that kernel resident per compute unit) x (compute units) - 1,
 *               at most 255.  Sets whose multi-workgroup solve would need more helpers run the
 *               single-workgroup solve (up to 7,168 features) or else the residual-form solve.
 *               A value above the resident count is rejected (BL_ERR_INVALID); -1 keeps the current.
 *   resident    out: workgroups of the multi-workgroup solve that fit on the device at once.
 *   cycle_min   working sets of bl_fit_path (squared loss) with at least this many features are solved
 *               by active-set cycling (Section 3.1.1: the descent iterates over the nonzero
 *               coefficients): sweeps over A = {j in E : beta_j != 0} until none changes a coefficient
 *               by tol, then one sweep over E, repeated until a sweep over E changes none by tol (the
 *               plain solve's stopping rule; the reported sweeps count both kinds).  Smaller sets
 *               sweep E throughout.  Default -1 (off): on the genotype designs measured, cycling took
 *               more coordinate updates in all than sweeping E (13.2 against 9.1 million on a
 *               5,000 x 500,000 path).  0 keeps the current value; -1 turns cycling off.
 */
typedef struct {
    int64_t cov_max;
    int32_t cd_helpers;
    int32_t resident;
    int64_t cycle_min;
} bl_limits;

bl_status bl_get_limits(bl_ctx ctx, bl_limits* out);
bl_status bl_set_limits(bl_ctx ctx, const bl_limits* in);

/*
 * Column centers and scales over the fitted rows (Section 3.1: only c and s are
 * kept, X~ is never formed).  center[j] = mean, scale[j] = SD with divisor n,
 * keep[j] = scale[j] > 1e-6 (constant columns are left out of the fit).
 * Int8 X: sums are exact integers.  n_rows (host, may be NULL) = rows in the fit.
 * Outputs: center, scale (double [p]), keep (uint8 [p]).
 */
bl_status bl_standardize(bl_ctx ctx, const bl_matrix* X, double* center, double* scale, uint8_t* keep,
                         int64_t* n_rows);

/*
 * lambda_max (Section 3.1.1, type (2) products): y_mean = mean of y over the fit,
 * ytilde = y - y_mean on fitted rows and 0 elsewhere, a[j] = z_j(ytilde)
 * (0 for columns not kept), lambda_max = max_j |a_j|, jstar = smallest j attaining it.
 * beta = 0 is the solution for every lambda >= lambda_max.
 * Inputs: y [n_total].  Outputs: ytilde [n_total], a [p]; y_mean, lambda_max, jstar are host.
 * Returns BL_ERR_INVALID if no column is kept.
 */
bl_status bl_lambda_max(bl_ctx ctx, const bl_matrix* X, const double* center, const double* scale,
                        const uint8_t* keep, const double* y, double* ytilde, double* a, double* y_mean,
                        double* lambda_max, int64_t* jstar);

/*
 * One-time inputs of the BEDPP safe rule (Section 2.2; Section 3.1.1 type (1)):
 * b[j] = x~_j' x~_* / n with x~_* the column jstar, and v = ||ytilde||^2 / n (host).
 */
bl_status bl_bedpp_setup(bl_ctx ctx, const bl_matrix* X, const double* center, const double* scale,
                         const uint8_t* keep, const double* ytilde, int64_t jstar, double* b, double* v);

/* State the screening rules read (all device arrays have p entries). */
typedef struct {
    int64_t p;
    int32_t rule;              /* bl_screen_rule                                            */
    const double* a;           /* z_j(ytilde)                                               */
    const double* b;           /* BEDPP b_j                                                 */
    const uint8_t* keep;       /* kept columns                                              */
    const uint8_t* active;     /* beta_j != 0 at the previous lambda (uint8), or NULL       */
    double lambda_max;
    double sign_star;          /* sign(a[jstar]), +1 or -1                                   */
    double v;                  /* ||ytilde||^2 / n                                          */
} bl_screen_state;

/*
 * Screening at lambda_k (Section 2.2):
 *   safe[j]   = 1 unless BEDPP discards j at lambda_k (always 1 for kept j when the
 *               rule has no BEDPP part; 0 for columns not kept).  BEDPP discards j when
 *               |(lm + l) a_j - (lm - l) sign_star lm b_j| < 2 l lm - (lm - l) sqrt(max(0, v - lm^2)).
 *   strong[j] = safe[j] and (active[j] or |z_prev[j]| >= 2 lambda_k - lambda_prev)
 *               (strong rule; for rule NONE or BEDPP: strong = safe).
 * z_prev [p] holds z at lambda_prev (only read where safe[j] = 1).
 * n_safe, n_strong: host counts.
 */
bl_status bl_screen(bl_ctx ctx, const bl_screen_state* st, double lambda_k, double lambda_prev,
                    const double* z_prev, uint8_t* safe, uint8_t* strong, int64_t* n_safe, int64_t* n_strong);

/*
 * Cyclic coordinate descent at fixed lambda (Section 1: the pathwise coordinate descent the
 * package is built on; Section 3.1.1: its inner products are type (3), x~_j' r, computed from raw
 * X with the stored c and s) over the features set[0..set_len-1] (visited in that order; int32
 * indices into 0..p-1, distinct, kept), warm-started from beta [p] and its residual
 * r [n_total] = ytilde - X~ beta, both updated in place.
 * Coordinate step: u = z_j(r) + beta_j, beta_j' = S(u, lambda), r -= (beta_j' - beta_j) x~_j.
 * Stops when the largest |beta_j' - beta_j| of a sweep is < tol.  sweeps (host) = sweeps run.
 * Returns BL_ERR_NOT_CONVERGED after max_sweeps sweeps (beta, r are then the last iterate).
 * Working sets up to bl_limits.cov_max features are solved in covariance form (Gram entries of the
 * set, type (1) products); larger sets update r after every coordinate, which this build supports
 * for n_total <= 16384 only (BL_ERR_UNSUPPORTED otherwise).
 */
bl_status bl_cd_solve(bl_ctx ctx, const bl_matrix* X, const double* center, const double* scale,
                      double lambda, const int32_t* set, int64_t set_len, double* beta, double* r, double tol,
                      int32_t max_sweeps, int32_t* sweeps);

/*
 * Post-convergence check (Sections 2.2 and 3.1.1, type (3)): for every j in
 * check_set[0..len-1] (int32, ascending) compute
 *   z[j] = (x_j' r - c_j sum(r)) / (n s_j)
 * (sum(r) is computed once per call) and collect the violators
 *   { j in check_set : exclude[j] == 0 and |z[j]| > lambda }
 * into violators[0..n_viol-1] in ascending order.  exclude [p] may be NULL
 * (nothing excluded).  z entries outside check_set are left untouched.
 * violators must have room for len entries; n_viol is host.
 */
bl_status bl_kkt_check(bl_ctx ctx, const bl_matrix* X, const double* center, const double* scale,
                       const double* r, double lambda, const int32_t* check_set, int64_t len,
                       const uint8_t* exclude, double* z, int32_t* violators, int64_t* n_viol);

/*
 * bl_kkt_check for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the same arguments, semantics and outputs as
 * bl_kkt_check, with no allocation of any kind.  Its working memory (violator marks, compaction counts,
 * lengths) is one fixed device array of BL_NOALLOC_BYTES bytes per GPU that the library holds until the
 * process ends; its device address is looked up when a context is created on that GPU.
 * p <= BL_NOALLOC_MAX_P (BL_ERR_UNSUPPORTED beyond).  Every call on one GPU shares that array and it
 * keeps the last call's contents (each call clears what it needs): calls that overlap on one GPU, from two
 * contexts or two host threads, race and must be serialized by the caller.
 */
#define BL_NOALLOC_MAX_P 4194304
#define BL_NOALLOC_BYTES (BL_NOALLOC_MAX_P + 8192 + 256)
bl_status bl_kkt_check_noalloc(bl_ctx ctx, const bl_matrix* X, const double* center, const double* scale,
                               const double* r, double lambda, const int32_t* check_set, int64_t len,
                               const uint8_t* exclude, double* z, int32_t* violators, int64_t* n_viol);

/* Arithmetic of the check scans. */
typedef enum {
    BL_PREC_FP64 = 0,      /* FP64 vector scan (any X type)                                          */
    BL_PREC_BF16X3 = 1,    /* int8 X: BF16 matrix cores against three BF16 pieces of the residual,
                              FP32 chunks promoted to FP64; decisions within the error bound are
                              re-taken on the FP64 scan, so they equal the FP64 decisions.
                              Batched form, f32 X: x and r each in three BF16 pieces, six products */
    BL_PREC_I8X4 = 2,      /* int8 X only: int8 dot products against four int8 pieces of the residual
                              with power-of-two scales, exact integer sums; decisions within the
                              error bound are re-taken on the FP64 scan, as for BL_PREC_BF16X3       */
    BL_PREC_BF16X2 = 3     /* batched form, f32 X only: x and r each in two BF16 pieces, three products
                              (bound about 5e-5 against 7e-6 for BF16X3: a wider band of FP64
                              re-scans for half the matrix-core work); decisions as the FP64 scan's  */
} bl_precision;

/*
 * The scan alone (Section 3.1.1, type (3)): z[j] = (x_j' r - c_j sum(r)) / (n s_j) for j in
 * cols[0..len-1], in the given precision.  For BL_PREC_BF16X3, err[j] (device, may be NULL)
 * receives the bound on |z[j] - exact| the precision form guarantees:
 *   err_j = (u_r + (1 + 2^-7) gc + g64) sqrt(n (s_j^2 + c_j^2)) ||r||_2 / (n s_j),
 *   u_r = (2^-8 + 2^-24)^3 (residual left after three BF16 pieces, relative to |r_i|),
 *   gc = 64 u / (1 - 64 u), u = 2^-24 (FP32 chunks of 64 rows), g64 = 65536 * 2^-53 (FP64 sums of up
 *   to 2^16 chunk and piece terms; n_total <= 2^21),
 * plus 1e-14 |z_j|.  For BL_PREC_I8X4 the residual is r = sum_k s_k q_k + t with int8 pieces q_1..q_4,
 * s_1 = 2^E the smallest power of two with max|r_i| <= 127 s_1 and s_{k+1} = s_k / 128, and
 *   err_j = ((||t||_2 + g3 ||w||_2)(1 + 2^-20) + g64 ||r||_2) sqrt(n (s_j^2 + c_j^2)) / (n s_j) + 1e-14 |z_j|,
 *   w_i = sum_k s_k |q_ik|, g3 = 3 u / (1 - 3 u), u = 2^-53 (the FP64 sum of the four exact integer
 *   dot products), g64 as above.  The I8X4 scan reads columns in whole 16-byte words: the bytes after
 *   row n_total - 1 in the aligned word that holds it are read and multiplied by zero pieces.
 * BL_ERR_UNSUPPORTED for BF16X3 and I8X4 unless X is int8 with 16-byte aligned columns (X pointer
 * and ldx a multiple of 16) and n_total <= 2^21.
 */
bl_status bl_scan(bl_ctx ctx, const bl_matrix* X, const double* center, const double* scale, const double* r,
                  const int32_t* cols, int64_t len, int32_t precision, double* z, double* err);

/* Options of bl_fit_path. */
typedef struct {
    int32_t nlambda;           /* K >= 1                                                      */
    double lambda_min_ratio;   /* 0 < ratio < 1; grid lambda_k = lambda_max ratio^(k/(K-1))   */
    const double* lambda;      /* host [K] user grid (decreasing, positive) or NULL           */
    int32_t rule;              /* bl_screen_rule                                              */
    double tol;                /* CD stop: largest |coefficient change| in a sweep < tol       */
    int32_t max_sweeps;        /* per CD solve                                                */
    int32_t max_rounds;        /* CD + check rounds per lambda before giving up (>= 1)        */
    int32_t precision;         /* bl_precision of the check scans                              */
    /* learned form (rule BL_SCREEN_LEARNED): network parameters and score threshold in (0, 1)   */
    const float* mlp;          /* DEVICE [BL_MLP_NPARAMS] or NULL                              */
    double mlp_tau;
    /* training records (any rule with the strong rule): for k >= 3 and every strong-rule candidate
     * j outside the active set of lambda_{k-1}, features
     *   ( |z_j(k-1)|/lambda_{k-1}, |z_j(k-2)|/lambda_{k-2}, |z_j(k-3)|/lambda_{k-3}, lambda_k/lambda_{k-1} )
     * (a |z| that was not scanned at that lambda counts as 0) and label 1 if beta_j(lambda_k) != 0.
     * Appended in lambda order, feature order within a lambda, until rec_cap records.            */
    float* rec_feat;           /* DEVICE [rec_cap x 4] or NULL                                  */
    float* rec_label;          /* DEVICE [rec_cap] or NULL                                      */
    int64_t rec_cap;
    /* resume (warm starts, Section 1): k_start = 0 runs the whole path.  k_start >= 1 starts at lambda
     * index k_start from beta_init = beta(lambda_{k_start - 1}) (DEVICE [p], standardized scale, the row
     * the earlier call wrote) and, if r_init is not NULL, its residual (DEVICE [n_total], rows outside
     * the fit 0).  Given the residual the earlier call ended that lambda with, the resumed rows are
     * bit-identical to the uninterrupted call's; with r_init NULL the residual is recomputed from
     * beta_init (equal up to rounding).  Results are written for k >= k_start only; k_done counts from
     * 0.  Not with the learned rule or training records (they need the history of earlier lambdas). */
    int32_t k_start;
    const double* beta_init;
    const double* r_init;
    double* r_out;             /* DEVICE [n_total] or NULL: the residual at the last finished lambda  */
    /* elastic net and penalty factors (Section 1: the package fits lasso and elastic-net penalties): the
     * penalty becomes lambda sum_j w_j (alpha |beta_j| + (1 - alpha) beta_j^2 / 2).  alpha in (0, 1]
     * (0 is read as 1, the lasso); penalty_factor = w, DEVICE [p] of finite w_j > 0, or NULL (all 1).
     * Then lambda_max = max_j |a_j| / (alpha w_j), the strong rule keeps j when |z_j(k-1)| >= alpha w_j
     * (2 lambda_k - lambda_{k-1}), a violation is |z_j| > lambda_k alpha w_j, the CD step is
     * S(u, lambda alpha w_j) / (1 + lambda (1 - alpha) w_j), and obj is the elastic-net objective.
     * BEDPP is a lasso rule: with alpha < 1 or weights the rules run without it (BEDPP alone keeps every
     * feature).  Not with the precision forms, the learned rule or the batched form (BL_ERR_UNSUPPORTED). */
    double alpha;
    const double* penalty_factor;
    /* model family: BL_FAMILY_GAUSSIAN (0, the lasso above) or BL_FAMILY_BINOMIAL (lasso-penalized logistic
     * regression, y in {0, 1}; see bl_fit_path) */
    int32_t family;
} bl_path_opts;

enum { BL_FAMILY_GAUSSIAN = 0, BL_FAMILY_BINOMIAL = 1 };

/* Results of bl_fit_path.  Host arrays have K entries; any pointer may be NULL (not written). */
typedef struct {
    double* beta;              /* DEVICE [K x p] row k = beta(lambda_k), standardized scale   */
    double* center;            /* DEVICE [p]                                                   */
    double* scale;             /* DEVICE [p]                                                   */
    uint8_t* keep;             /* DEVICE [p]                                                   */
    double* lambda;            /* host: grid used                                             */
    double* intercept;         /* host: y_mean - sum_j c_j beta_j / s_j (original scale)     */
    double* rss;               /* host: ||r||^2                                               */
    double* obj;               /* host: Q(beta; lambda_k)                                      */
    int32_t* sweeps;           /* host: CD sweeps summed over rounds                          */
    int32_t* rounds;           /* host: CD solves (0 at k = 0)                                 */
    int64_t* n_active;         /* host: nonzero coefficients                                  */
    int64_t* n_strong;         /* host: size of the working set after the last round          */
    int64_t* n_safe;           /* host: BEDPP survivors (p - safe rejections)                  */
    int64_t* n_viol;           /* host: features the check added back                          */
    int64_t* n_scanned;        /* host: columns scanned by checks at this lambda               */
    int64_t* n_recheck;        /* host: precision form: columns re-scanned in FP64 (band + set) */
    double y_mean;             /* out                                                          */
    double lambda_max;         /* out                                                          */
    int64_t jstar;             /* out                                                          */
    int32_t k_done;            /* out: lambdas finished (results valid for k < k_done)         */
    double time_ms;            /* out: wall time of the call                                   */
    int64_t n_recorded;        /* out: training records written (opts->rec_feat)              */
} bl_path_result;

/*
 * The whole lasso path (Sections 2.2 and 3): standardize, lambda_max, BEDPP set-up,
 * then for k = 1..K-1 with warm starts:
 *   S_k   = BEDPP survivors at lambda_k (grows along the path);
 *   E_k   = active(k-1) u { j in S_k : |z_j(k-1)| >= 2 lambda_k - lambda_{k-1} };
 *   repeat: CD over E_k; scan z over S_{k+1} (which contains S_k);
 *           V = { j in S_k \ E_k : |z_j| > lambda_k }; stop if V is empty; E_k u= V.
 * The scan at lambda_k also supplies the strong-rule input for lambda_{k+1}.
 * y [n_total] device.  Returns BL_ERR_NOT_CONVERGED if CD or max_rounds gave out
 * (res->k_done tells how far the path got).
 *
 * family BL_FAMILY_BINOMIAL (Section 1: sparse logistic regression; Section 2.2: its hybrid rule pairs the
 * strong rule with a safe rule): y_i in {0, 1} on the fitted rows (both values present), eta = b0 + X~ beta,
 *   Q(b0, beta) = (1/n) sum_i [log(1 + e^eta_i) - y_i eta_i] + lambda ||beta||_1, b0 unpenalized,
 * z_j = x~_j' (y - pi) / n with pi = 1/(1 + e^-eta) in the strong rule and the check, lambda_max =
 * max |x~_j'(y - y_mean)| / n.  The safe part of rules BEDPP / SSR_BEDPP is the gap-safe sphere around the
 * dual point known exactly at lambda_max: j is discarded at lambda when |a_j| < lambda_max (1 - sqrt(G / (2 n))
 * / lambda), G the duality gap of (logit(y_mean), 0) at lambda (Slores, the rule the paper names, is not printed
 * in it).  Each solve majorizes the loss with curvature 1/4 and minimizes the bound with the lasso coordinate
 * descent (threshold 4 lambda on the residual 4 (y - pi), intercept stepped by the residual's mean) until a
 * majorization step changes no coefficient by tol.  Outputs: intercept = original-scale intercept, rss = the
 * deviance 2 sum_i [log(1 + e^eta_i) - y_i eta_i], obj = Q, y_mean = mean of y.  FP64 scans, lasso penalty,
 * no learned rule or resume (BL_ERR_UNSUPPORTED).
 */
bl_status bl_fit_path(bl_ctx ctx, const bl_matrix* X, const double* y, const bl_path_opts* opts,
                      bl_path_result* res);

/*
 * The path with X in host memory (Section 2.1: the package keeps X, which may exceed RAM, in a memory-
 * mapped file and streams what each step needs; here X may exceed the GPU's memory and stays in host
 * memory).  X->X is a HOST pointer: memory from hipHostMalloc (pinned) moves at full PCIe speed, pageable
 * memory works but slower.  y, X->row_mask and every output are device arrays as for bl_fit_path.  Column
 * panels of hs->panel_cols columns (0: about 512 MB per panel) are copied to the device on a library stream,
 * two in flight, while the previous panel is scanned: the set-up passes stream every panel, and each check
 * scan only the panels holding a BEDPP survivor (panels of discarded features are never moved).  Columns
 * that enter a working set are kept in a device cache, which their Gram entries and the residual updates
 * read.  The results equal bl_fit_path's on the same X in device memory bit for bit.  FP64 scans only, no
 * learned rule; working sets must stay within the covariance solve's limits (bl_limits), and a resume
 * needs r_init (BL_ERR_UNSUPPORTED otherwise).  hs (may be NULL) receives the streaming counters.
 */
typedef struct {
    int64_t panel_cols;        /* in: columns per panel (0: about 512 MB); out: the value used           */
    int64_t panels_streamed;   /* out: panel copies to the device                                        */
    int64_t panels_skipped;    /* out: panels scans did not need (no listed column in them)               */
    double bytes_streamed;     /* out: host-to-device bytes (panels, cached columns, the BEDPP column)    */
} bl_host_stream;

bl_status bl_fit_path_host(bl_ctx ctx, const bl_matrix* X, const double* y, const bl_path_opts* opts,
                           bl_host_stream* hs, bl_path_result* res);

/*
 * Batched form: nprob <= 64 lasso problems over one design matrix (Section 3.1.2:
 * cross-validation fits and several responses share X; each problem selects its
 * rows with its own mask instead of copying X).  Problem b has its own response,
 * rows, standardization, lambda grid (its own lambda_max, the ratio of opts),
 * screening sets and coefficients.  The problems advance through their grids in
 * lockstep; every pass over X (column statistics, lambda_max and BEDPP products,
 * post-convergence scans) serves all problems at once on FP64 matrix cores.  The screening
 * kernels of a lambda step are captured once per call in a HIP graph and replayed.
 * Options as bl_fit_path (no learned rule, resume, elastic net or penalty factors); X->row_mask must
 * be NULL; X is f32 or f64.  opts->precision: BL_PREC_FP64 (FP64 matrix cores), or for f32 X
 * BL_PREC_BF16X3 / BL_PREC_BF16X2, the check scans on BF16 matrix cores with x and r split into
 * three / two BF16 pieces; every (column, problem) whose z lies within the scan's error bound of a
 * threshold the path decides on (this check, the next strong rule) is re-scanned in FP64, and every
 * solve starts from FP64 gradients of its working set, so coefficients and counts are bit-identical to
 * the FP64 form's.  opts->lambda NULL gives each problem its own grid from its own lambda_max; a host grid
 * (K decreasing values) is shared by every problem, as cross-validation needs (Section 3.1.2), and is
 * solved from its first point (beta = 0 where that point is at or above the problem's lambda_max).
 */
typedef struct {
    int32_t nprob;             /* 1..64                                                                */
    const double* Y;           /* DEVICE [nprob x n_total]: response of problem b at Y[b*n_total + i]   */
    const uint8_t* masks;      /* DEVICE [nprob x n_total]: 1 = row i is in problem b's fit; NULL = all */
    int32_t flags;             /* BL_BATCH_EAGER: launch each lambda step's screening kernels one by one
                                  instead of replaying the captured HIP graph (same results)            */
} bl_batch;

enum { BL_BATCH_EAGER = 1 };

typedef struct {
    double* beta;              /* DEVICE [nprob x K x p] (problem-major, then lambda) or NULL           */
    double* lambda;            /* host [nprob x K]                                                     */
    double* intercept;         /* host [nprob x K]                                                     */
    double* rss;               /* host [nprob x K]                                                     */
    double* obj;               /* host [nprob x K]                                                     */
    int32_t* sweeps;           /* host [nprob x K]                                                     */
    int32_t* rounds;           /* host [nprob x K]                                                     */
    int64_t* n_active;         /* host [nprob x K]                                                     */
    int64_t* n_strong;         /* host [nprob x K]                                                     */
    int64_t* n_safe;           /* host [nprob x K]                                                     */
    int64_t* n_viol;           /* host [nprob x K]                                                     */
    int32_t k_done;            /* out: lambda indices finished by every problem                        */
    double time_ms;            /* out                                                                  */
    int32_t scan_cols;         /* out: columns per workgroup of the shared scan, picked by timing the
                                  candidates (64, 128, 256, with or without register prefetch) on this
                                  shape once per context; with the environment variable
                                  BL_AUTOTUNE_CACHE naming a file, the pick is read from it (one line
                                  "bscan <arch> <xtype> <n_total> <p> <variant>" per shape) and a new
                                  shape's pick appended, so later processes skip the timing            */
} bl_batch_result;

bl_status bl_fit_path_batch(bl_ctx ctx, const bl_matrix* X, const bl_batch* batch, const bl_path_opts* opts,
                            bl_batch_result* res);

/*
 * K-fold cross-validation of the lasso path (Section 3.1.2: every fold is a row subset of the one X, chosen
 * by a mask, never a copy; Section 5.2: the cross-validation curve with standard errors and the lambda at
 * its minimum).  The grid comes from the full data, the rows with fold >= 0: their path is fitted first
 * (bl_fit_path, written to res->beta when not NULL).  Fold f is then fitted on the rows with fold >= 0
 * and fold != f over that same grid, all folds in one bl_fit_path_batch call, and predicts its held-out
 * rows (fold == f) on the original scale:
 *   y^_i(lambda_k) = intercept_fk + sum_j x_ij beta_fkj / s_fj     (s_fj: column SD over fold f's rows)
 *   loss_ik = (y_i - y^_i(lambda_k))^2 over the N rows with fold >= 0
 *   cve_k = mean_i loss_ik,  cvse_k = sqrt(sum_i (loss_ik - cve_k)^2 / (N - 1)) / sqrt(N)
 *   fold_err[f*K + k] = mean of loss_ik over the rows of fold f
 *   k_min = the first k with the smallest cve_k (lambda.min); k_1se = the smallest k (largest lambda)
 *           with cve_k <= cve_kmin + cvse_kmin.
 * X: f32 or f64, row_mask NULL.  Options as bl_fit_path_batch (opts->lambda NULL: the grid is
 * lambda_max ratio^(k/(K-1)) of the full data; else that host grid).  Every fold must hold a row.
 */
typedef struct {
    int32_t nfolds;            /* 2..64                                                                 */
    const int32_t* fold;       /* DEVICE [n_total]: fold of row i in 0..nfolds-1, or -1 (row left out)  */
    const double* y;           /* DEVICE [n_total]                                                      */
} bl_cv;

typedef struct {
    double* beta;              /* DEVICE [K x p] or NULL: the full-data path, standardized scale          */
    double* fold_beta;         /* DEVICE [nfolds x K x p] or NULL: each fold's path on its own scale      */
    double* pred;              /* DEVICE [K x n_total] or NULL: held-out predictions (0 where fold = -1)  */
    double* lambda;            /* host [K]                                                               */
    double* cve;               /* host [K]                                                               */
    double* cvse;              /* host [K]                                                               */
    double* fold_err;          /* host [nfolds x K]                                                      */
    int32_t k_min;             /* out */
    int32_t k_1se;             /* out */
    double lambda_min;         /* out */
    double lambda_1se;         /* out */
    int64_t n_rows;            /* out: N                                                                 */
    int32_t k_done;            /* out: K on success                                                      */
    double time_ms;            /* out                                                                    */
} bl_cv_result;

bl_status bl_cv_fit(bl_ctx ctx, const bl_matrix* X, const bl_cv* cv, const bl_path_opts* opts, bl_cv_result* res);

/*
 * Screening network of the learned form (the paper has none; it stands beside the strong rule,
 * which stays the fallback, and the exact check, which keeps the last word).
 *   input f (4 floats, as recorded above) -> h1 = relu(W1 f + b1) (64) -> h2 = relu(W2 h1 + b2) (64)
 *   -> logit o = w3 . h2 + b3 -> score sigmoid(o).
 * Parameters: FP32 vector of BL_MLP_NPARAMS = 4545 in the order W1[64][4], b1[64], W2[64][64], b2[64],
 * w3[64], b3 (row-major).  All arrays DEVICE, caller-owned; m < 2^31.
 */
#define BL_MLP_HIDDEN 64
#define BL_MLP_NPARAMS (BL_MLP_HIDDEN * BL_MLP_HIDDEN + 7 * BL_MLP_HIDDEN + 1)

/* prob[i] = score of feat[4i .. 4i+3]. */
bl_status bl_mlp_forward(bl_ctx ctx, const float* feat, int64_t m, const float* params, float* prob);

/* Mean binary cross-entropy L = (1/m) sum_i [log(1 + e^{o_i}) - y_i o_i] over all m samples and its
 * gradient (grad [BL_MLP_NPARAMS] device, same layout as params); *loss (host) may be NULL.
 * label[i] in {0, 1}. */
bl_status bl_mlp_loss_grad(bl_ctx ctx, const float* feat, const float* label, int64_t m, const float* params,
                           float* grad, double* loss);

typedef struct {
    int32_t epochs;            /* passes over the records                                         */
    int32_t batch;             /* records per Adam step, multiple of 128                          */
    double lr, beta1, beta2, eps;  /* Adam (Kingma and Ba): step lr m^/(sqrt(v^) + eps)           */
    uint64_t seed;             /* order of the records within each epoch                          */
    double target_recall;      /* tau: the largest 1/4096-grid score such that at least this
                                  fraction of the positive records scores at or above it        */
} bl_mlp_train_opts;

typedef struct {
    double loss_first;         /* mean loss over the first epoch's steps                          */
    double loss_last;          /* mean loss over the last epoch's steps                           */
    double tau;                /* threshold for opts->mlp_tau                                     */
    double recall;             /* fraction of positive records scored >= tau                      */
    double neg_pass;           /* fraction of negative records scored >= tau                      */
    int64_t steps;
    double time_ms;
} bl_mlp_train_result;

/* Adam on the mean cross-entropy, params (device) trained in place from their initial values.
 * The steps of an epoch replay a captured HIP graph. */
bl_status bl_mlp_train(bl_ctx ctx, const float* feat, const float* label, int64_t m, float* params,
                       const bl_mlp_train_opts* opts, bl_mlp_train_result* res);

/*
 * Kernel timing (diagnostics for measurement).  When enabled, bl_fit_path records HIP
 * events on the context stream around each launch of the scan, the CD solve and the
 * column statistics, and accumulates per kernel: launches, summed duration and the
 * algorithmic bytes those launches had to read:
 *   scan      columns scanned x n_total x sizeof(element)   (+ the residual once per launch);
 *             in the precision form this is the BF16 matrix-core scan
 *   CD        covariance solve: sweeps x m^2 x 8 (the Gram of the working set, m features, per sweep);
 *             residual solve (working sets above the covariance limit): sweeps x m x n_total x sizeof(element)
 *   colstats  p x n_total x sizeof(element)
 *   gram      Gram entries of new pool members and the gather of the working set's Gram
 *   rupdate   residual update after a solve: m x n_total x sizeof(element)
 *   recheck   precision form: residual pieces, error band and FP64 re-scans of flagged and set columns;
 *             batched form: the FP64 scan of the working sets' union before each solve and (BF16 scans)
 *             the band and its FP64 re-scan after it, units = columns re-scanned
 *   setup     precision and batched forms: the two FP64 set-up scans (lambda_max and BEDPP products); the
 *             plain path counts them under scan (same kernel)
 *   bscan     batched form: the check scans X_cols'R, columns x n_total x sizeof(element) + the right-hand
 *             sides once (n_total x nprob x 8 bytes; BF16 forms: their 2 or 3 BF16 pieces) bytes and
 *             2 x columns x n_total x nprob flops (the FP64 contraction's) per launch
 * bl_profile(ctx, 1) enables and resets the counters, bl_profile(ctx, 0) disables.
 */
typedef struct {
    int64_t launches;
    double total_ms;
    double bytes;
    double flops;              /* algorithmic floating-point operations (matrix-core scans), else 0 */
    double units;              /* CD: coordinate updates (sweeps x working-set size, summed over solves and
                                  problems); scans: columns scanned; else 0                            */
} bl_kernel_profile;

enum { BL_PROF_SCAN = 0, BL_PROF_CD = 1, BL_PROF_COLSTATS = 2, BL_PROF_GRAM = 3, BL_PROF_RUPDATE = 4,
       BL_PROF_RECHECK = 5, BL_PROF_BSCAN = 6, BL_PROF_SETUP = 7, BL_PROF_COUNT = 8 };

bl_status bl_profile(bl_ctx ctx, int enable);
bl_status bl_profile_get(bl_ctx ctx, int kernel, bl_kernel_profile* out);

#ifdef __cplusplus
}
#endif
#endif /* BL_H */
