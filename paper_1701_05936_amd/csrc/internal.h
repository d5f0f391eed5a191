// Internal interface between the path driver (api.cpp) and the HIP kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace blk {

// Per-lambda statistics reduced on the device (one record per lambda).
struct LamStats {
    double rss;        // ||r||^2
    double obj;        // Q(beta; lambda)
    double intercept;  // y_mean - sum_j c_j beta_j / s_j
    double l1;         // ||beta||_1
    int64_t n_active;  // nonzero coefficients
    int64_t n_strong;  // working-set size after the last round
    int64_t n_safe;    // BEDPP survivors at this lambda
    int64_t n_scan;    // columns in one check scan
};

// Outcome of one CD solve plus the following check, read back by the host in one copy.
struct RoundInfo {
    uint32_t n_viol;   // violators found by the check
    int32_t sweeps;    // CD sweeps of the solve
    int32_t status;    // 0 converged, 1 max_sweeps reached
    int32_t cd_len;    // size of the set the solve cycled over
    int64_t scan_len;  // columns the check scanned
};

// Scalars the kernels share through device memory.
struct DevScalars {
    double sum_r;      // sum of the residual over the rows (for the simplified scan)
    double rss;        // ||r||^2 after the last CD solve
    double y_mean;
    double yy;         // ||y~||^2
    double lmax;       // lambda_max
    int64_t jstar;
    int64_t n_rows;
    int64_t n_new;     // features the last pool update added
    int64_t stage;     // host staging slot for small device-to-host and host-to-device copies
    RoundInfo round;
    double i8_scale[4];   // power-of-two scales of the int8 residual pieces (int8 matrix-core form)
    double i8_a;          // that form's bound numerator: (||remainder||_2 + gamma_3 ||sum_k s_k |q_k| ||_2)(1 + 2^-20)
    // logistic regression
    double lg_b0;         // intercept (standardized scale)
    double lg_db0;        // the last majorization step's intercept change
    double lg_n1;         // fitted rows with y = 1
    double lg_bad;        // fitted rows with y outside {0, 1}
};

struct Mat {
    const void* X;
    int xtype;         // bl_xtype
    int64_t n_total, p, ldx;
    const uint8_t* mask;
};

int device_cu_count();
int64_t device_lds_per_block();   // dynamic LDS bytes one workgroup may take

// column statistics: center, scale, keep; n_rows written to *n_rows_dev (device) when not null
hipError_t launch_colstats(const Mat& m, double* c, double* s, uint8_t* keep, int64_t n_rows, hipStream_t st);
// rows in the fit
hipError_t launch_count_rows(const Mat& m, int64_t* out_dev, hipStream_t st);
// y_mean, y~ (0 outside the fit), ||y~||^2 -> sc->y_mean, sc->yy; also r = y~ when r != nullptr
hipError_t launch_center_y(const Mat& m, const double* y, double* ytilde, double* r, DevScalars* sc, hipStream_t st);
// sc->sum_r (and sc->rss when want_rss) of a row vector
hipError_t launch_sum_r(const Mat& m, const double* r, DevScalars* sc, bool want_rss, hipStream_t st);
// v_i = (x_{i,j} - c_j)/s_j on fitted rows, 0 elsewhere
hipError_t launch_std_column(const Mat& m, int64_t j, const double* c, const double* s, double* v, hipStream_t st);

// z_j = (x_j'r - c_j sum_r)/(n s_j) for j = cols[t], t < len (cols == nullptr: j = t).
// len is read from len_dev when not null (device-side length), else len_host.
// Epilogue when check is true: j is a violator if (in_s == null || in_s[j]) && excl[j] == 0 && |z_j| > lam;
// violators get mark[j] = 1 and bump *nviol.  keep[j] == 0 gives z_j = 0 and is never a violator.
struct ScanArgs {
    const int32_t* cols;
    const int64_t* len_dev;
    int64_t len_host;
    const double* r;
    const DevScalars* sc;     // sum_r, n_rows
    const double* c;
    const double* s;
    const uint8_t* keep;
    double* z;
    bool check;
    double lam;
    const uint8_t* in_s;
    const uint8_t* excl;
    uint8_t* mark;
    uint32_t* nviol;
    int64_t* len_out;   // when not null, block 0 stores the scanned length here
    const double* w;    // check threshold lam * w[j] (elastic-net penalty weights) when not null
};
hipError_t launch_scan(const Mat& m, const ScanArgs& a, hipStream_t st);

// argmax_j |a_j| over kept columns (ties -> smallest j) -> sc->lmax, sc->jstar
hipError_t launch_argmax_abs(const double* a, const uint8_t* keep, int64_t p, double* part_v, int64_t* part_i,
                             DevScalars* sc, hipStream_t st);

// safe[j] = keep[j] && !BEDPP-discard(j)  (bedpp false: safe = keep); counts into *cnt (device, += )
hipError_t launch_bedpp(int64_t p, const double* a, const double* b, const uint8_t* keep, bool bedpp, double lmax,
                        double sgn, double lam, double rhs, uint8_t* safe, hipStream_t st);
// strong[j] = safe[j] && (act(j) || (ssr && |zprev_j| >= thr w_j)); act(j) = active ? active[j] : beta[j] != 0;
// w null: w_j = 1
hipError_t launch_ssr(int64_t p, const uint8_t* safe, const uint8_t* active, const double* beta, const double* zprev,
                      bool ssr, double thr, uint8_t* strong, hipStream_t st, const double* w = nullptr);
// out[j] = |a_j| / (alpha w_j) (the elastic net's lambda_max is its largest kept value)
hipError_t launch_enet_lmax_terms(const double* a, const double* w, double alpha, int64_t p, double* out,
                                  hipStream_t st);

// ordered compaction of a uint8 mask: out[0..len) = ascending j with mask[j] != 0; *len_dev = len
size_t compact_scratch_bytes(int64_t p);
// flag[set[e]] = 1 where beta[set[e]] != 0, e < *len_dev <= m_max (flag cleared by the caller)
hipError_t launch_mark_nonzero(const int32_t* set, const int64_t* len_dev, int64_t m_max, const double* beta,
                               uint8_t* flag, hipStream_t st);
// sc->round.{sweeps, status, cd_len} = the given totals
hipError_t launch_set_round(DevScalars* sc, int32_t sweeps, int32_t status, int32_t cd_len, hipStream_t st);
hipError_t launch_compact(const uint8_t* mask, int64_t p, int32_t* out, int64_t* len_dev, void* scratch,
                          hipStream_t st);

// cyclic CD over set[0..len) (len from len_dev if not null); writes sc->round.{sweeps,status}, sc->sum_r, sc->rss
struct CdArgs {
    const int32_t* set;
    const int64_t* len_dev;
    int64_t len_host;
    const double* c;
    const double* s;
    double lam;
    double* beta;
    double* r;
    double tol;
    int max_sweeps;
    DevScalars* sc;
    double alpha;         // elastic-net mixing (1: lasso)
    const double* w;      // penalty weights or null (all 1)
};
bool cd_supported(int64_t n_total);
hipError_t launch_cd(const Mat& m, const CdArgs& a, hipStream_t st);

// per-lambda record: stats over the set (beta nonzero only there) into *out
// obj = rss / (2n) + lam sum_j w_j (alpha |beta_j| + (1 - alpha) beta_j^2 / 2) (lasso: alpha 1, w null)
hipError_t launch_record(const int32_t* set, const int64_t* len_dev, const int64_t* len_safe, const int64_t* len_scan,
                         const double* beta, const double* c, const double* s, const DevScalars* sc, double lam,
                         LamStats* out, hipStream_t st, double alpha = 1.0, const double* w = nullptr);

// ---- coordinate descent with covariance updates (gram_cd.hip) ----
constexpr int GCD_B = 64;       // coordinates per sequential block
constexpr int GCD_MAX = 7168;   // largest working set the covariance solve holds in LDS

struct GcdArgs {
    const double* G;      // m x m Gram of the set (column-major, ld m)
    int64_t m;
    const double* g0;     // gradient at the start
    const double* b0;     // coefficients at the start
    double* b1;           // coefficients at the end (per set position)
    const int32_t* set;
    double* beta;         // [p], updated at set positions
    double lam, tol;
    int max_sweeps;
    DevScalars* sc;
    const double* lamv;   // per set position threshold (weighted penalties) or null (lam for all)
};
hipError_t launch_pool_add(const int32_t* set, const int64_t* len_dev, int64_t len_host, int32_t* pool_pos,
                           int32_t* pool_list, int64_t pool_size, int64_t* n_new_out, hipStream_t st);
hipError_t launch_gram_update(const Mat& m, const int32_t* pool_list, int64_t P, int64_t P0, int64_t N,
                              const double* c, const double* s, double n_rows, double* G, int64_t ldg,
                              hipStream_t st);
hipError_t launch_gather_gram(const int32_t* set, int64_t m, const int32_t* pool_pos, const double* Gp, int64_t ldg,
                              double* GE, hipStream_t st);
hipError_t launch_gather_start(const int32_t* set, int64_t m, const double* z, const double* beta, double* g0,
                               double* b0, hipStream_t st);
hipError_t launch_gcd(const GcdArgs& a, hipStream_t st);

// multi-workgroup covariance solve (leader + helpers); g, b are device arrays of m entries holding the
// start values (g0, b0) on entry and the final values on exit; sync must be zeroed before the launch.
struct GcdMultiArgs {
    const double* G;
    int64_t m;
    double* g;
    double* b;
    double* delta;        // m entries (block changes)
    uint32_t* sync;       // gcd_multi_sync_words(H) words, zeroed
    int H;                // helper workgroups
    uint32_t spin_limit;  // bound of every wait (sleep iterations)
    double lam, tol;
    int max_sweeps;
    DevScalars* sc;
};
// helper workgroups of the multi-workgroup solve of m features: one per block of 32 when at most cap, else one
// per two blocks; 0: use the single-workgroup solve
int gcd_multi_helpers(int64_t m, int cap);
int gcd_multi_resident();          // workgroups of the multi-workgroup solve resident on the device at once
// Elastic net in the covariance solve: with q_e = sqrt(1 + lam (1 - alpha) w_e) the working set's problem in
// gamma_e = q_e beta_e is a lasso with unit-diagonal Gram G~ = Q^-1 (G + lam (1 - alpha) W) Q^-1, gradient
// g~_e = (z_e - lam (1 - alpha) w_e beta_e) / q_e and thresholds lam alpha w_e / q_e (lamv, when w is not null).
hipError_t launch_enet_scale(const int32_t* set, int64_t m, const double* w, double lam, double alpha, double* GE,
                             double* g0, double* b0, double* lamv, hipStream_t st);
// out[e] = pool_pos[set[e]]
hipError_t launch_map_pos(const int32_t* set, int64_t m, const int32_t* pool_pos, int32_t* out, hipStream_t st);
// back to beta: b0 /= q, b1 /= q, beta[set[e]] = b1[e]
hipError_t launch_enet_unscale(const int32_t* set, int64_t m, const double* w, double lam, double alpha, double* b0,
                               double* b1, double* beta, hipStream_t st);
int64_t gram_cd_max();              // largest working set of the covariance solve
size_t gcd_multi_sync_words(int H);
hipError_t launch_gcd_multi(const GcdMultiArgs& a, hipStream_t st);
hipError_t launch_copy_f64(const double* src, double* dst, int64_t n, hipStream_t st);
hipError_t launch_scatter_beta(const int32_t* set, int64_t m, const double* b1, double* beta, hipStream_t st);
size_t r_update_scratch_bytes(int64_t n_total, int64_t m);
hipError_t launch_r_update(const Mat& mt, const int32_t* set, int64_t m, const double* b0, const double* b1,
                           const double* c, const double* s, double* part, double* r, hipStream_t st);

// ---- precision forms: int8 codes on BF16 or int8 matrix cores (lowp.hip) ----
constexpr int LOWP_PIECES = 3;  // BF16 pieces of the residual
int64_t lowp_pad(int64_t n_total);          // rows of each BF16 residual piece (multiple of 128)
int64_t lowp_pad_i8(int64_t n_total);       // rows of each int8 residual piece (multiple of 512)
size_t lowp_piece_bytes(int64_t n_total);  // piece buffer of either form
double lowp_coef();                         // error coefficient of the scan bound
bool lowp_supported(const Mat& m);          // int8 X, 16-byte aligned columns
hipError_t launch_r_pieces(const double* r, int64_t n_total, __bf16* pieces, hipStream_t st);
hipError_t launch_scan_bf16(const Mat& m, const __bf16* pieces, const int32_t* cols, const int64_t* len_dev,
                            int64_t len_host, const DevScalars* sc, const double* c, const double* s,
                            const uint8_t* keep, double* z, hipStream_t st);
// int8 codes on int8 matrix cores against LOWP_I8_PIECES int8 pieces of the residual
constexpr int LOWP_I8_PIECES = 4;
// pieces [LOWP_I8_PIECES][lowp_pad_i8(n_total)] int8 plus sc->i8_scale and sc->i8_a (one workgroup)
hipError_t launch_r_pieces_i8(const double* r, int64_t n_total, int8_t* pieces, DevScalars* sc, hipStream_t st);
// cols must be non-null
hipError_t launch_scan_i8(const Mat& m, const int8_t* pieces, const int32_t* cols, const int64_t* len_dev,
                          int64_t len_host, const DevScalars* sc, const double* c, const double* s,
                          const uint8_t* keep, double* z, hipStream_t st);
// flag[j] = 1 (flag pre-zeroed) when |z_j| is within its bound of lam (j in in_s, not in excl) or of thr2 (>= 0);
// err_out[j] = the bound (either pointer may be null); i8 selects the int8 form's bound
hipError_t launch_band(const int32_t* cols, const int64_t* len_dev, const double* z, const double* c, const double* s,
                       const DevScalars* sc, double lam, const uint8_t* in_s, const uint8_t* excl, double thr2,
                       uint8_t* flag, double* err_out, int64_t p, bool i8, hipStream_t st);
hipError_t launch_viol(const int32_t* cols, const int64_t* len_dev, const double* z, const uint8_t* in_s, uint8_t* inE,
                       double lam, uint32_t* nviol, int64_t p, hipStream_t st);

// ---- batched form (batch.hip) ----
constexpr int BNP = 64;          // problems per batch (right-hand-side columns of the shared contraction)
constexpr int BCD_MAX = 7168;    // largest working set of a problem in the batched solve

struct BatchScalars {
    double sum_r, rss, y_mean, yy, lmax, sign_star;
    int64_t jstar, n_rows, n_new, pool_size;
    uint32_t n_viol;
    int32_t sweeps, status, pad;
};
int64_t batch_pad(int64_t n_total);  // rows of the row-major right-hand sides (multiple of 64)
// out[b*p + j] for j = cols[t]: mode 0 raw x_j' B[:, b]; mode 1 (x_j o x_j)' B[:, b];
// mode 2 (x_j' B[:, b] - c_bj sum_r(b)) / (n_b s_bj)
// variant 0..5: workgroups of 2, 4, 8 waves (64, 128, 256 columns), without (0-2) or with (3-5) register
// prefetch of the next row batch
constexpr int BSCAN_VARIANTS = 6;
int bscan_variant_cols(int variant);
// the standardized correlations of a short column list (len from the host) split over row ranges: more
// workgroups than the one-pass scan, the ranges added in order by a second kernel (part: scratch)
size_t bscan_split_part_bytes(int64_t n_total, int64_t len);
hipError_t launch_bscan_split(const Mat& mt, const int32_t* cols, int64_t len, const double* B, int nprob,
                              const BatchScalars* bs, const double* c, const double* s, const uint8_t* keep,
                              double* part, double* out, hipStream_t st);
// BF16 form of the batched check scan (f32 X, pc = 2 or 3 pieces of x and r): residual pieces, the scan, its
// bound and the band flags
double bscan_bf16_rel(int64_t n_total, int pc);
int64_t bscan_bf16_pieces_bytes(int64_t n_total, int pc);
hipError_t launch_b_r_pieces(const double* R, int64_t n_total, int nprob, int pc, __bf16* Rp, hipStream_t st);
// the scan takes as many workgroups as the device holds at once and splits the column list between them
// evenly, cutting tiles by rows where needed (part: scratch of bscan_bf16_part_bytes(pc) bytes for the rows of
// the cut tiles)
int bscan_bf16_slots(int pc);
size_t bscan_bf16_part_bytes(int pc);
hipError_t launch_bscan_bf16(const Mat& mt, const int32_t* cols, const int64_t* len_dev, int64_t len_host, int pc,
                             const __bf16* Rp, int nprob, const BatchScalars* bs, const double* c, const double* s,
                             const uint8_t* keep, double* part, double* out, hipStream_t st);
hipError_t launch_b_band(const int32_t* cols, const int64_t* len_dev, int64_t p, int nprob, const double* z,
                         const double* c, const double* s, const uint8_t* keep, const BatchScalars* bs,
                         const double* lam, const double* thr, double rel, uint8_t* flag, hipStream_t st);
// modes 0-2 take as many workgroups as the device holds at once and split the column list evenly between
// them, cutting tiles by rows where needed (part: scratch of bscan_part_bytes() bytes for the rows of the cut
// tiles)
size_t bscan_part_bytes();
hipError_t launch_bscan(const Mat& mt, int mode, const int32_t* cols, const int64_t* len_dev, int64_t len_host,
                        const double* B, int nprob, BatchScalars* bs, const double* c, const double* s,
                        const uint8_t* keep, double* part, double* out, hipStream_t st, int variant = 1);
hipError_t launch_b_masks(const uint8_t* masks, int64_t n_total, int nprob, double* Mb, hipStream_t st);
hipError_t launch_b_center_y(const uint8_t* masks, const double* Y, int64_t n_total, int nprob, double* Yt, double* R,
                             BatchScalars* bs, hipStream_t st);
hipError_t launch_b_sum_r(const double* R, int64_t n_total, int nprob, BatchScalars* bs, hipStream_t st);
hipError_t launch_b_stats(const double* S1, const double* S2, int64_t p, int nprob, const BatchScalars* bs, double* c,
                          double* s, uint8_t* keep, hipStream_t st);
hipError_t launch_b_argmax(const double* a, const uint8_t* keep, int64_t p, int nprob, BatchScalars* bs,
                           hipStream_t st);
hipError_t launch_b_std_column(const Mat& mt, const uint8_t* masks, int nprob, const BatchScalars* bs, const double* c,
                               const double* s, double* Bm, hipStream_t st);
// lambda (threshold) of problem b at step k = koff (+ *kdev if kdev): lamg[k * BNP + b]
hipError_t launch_b_bedpp(int64_t p, int nprob, const double* a, const double* bb, const uint8_t* keep, bool bedpp,
                          const BatchScalars* bs, const double* lamg, int koff, const int64_t* kdev, uint8_t* safe,
                          hipStream_t st);
hipError_t launch_b_ssr(int64_t p, int nprob, const uint8_t* safe, const double* beta, const double* zprev, bool ssr,
                        const double* thrg, int koff, const int64_t* kdev, const uint8_t* want, uint8_t* strong,
                        hipStream_t st);
hipError_t launch_b_kinc(int64_t* kdev, hipStream_t st);
hipError_t launch_b_union(int64_t p, int nprob, const uint8_t* mask, uint8_t* out, hipStream_t st);
hipError_t launch_b_viol(const int32_t* cols, const int64_t* len_dev, int64_t p, int nprob, const double* z,
                         const uint8_t* in_s, uint8_t* inE, const double* lam, const uint8_t* want, BatchScalars* bs,
                         hipStream_t st);
size_t b_compact_scratch_bytes(int64_t p);
hipError_t launch_b_compact(const uint8_t* mask, int64_t p, int nprob, const uint8_t* want, int32_t* out,
                            int64_t* lens, void* scratch, hipStream_t st);
hipError_t launch_b_pool_add(const int32_t* sets, const int64_t* lens, int64_t p, int nprob, const uint8_t* want,
                             int32_t* pool_pos, int32_t* pool_list, BatchScalars* bs, hipStream_t st);
hipError_t launch_b_commit(int nprob, const uint8_t* want, BatchScalars* bs, hipStream_t st);
hipError_t launch_b_gram_update(const Mat& mt, const uint8_t* masks, int nprob, const int32_t* pool_list,
                                const BatchScalars* bs, const double* c, const double* s, double* Gp, int64_t cap,
                                int64_t max_P, int64_t max_N, const uint8_t* want, hipStream_t st);
hipError_t launch_b_gather(const int32_t* sets, const int64_t* lens, int64_t p, int nprob, const uint8_t* want,
                           const int32_t* pool_pos, const double* Gp, int64_t cap, const double* z, const double* beta,
                           double* GE, int64_t ge_stride, double* g0, double* b0, int64_t max_m, hipStream_t st);
hipError_t launch_b_gcd(const int32_t* sets, const int64_t* lens, int64_t p, int nprob, const uint8_t* want,
                        const double* GE, int64_t ge_stride, const double* g0, const double* b0, double* b1,
                        double* beta, const double* lam, double tol, int max_sweeps, BatchScalars* bs,
                        hipStream_t st);
hipError_t launch_b_r_update(const Mat& mt, const uint8_t* masks, const int32_t* sets, const int64_t* lens, int nprob,
                             const uint8_t* want, const double* b0, const double* b1, const double* c,
                             const double* s, double* R, hipStream_t st);
hipError_t launch_b_record(const int32_t* sets, const int64_t* lens, int64_t p, int nprob, const double* beta,
                           const double* c, const double* s, const BatchScalars* bs, const double* lam,
                           LamStats* out, int k, int K, const int64_t* n_safe, hipStream_t st);

// ---- screening network of the learned form (mlp.hip) ----
constexpr int MLP_HIDDEN = 64;
constexpr int MLP_NPARAMS = MLP_HIDDEN * MLP_HIDDEN + 7 * MLP_HIDDEN + 1;
hipError_t launch_mlp_fwd(const float* feat, int64_t m, const float* P, float* prob, hipStream_t st);
int mlp_grad_blocks(int64_t batch);
// step: device counter (the minibatch is step mod nb of epoch step / nb, order given by perm[2e], perm[2e+1]:
// sample (a (base + t) + c) mod m); step == nullptr: the single batch of all m samples in order
hipError_t launch_mlp_grad(const float* feat, const float* label, int64_t m, int64_t batch, int64_t nb,
                           const int64_t* perm, const int64_t* step, const float* P, float* partial,
                           double* loss_part, hipStream_t st);
hipError_t launch_mlp_adam(const float* partial, int nblk, const double* loss_part, float* P, float* mom, float* vel,
                           const int64_t* step, int64_t m, int64_t batch, int64_t nb, double lr, double b1,
                           double b2, double eps, int apply, float* grad_out, double* loss_out, hipStream_t st);
hipError_t launch_step_inc(int64_t* step, hipStream_t st);
hipError_t launch_mlp_hist(const float* prob, const float* label, int64_t m, int bins, uint32_t* hist,
                           hipStream_t st);
hipError_t launch_learned(uint8_t* strong, const double* beta, const float* zh, int64_t p, int s1, int s2, int s3,
                          float ratio, const float* P, float tau_logit, int apply, uint8_t* cand, hipStream_t st);
hipError_t launch_zhist(const int32_t* cols, const int64_t* len_dev, int64_t len_host, const double* z, double lam,
                        float* slot, int64_t p, hipStream_t st);
hipError_t launch_zhist_keep(const uint8_t* keep, int64_t p, const double* z, double lam, float* slot,
                             hipStream_t st);
hipError_t launch_rec_feat(const int32_t* list, const int64_t* len_dev, const float* zh, int64_t p, int s1, int s2,
                           int s3, float ratio, const double* beta, int64_t cap, int64_t* count, float* feat,
                           float* label, hipStream_t st);

hipError_t launch_fill_u8(uint8_t* p, uint8_t v, int64_t n, hipStream_t st);
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t st);
hipError_t launch_or_u8(uint8_t* dst, const uint8_t* src, int64_t n, hipStream_t st);


// ---- cross-validation (cv.hip) ----
hipError_t launch_cv_setup(const int32_t* fold, const double* y, int64_t n_total, int nfolds, uint8_t* masks,
                           uint8_t* test, double* Y, uint8_t* all_rows, hipStream_t st);
hipError_t launch_cv_union(const double* beta, int64_t p, int K, int nfolds, uint8_t* mark, hipStream_t st);
hipError_t launch_cv_predict(const Mat& m, int nfolds, int K, int64_t max_rows, const double* beta, const double* s,
                             const int32_t* ulist, const int64_t* ulens, const int32_t* rows, const int64_t* rlens,
                             const double* icpt, const double* y, double* pred, double* loss, hipStream_t st);
hipError_t launch_cv_reduce(const double* loss, const uint8_t* all_rows, const int32_t* rows, const int64_t* rlens,
                            int64_t n_total, int K, int nfolds, double* cve, double* cvse, double* ferr,
                            hipStream_t st);


// ---- lasso-penalized logistic regression (logit.hip) ----
// sc->lg_n1 = fitted rows with y = 1, sc->lg_bad = fitted rows with y outside {0, 1}
hipError_t launch_logit_check_y(const Mat& m, const double* y, DevScalars* sc, hipStream_t st);
// eta = b0 (fitted rows, 0 elsewhere), sc->lg_b0 = b0
hipError_t launch_logit_init(const Mat& m, double b0, double* eta, DevScalars* sc, hipStream_t st);
// g = y - sigmoid(eta) on fitted rows (0 elsewhere); r0 = 4 g when r0 is not null
hipError_t launch_logit_resid(const Mat& m, const double* y, const double* eta, double* g, double* r0, hipStream_t st);
// majorization step of the intercept: db0 = sum(r0) / n (sc->sum_r, sc->n_rows), r0 -= db0 on fitted rows,
// sc->lg_db0 = db0, sc->lg_b0 += db0; keeps a copy of r0 in r0c
hipError_t launch_logit_center(const Mat& m, double* r0, double* r0c, DevScalars* sc, hipStream_t st);
// eta += db0 + (r0c - r) on fitted rows (the change of the linear predictor over the solve)
hipError_t launch_logit_eta(const Mat& m, const double* r0c, const double* r, double* eta, const DevScalars* sc,
                            hipStream_t st);
// sc->rss = 2 sum_i [log(1 + e^eta_i) - y_i eta_i] (the deviance) and sc->y_mean = sc->lg_b0, for launch_record
hipError_t launch_logit_loss(const Mat& m, const double* y, const double* eta, DevScalars* sc, hipStream_t st);

}  // namespace blk
