/*
 * Plain FP64 CPU oracle for the pathwise lasso (Zeng & Breheny, "The biglasso
 * Package").  TEST INFRASTRUCTURE ONLY: it exists so the GPU library can be
 * checked against an obviously correct implementation.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark may load it; the
 * GPU library never calls it and shares no code with it.
 *
 * Conventions shared by every function:
 *   X        column-major n_total x p, leading dimension ldx >= n_total
 *   mask     row subset: uint8[n_total], 1 = row is in the fit; NULL = all rows
 *   n        number of rows in the fit
 *   vectors over rows (y~, r) have length n_total and are zero outside the fit
 *   x~_ij    = (x_ij - c_j) / s_j, the standardized column (never stored)
 *   Q(b; l)  = ||y~ - X~ b||^2 / (2n) + l * ||b||_1   (standardized scale)
 */
#ifndef BL_ORACLE_H
#define BL_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

int or_num_threads(void);
void or_set_threads(int t);
int64_t or_standardize(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                       double* c, double* s, uint8_t* keep);
void or_zscan(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
              const double* c, const double* s, const uint8_t* keep, const double* r, double* z);
int or_lambda_max(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                  const double* c, const double* s, const uint8_t* keep, const double* y,
                  double* ybar, double* ytilde, double* a, double* lambda_max, int64_t* jstar);
void or_bedpp_b(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                const double* c, const double* s, const uint8_t* keep, int64_t jstar, double* b);
int64_t or_bedpp_discard(int64_t p, const double* a, const double* b, const uint8_t* keep,
                         double lambda_max, double sign_star, double v, double lambda, uint8_t* discard);
void or_lambda_grid(double lambda_max, double ratio, int64_t K, double* lam);
int or_cd(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
          const double* c, const double* s, double lambda, const int64_t* set, int64_t set_len,
          double* beta, double* r, double tol, int64_t max_sweeps, int64_t* sweeps);
void or_residual(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                 const double* c, const double* s, const double* ytilde, const double* beta, double* r);
double or_objective(int64_t n_total, const uint8_t* mask, const double* r, int64_t p, const double* beta,
                    double lambda);
double or_duality_gap(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                      const double* c, const double* s, const uint8_t* keep, const double* ytilde,
                      const double* r, const double* beta, double lambda);

/* per-lambda statistics written by or_fit_path (each array has K entries) */
typedef struct {
    int64_t* sweeps;     /* CD sweeps summed over KKT rounds                      */
    int64_t* n_strong;   /* |E_k| after the last round                           */
    int64_t* n_viol;     /* features added back by the post-convergence check     */
    int64_t* n_rounds;   /* CD solves at this lambda                              */
    int64_t* n_safe;     /* BEDPP survivors (predicate only, not used in solving) */
    int64_t* n_active;   /* nonzero coefficients                                 */
    double* rss;         /* ||r||^2                                              */
    double* obj;         /* Q(beta; lambda_k)                                     */
    double* gap;         /* relative duality gap (P - D) / P                      */
} or_path_stats;

/* OR_SCREEN_ACTIVE: working set = previous active set only, so every feature entering the path is
 * found by the post-convergence check (exercises the repair branch) */
enum { OR_SCREEN_NONE = 0, OR_SCREEN_SSR = 1, OR_SCREEN_ACTIVE = 2 };

int or_fit_path(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                const double* y, int64_t K, double ratio, const double* lam_in, int screen, double tol,
                int64_t max_sweeps,
                double* c, double* s, uint8_t* keep, double* lambda, double* beta /* p x K */,
                double* ybar, or_path_stats* st, int64_t* k_done);

/* learned screening network: 4 -> H -> H -> 1, ReLU hidden layers, logistic output */
void or_mlp_forward(int64_t m, int64_t H, const double* feat /* m x 4 row-major */, const double* params,
                    double* prob);
double or_mlp_loss_grad(int64_t m, int64_t H, const double* feat, const double* label, const double* params,
                        double* grad);


/* lasso-penalized logistic regression (y in {0, 1}); b0 [K] intercepts on the standardized scale */
double or_logistic_objective(int64_t n_total, const uint8_t* mask, const double* y, const double* eta, int64_t p,
                             const double* beta, double lambda);
double or_logistic_gap(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                       const double* c, const double* s, const uint8_t* keep, const double* y, const double* eta,
                       const double* beta, double lambda);
double or_logistic_safe_threshold(int64_t n, int64_t n1, double lambda_max, double lambda);
int64_t or_logistic_discard(int64_t p, const double* a, const uint8_t* keep, double thr, uint8_t* discard);
int or_fit_path_logistic(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                         const double* y, int64_t K, double ratio, int screen, double tol, int64_t max_iter,
                         double* c, double* s, uint8_t* keep, double* lambda, double* beta, double* b0out,
                         or_path_stats* st, int64_t* k_done);

#ifdef __cplusplus
}
#endif

/* elastic net with feature weights (w may be NULL: all 1); alpha = 1, w = NULL is the lasso */
int or_cd_enet(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
               const double* c, const double* s, double lambda, double alpha, const double* w,
               const int64_t* set, int64_t set_len, double* beta, double* r, double tol, int64_t max_sweeps,
               int64_t* sweeps);
double or_objective_enet(int64_t n_total, const uint8_t* mask, const double* r, int64_t p, const double* beta,
                         double lambda, double alpha, const double* w);
double or_duality_gap_enet(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                           const double* c, const double* s, const uint8_t* keep, const double* ytilde,
                           const double* r, const double* beta, double lambda, double alpha, const double* w);
int or_fit_path_enet(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                     const double* y, int64_t K, double ratio, const double* lam_in, double alpha, const double* w,
                     int screen, double tol, int64_t max_sweeps, double* c, double* s, uint8_t* keep,
                     double* lambda, double* beta, double* ybar, or_path_stats* st, int64_t* k_done);

#endif
