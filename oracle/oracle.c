/*
 * Plain FP64 CPU oracle for the pathwise lasso of Zeng & Breheny, "The
 * biglasso Package" (arXiv:1701.05936).
 *
 * TEST INFRASTRUCTURE ONLY.  Loaded by the test suite, the smoke check and
 * the benchmark's CPU-baseline leg; never by the GPU library, with which it
 * shares no code.
 *
 * Every quantity is computed from its plain definition, in double precision,
 * one loop per formula, without blocking or fusion.  Column scans run their
 * columns in parallel with OpenMP (each column's sum is still a plain loop in
 * row order), as the paper parallelizes matrix-vector products (Section 3.2).
 *
 * Readings of the paper taken here (the paper leaves these open):
 *   - standard deviation uses divisor n, so (1/n) sum_i x~_ij^2 = 1
 *     (the paper's notation block in Section 2);
 *   - objective Q(b; l) = ||y~ - X~ b||^2 / (2n) + l ||b||_1, which makes
 *     l_max = max_j |x~_j' y~| / n;
 *   - lambda grid geometric from l_max down to ratio * l_max (Section 4 and the
 *     printed lambda values of the Section 5 example);
 *   - a column with s_j <= 1e-6 is constant and is left out (beta_j = 0);
 *   - the intercept is the mean of y over the fitted rows (y is centered);
 *   - CD stops when the largest |change| of a coefficient over one sweep of the
 *     set is below tol;
 *   - the strong rule keeps j when |z_j(prev)| >= 2 l_k - l_{k-1}; the
 *     post-convergence check flags j when |z_j| > l_k (strict).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* threads the column scans use (1 without OpenMP) */
int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* set the thread count of the column scans (no effect without OpenMP) */
void or_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

#define KEEP_MIN_SD 1e-6

static int64_t count_rows(int64_t n_total, const uint8_t* mask) {
    if (!mask) return n_total;
    int64_t n = 0;
    for (int64_t i = 0; i < n_total; ++i) n += mask[i] ? 1 : 0;
    return n;
}

static inline int in_fit(const uint8_t* mask, int64_t i) { return mask == NULL || mask[i] != 0; }

static double soft_threshold(double u, double l) {
    if (u > l) return u - l;
    if (u < -l) return u + l;
    return 0.0;
}

/*
 * Column centers c and scales s (Section 3.1: the package keeps only the
 * column means and standard deviations and standardizes cell by cell).
 * Two passes per column: mean, then mean squared deviation.
 */
int64_t or_standardize(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                       double* c, double* s, uint8_t* keep) {
    int64_t n = count_rows(n_total, mask);
    if (n <= 0) return 0;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < p; ++j) {
        const double* x = X + j * ldx;
        double sum = 0.0;
        for (int64_t i = 0; i < n_total; ++i)
            if (in_fit(mask, i)) sum += x[i];
        double mean = sum / (double)n;
        double ss = 0.0;
        for (int64_t i = 0; i < n_total; ++i)
            if (in_fit(mask, i)) ss += (x[i] - mean) * (x[i] - mean);
        double sd = sqrt(ss / (double)n);
        c[j] = mean;
        s[j] = sd;
        keep[j] = sd > KEEP_MIN_SD ? 1 : 0;
    }
    return n;
}

/*
 * z_j = (1/n) sum_{i in fit} x~_ij r_i  with x~_ij = (x_ij - c_j)/s_j, the
 * standardized correlation of Section 3.1.1 (type (3) divided by n), written
 * with the explicit standardized cell rather than the simplified form.
 * z_j = 0 for columns left out.
 */
void or_zscan(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
              const double* c, const double* s, const uint8_t* keep, const double* r, double* z) {
    int64_t n = count_rows(n_total, mask);
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < p; ++j) {
        if (!keep[j]) {
            z[j] = 0.0;
            continue;
        }
        const double* x = X + j * ldx;
        double acc = 0.0;
        for (int64_t i = 0; i < n_total; ++i)
            if (in_fit(mask, i)) acc += ((x[i] - c[j]) / s[j]) * r[i];
        z[j] = acc / (double)n;
    }
}

/*
 * y-bar, centered y~, the initial correlations a_j = z_j(y~) (Section 3.1.1,
 * type (2)), lambda_max = max_j |a_j| and the smallest index attaining it.
 * At any lambda >= lambda_max the zero vector satisfies the optimality
 * conditions, so the path starts at beta = 0.
 */
int or_lambda_max(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                  const double* c, const double* s, const uint8_t* keep, const double* y,
                  double* ybar, double* ytilde, double* a, double* lambda_max, int64_t* jstar) {
    int64_t n = count_rows(n_total, mask);
    if (n <= 0) return 1;
    double sum = 0.0;
    for (int64_t i = 0; i < n_total; ++i)
        if (in_fit(mask, i)) sum += y[i];
    double mean = sum / (double)n;
    for (int64_t i = 0; i < n_total; ++i) ytilde[i] = in_fit(mask, i) ? y[i] - mean : 0.0;
    or_zscan(n_total, p, X, ldx, mask, c, s, keep, ytilde, a);
    double best = -1.0;
    int64_t arg = -1;
    for (int64_t j = 0; j < p; ++j) {
        if (!keep[j]) continue;
        if (fabs(a[j]) > best) {
            best = fabs(a[j]);
            arg = j;
        }
    }
    *ybar = mean;
    *lambda_max = best < 0 ? 0.0 : best;
    *jstar = arg;
    return arg < 0 ? 1 : 0;
}

/* b_j = x~_j' x~_* / n, the correlation with the column attaining lambda_max (type (1) of Section 3.1.1) */
void or_bedpp_b(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                const double* c, const double* s, const uint8_t* keep, int64_t jstar, double* b) {
    int64_t n = count_rows(n_total, mask);
    const double* xs = X + jstar * ldx;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < p; ++j) {
        if (!keep[j]) {
            b[j] = 0.0;
            continue;
        }
        const double* x = X + j * ldx;
        double acc = 0.0;
        for (int64_t i = 0; i < n_total; ++i)
            if (in_fit(mask, i)) acc += ((x[i] - c[j]) / s[j]) * ((xs[i] - c[jstar]) / s[jstar]);
        b[j] = acc / (double)n;
    }
}

/*
 * Basic EDPP safe rule (Section 2.2): EDPP of Wang, Wonka & Ye (JMLR 2015)
 * with the reference point at lambda_max, where the dual solution is known
 * exactly (y~ / (n lambda_max)).  Rewritten for the scaling above
 * (their penalty n*lambda, ||x~_j||^2 = n), feature j is discarded at
 * lambda < lambda_max when
 *   | (lmax + l) a_j - (lmax - l) sgn(a_*) lmax b_j |
 *        < 2 l lmax - (lmax - l) sqrt(max(0, v - lmax^2)),   v = ||y~||^2 / n.
 * At l = lmax this is |a_j| < lmax.  Returns the number discarded.
 */
int64_t or_bedpp_discard(int64_t p, const double* a, const double* b, const uint8_t* keep,
                         double lambda_max, double sign_star, double v, double lambda, uint8_t* discard) {
    double lm = lambda_max, l = lambda;
    double slack = v - lm * lm;
    if (slack < 0.0) slack = 0.0;
    double rhs = 2.0 * l * lm - (lm - l) * sqrt(slack);
    int64_t cnt = 0;
    for (int64_t j = 0; j < p; ++j) {
        if (!keep[j]) {
            discard[j] = 1;
            ++cnt;
            continue;
        }
        double lhs = fabs((lm + l) * a[j] - (lm - l) * sign_star * lm * b[j]);
        discard[j] = lhs < rhs ? 1 : 0;
        cnt += discard[j];
    }
    return cnt;
}

/* lambda_k = lambda_max * ratio^(k/(K-1)), k = 0..K-1 (geometric grid, Section 4) */
void or_lambda_grid(double lambda_max, double ratio, int64_t K, double* lam) {
    if (K == 1) {
        lam[0] = lambda_max;
        return;
    }
    for (int64_t k = 0; k < K; ++k) lam[k] = lambda_max * pow(ratio, (double)k / (double)(K - 1));
}

/*
 * Cyclic coordinate descent at a fixed lambda over the features in `set`,
 * visited in the order given, warm-started from beta and its residual r
 * (the pathwise coordinate descent the package builds on, Section 1).
 * One coordinate step:
 *   g = (1/n) x~_j' r,  u = g + beta_j,  beta_j' = S(u, lambda),
 *   r <- r - (beta_j' - beta_j) x~_j
 * (the curvature (1/n) ||x~_j||^2 is 1).  Returns 0 when the largest |change|
 * over a sweep fell below tol, 1 when max_sweeps ran out.
 */
/* penalty weight of feature j (penalty.factor): w[j], or 1 without weights */
static double pw(const double* w, int64_t j) { return w ? w[j] : 1.0; }

int or_cd(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
          const double* c, const double* s, double lambda, const int64_t* set, int64_t set_len,
          double* beta, double* r, double tol, int64_t max_sweeps, int64_t* sweeps) {
    return or_cd_enet(n_total, p, X, ldx, mask, c, s, lambda, 1.0, NULL, set, set_len, beta, r, tol, max_sweeps,
                      sweeps);
}

/*
 * The same descent for the elastic-net penalty with feature weights (Section 1: the package fits
 * lasso and elastic-net penalties), lambda sum_j w_j (alpha |beta_j| + (1 - alpha) beta_j^2 / 2):
 * the coordinate minimizer is S(g + beta_j, lambda alpha w_j) / (1 + lambda (1 - alpha) w_j).
 * alpha = 1 and w = NULL is the lasso step above.
 */
int or_cd_enet(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
               const double* c, const double* s, double lambda, double alpha, const double* w,
               const int64_t* set, int64_t set_len, double* beta, double* r, double tol, int64_t max_sweeps,
               int64_t* sweeps) {
    (void)p;
    int64_t n = count_rows(n_total, mask);
    for (int64_t sweep = 1; sweep <= max_sweeps; ++sweep) {
        double max_change = 0.0;
        for (int64_t t = 0; t < set_len; ++t) {
            int64_t j = set[t];
            const double* x = X + j * ldx;
            double g = 0.0;
            for (int64_t i = 0; i < n_total; ++i)
                if (in_fit(mask, i)) g += ((x[i] - c[j]) / s[j]) * r[i];
            g /= (double)n;
            double bnew = soft_threshold(g + beta[j], lambda * alpha * pw(w, j)) /
                          (1.0 + lambda * (1.0 - alpha) * pw(w, j));
            double delta = bnew - beta[j];
            if (delta != 0.0) {
                for (int64_t i = 0; i < n_total; ++i)
                    if (in_fit(mask, i)) r[i] -= delta * ((x[i] - c[j]) / s[j]);
                beta[j] = bnew;
            }
            if (fabs(delta) > max_change) max_change = fabs(delta);
        }
        if (max_change < tol) {
            *sweeps = sweep;
            return 0;
        }
    }
    *sweeps = max_sweeps;
    return 1;
}

/* r = y~ - X~ beta over the fitted rows, recomputed from scratch */
void or_residual(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                 const double* c, const double* s, const double* ytilde, const double* beta, double* r) {
    for (int64_t i = 0; i < n_total; ++i) r[i] = in_fit(mask, i) ? ytilde[i] : 0.0;
    for (int64_t j = 0; j < p; ++j) {
        if (beta[j] == 0.0) continue;
        const double* x = X + j * ldx;
        for (int64_t i = 0; i < n_total; ++i)
            if (in_fit(mask, i)) r[i] -= beta[j] * ((x[i] - c[j]) / s[j]);
    }
}

/* Q(beta; lambda) = ||r||^2/(2n) + lambda ||beta||_1 with r = y~ - X~ beta */
double or_objective(int64_t n_total, const uint8_t* mask, const double* r, int64_t p, const double* beta,
                    double lambda) {
    int64_t n = count_rows(n_total, mask);
    double rss = 0.0, l1 = 0.0;
    for (int64_t i = 0; i < n_total; ++i)
        if (in_fit(mask, i)) rss += r[i] * r[i];
    for (int64_t j = 0; j < p; ++j) l1 += fabs(beta[j]);
    return rss / (2.0 * (double)n) + lambda * l1;
}

/* Elastic-net objective ||r||^2/(2n) + lambda sum_j w_j (alpha |beta_j| + (1 - alpha) beta_j^2 / 2) */
double or_objective_enet(int64_t n_total, const uint8_t* mask, const double* r, int64_t p, const double* beta,
                         double lambda, double alpha, const double* w) {
    int64_t n = count_rows(n_total, mask);
    double rss = 0.0, pen = 0.0;
    for (int64_t i = 0; i < n_total; ++i)
        if (in_fit(mask, i)) rss += r[i] * r[i];
    for (int64_t j = 0; j < p; ++j)
        pen += pw(w, j) * (alpha * fabs(beta[j]) + 0.5 * (1.0 - alpha) * beta[j] * beta[j]);
    return rss / (2.0 * (double)n) + lambda * pen;
}

/*
 * Relative duality gap of the elastic net, through its lasso form on augmented data: rows
 * sqrt(n lambda (1 - alpha) w_j) e_j' appended to X~ (and 0 to y~) turn the ridge part into squared
 * error, leaving the weighted lasso (1/2)||b - A beta||^2 + sum_j mu_j |beta_j| with mu_j = n lambda
 * alpha w_j.  Its residual rho = (r, -sqrt(n lambda (1 - alpha) w) beta) scaled by
 * t = min(1, min_j mu_j / |a_j' rho|), a_j' rho = n (z_j - lambda (1 - alpha) w_j beta_j), is dual
 * feasible: D = ||y~||^2/2 - (||y~ - t r||^2 + t^2 n lambda (1 - alpha) sum_j w_j beta_j^2)/2 and
 * P = n Q.  With alpha = 1 and no weights it is the lasso gap below.
 */
double or_duality_gap_enet(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                           const double* c, const double* s, const uint8_t* keep, const double* ytilde,
                           const double* r, const double* beta, double lambda, double alpha, const double* w) {
    int64_t n = count_rows(n_total, mask);
    double* z = (double*)malloc(sizeof(double) * (size_t)p);
    or_zscan(n_total, p, X, ldx, mask, c, s, keep, r, z);
    double t = 1.0, ridge = 0.0;
    for (int64_t j = 0; j < p; ++j) {
        if (!keep[j]) continue;
        double ar = (double)n * fabs(z[j] - lambda * (1.0 - alpha) * pw(w, j) * beta[j]);
        double mu = (double)n * lambda * alpha * pw(w, j);
        if (ar > 0.0 && mu / ar < t) t = mu / ar;
        ridge += pw(w, j) * beta[j] * beta[j];
    }
    free(z);
    double primal = (double)n * or_objective_enet(n_total, mask, r, p, beta, lambda, alpha, w);
    double yy = 0.0, dd = 0.0;
    for (int64_t i = 0; i < n_total; ++i) {
        if (!in_fit(mask, i)) continue;
        double d = ytilde[i] - t * r[i];
        yy += ytilde[i] * ytilde[i];
        dd += d * d;
    }
    dd += t * t * (double)n * lambda * (1.0 - alpha) * ridge;
    double dual = 0.5 * yy - 0.5 * dd;
    return primal > 0.0 ? (primal - dual) / primal : 0.0;
}

/*
 * Relative duality gap of beta at lambda.  Primal P = n Q; dual point
 * theta = r / max(n lambda, ||X~' r||_inf); D = ||y~||^2/2 - ||y~ - n lambda theta||^2/2.
 */
double or_duality_gap(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                      const double* c, const double* s, const uint8_t* keep, const double* ytilde,
                      const double* r, const double* beta, double lambda) {
    int64_t n = count_rows(n_total, mask);
    double* z = (double*)malloc(sizeof(double) * (size_t)p);
    or_zscan(n_total, p, X, ldx, mask, c, s, keep, r, z);
    double zmax = 0.0;
    for (int64_t j = 0; j < p; ++j)
        if (keep[j] && fabs(z[j]) * (double)n > zmax) zmax = fabs(z[j]) * (double)n;
    free(z);
    double nl = (double)n * lambda;
    double scale = zmax > nl ? zmax : nl;
    double primal = (double)n * or_objective(n_total, mask, r, p, beta, lambda);
    double yy = 0.0, dd = 0.0;
    for (int64_t i = 0; i < n_total; ++i) {
        if (!in_fit(mask, i)) continue;
        double theta = r[i] / scale;
        double d = ytilde[i] - nl * theta;
        yy += ytilde[i] * ytilde[i];
        dd += d * d;
    }
    double dual = 0.5 * yy - 0.5 * dd;
    return primal > 0.0 ? (primal - dual) / primal : 0.0;
}

/*
 * The lasso path over the geometric grid (or the decreasing grid lam_in when it is not NULL: cross-
 * validation fits every fold on the full-data grid) with warm starts, screened by the
 * sequential strong rule (or not screened) and repaired by a post-convergence
 * check over every kept feature:
 *   E_k = {j : beta_j != 0} u {j : |z_j(prev)| >= 2 l_k - l_{k-1}}
 * (OR_SCREEN_ACTIVE keeps only the first part, the previous active set: a
 * deliberately weak screen under which the check must add features back)
 *   repeat: CD over E_k; z = scan of all kept j;
 *           V = {j not in E_k : |z_j| > l_k}; stop if V is empty; E_k u= V.
 * BEDPP is evaluated only to report its survivor count; the solve never uses
 * it.  beta is p x K on the standardized scale.  Returns 0 on success, 1 if
 * CD did not converge (k_done then counts the finished lambdas), 2 on bad input.
 */
int or_fit_path(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                const double* y, int64_t K, double ratio, const double* lam_in, int screen, double tol,
                int64_t max_sweeps, double* c, double* s, uint8_t* keep, double* lambda, double* beta,
                double* ybar, or_path_stats* st, int64_t* k_done) {
    return or_fit_path_enet(n_total, p, X, ldx, mask, y, K, ratio, lam_in, 1.0, NULL, screen, tol, max_sweeps, c,
                            s, keep, lambda, beta, ybar, st, k_done);
}

/*
 * The path for the elastic-net penalty with feature weights (alpha in (0, 1], w_j > 0 or NULL).  What
 * changes against the lasso: lambda_max = max_j |a_j| / (alpha w_j); the strong rule keeps j when
 * |z_j(prev)| >= alpha w_j (2 l_k - l_{k-1}); a violation is |z_j| > l_k alpha w_j; the CD step is
 * or_cd_enet's; the objective and gap are the elastic net's.  BEDPP is a lasso rule: with alpha < 1 or
 * weights, n_safe reports every kept feature (no safe rule).
 */
int or_fit_path_enet(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                     const double* y, int64_t K, double ratio, const double* lam_in, double alpha, const double* w,
                     int screen, double tol, int64_t max_sweeps, double* c, double* s, uint8_t* keep,
                     double* lambda, double* beta, double* ybar, or_path_stats* st, int64_t* k_done) {
    *k_done = 0;
    if (!(alpha > 0.0 && alpha <= 1.0)) return 2;
    const int enet = alpha < 1.0 || w != NULL;
    if (p <= 0 || K <= 0) return 2;
    int64_t n = or_standardize(n_total, p, X, ldx, mask, c, s, keep);
    if (n <= 0) return 2;
    double* ytilde = (double*)calloc((size_t)n_total, sizeof(double));
    double* r = (double*)calloc((size_t)n_total, sizeof(double));
    double* a = (double*)calloc((size_t)p, sizeof(double));
    double* b = (double*)calloc((size_t)p, sizeof(double));
    double* z = (double*)calloc((size_t)p, sizeof(double));
    double* zprev = (double*)calloc((size_t)p, sizeof(double));
    double* bcur = (double*)calloc((size_t)p, sizeof(double));
    uint8_t* inE = (uint8_t*)calloc((size_t)p, 1);
    uint8_t* disc = (uint8_t*)calloc((size_t)p, 1);
    int64_t* set = (int64_t*)malloc(sizeof(int64_t) * (size_t)p);
    int status = 0;

    double lmax;
    int64_t jstar;
    if (or_lambda_max(n_total, p, X, ldx, mask, c, s, keep, y, ybar, ytilde, a, &lmax, &jstar)) {
        status = 2;
        goto done;
    }
    if (enet) {
        lmax = 0.0;
        for (int64_t j = 0; j < p; ++j)
            if (keep[j] && fabs(a[j]) / (alpha * pw(w, j)) > lmax) lmax = fabs(a[j]) / (alpha * pw(w, j));
    }
    or_bedpp_b(n_total, p, X, ldx, mask, c, s, keep, jstar, b);
    double v = 0.0;
    for (int64_t i = 0; i < n_total; ++i) v += ytilde[i] * ytilde[i];
    v /= (double)n;
    double sgn = a[jstar] >= 0 ? 1.0 : -1.0;
    if (lam_in)
        memcpy(lambda, lam_in, sizeof(double) * (size_t)K);
    else
        or_lambda_grid(lmax, ratio, K, lambda);
    memcpy(r, ytilde, sizeof(double) * (size_t)n_total);
    memcpy(zprev, a, sizeof(double) * (size_t)p);

    for (int64_t k = 0; k < K; ++k) {
        double lk = lambda[k];
        int64_t sweeps_k = 0, viol_k = 0, rounds_k = 0, nE = 0;
        /* beta = 0 solves every lambda >= lambda_max; below it, warm start from the previous lambda
         * (lambda_max, with z = a, before the first point of the grid) */
        if (lk < lmax) {
            double thr = 2.0 * lk - (k > 0 ? lambda[k - 1] : lmax);
            for (int64_t j = 0; j < p; ++j) {
                if (!keep[j]) {
                    inE[j] = 0;
                    continue;
                }
                if (screen == OR_SCREEN_NONE)
                    inE[j] = 1;
                else if (screen == OR_SCREEN_ACTIVE)
                    inE[j] = bcur[j] != 0.0 ? 1 : 0;
                else
                    inE[j] = (bcur[j] != 0.0 || fabs(zprev[j]) >= thr * alpha * pw(w, j)) ? 1 : 0;
            }
            for (;;) {
                nE = 0;
                for (int64_t j = 0; j < p; ++j)
                    if (inE[j]) set[nE++] = j;
                int64_t sw = 0;
                int rc = or_cd_enet(n_total, p, X, ldx, mask, c, s, lk, alpha, w, set, nE, bcur, r, tol, max_sweeps,
                                    &sw);
                sweeps_k += sw;
                rounds_k += 1;
                if (rc) {
                    status = 1;
                    goto done;
                }
                or_zscan(n_total, p, X, ldx, mask, c, s, keep, r, z);
                int64_t nv = 0;
                for (int64_t j = 0; j < p; ++j) {
                    if (keep[j] && !inE[j] && fabs(z[j]) > lk * alpha * pw(w, j)) {
                        inE[j] = 1;
                        ++nv;
                    }
                }
                viol_k += nv;
                if (nv == 0) break;
            }
            memcpy(zprev, z, sizeof(double) * (size_t)p);
        }
        memcpy(beta + k * p, bcur, sizeof(double) * (size_t)p);
        int64_t nact = 0;
        for (int64_t j = 0; j < p; ++j) nact += bcur[j] != 0.0;
        if (st) {
            if (st->sweeps) st->sweeps[k] = sweeps_k;
            if (st->n_strong) st->n_strong[k] = nE;
            if (st->n_viol) st->n_viol[k] = viol_k;
            if (st->n_rounds) st->n_rounds[k] = rounds_k;
            if (st->n_safe) {
                int64_t nk = 0;
                for (int64_t j = 0; j < p; ++j) nk += keep[j] != 0;
                st->n_safe[k] = enet ? nk : p - or_bedpp_discard(p, a, b, keep, lmax, sgn, v, lk, disc);
            }
            if (st->n_active) st->n_active[k] = nact;
            double rss = 0.0;
            for (int64_t i = 0; i < n_total; ++i) rss += r[i] * r[i];
            if (st->rss) st->rss[k] = rss;
            if (st->obj) st->obj[k] = or_objective_enet(n_total, mask, r, p, bcur, lk, alpha, w);
            if (st->gap)
                st->gap[k] = or_duality_gap_enet(n_total, p, X, ldx, mask, c, s, keep, ytilde, r, bcur, lk, alpha, w);
        }
        *k_done = k + 1;
    }
done:
    free(ytilde);
    free(r);
    free(a);
    free(b);
    free(z);
    free(zprev);
    free(bcur);
    free(inE);
    free(disc);
    free(set);
    return status;
}

/*
 * Lasso-penalized logistic regression (Section 1: the package fits sparse logistic regression; Section 2.2
 * pairs the strong rule with a safe rule for it).  y_i in {0, 1}, eta_i = b0 + x~_i' beta,
 *   Q(b0, beta) = (1/n) sum_i [log(1 + e^{eta_i}) - y_i eta_i] + lambda ||beta||_1   (b0 unpenalized).
 * z_j = x~_j' (y - pi) / n is the negative gradient, pi_i = 1 / (1 + e^{-eta_i}).  At beta = 0 the optimal
 * intercept is logit(y-bar) and lambda_max = max_j |x~_j' (y - y-bar)| / n.
 */
static double sigmoid(double e) { return e >= 0.0 ? 1.0 / (1.0 + exp(-e)) : exp(e) / (1.0 + exp(e)); }
static double log1pexp(double e) { return e > 0.0 ? e + log1p(exp(-e)) : log1p(exp(e)); }

double or_logistic_objective(int64_t n_total, const uint8_t* mask, const double* y, const double* eta, int64_t p,
                             const double* beta, double lambda) {
    int64_t n = count_rows(n_total, mask);
    double loss = 0.0, l1 = 0.0;
    for (int64_t i = 0; i < n_total; ++i)
        if (in_fit(mask, i)) loss += log1pexp(eta[i]) - y[i] * eta[i];
    for (int64_t j = 0; j < p; ++j) l1 += fabs(beta[j]);
    return loss / (double)n + lambda * l1;
}

/* negative binary entropy t log t + (1 - t) log(1 - t), 0 at t = 0 and t = 1 */
static double negent(double t) {
    double a = t > 0.0 ? t * log(t) : 0.0;
    double b = t < 1.0 ? (1.0 - t) * log(1.0 - t) : 0.0;
    return a + b;
}

/*
 * Relative duality gap of (b0, beta) at lambda.  With f_i(e) = log(1 + e^e) - y_i e the primal is
 * P = sum_i f_i(eta_i) + n lambda ||beta||_1 and the dual D(theta) = -sum_i f_i*(-n lambda theta_i) with
 * f_i*(u) = negent(u + y_i), over ||X~' theta||_inf <= 1 and sum_i theta_i = 0.  The dual point is the scaled
 * negative gradient theta = (y - pi) / max(n lambda, ||X~'(y - pi)||_inf).
 */
double or_logistic_gap(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                       const double* c, const double* s, const uint8_t* keep, const double* y, const double* eta,
                       const double* beta, double lambda) {
    int64_t n = count_rows(n_total, mask);
    double* g = (double*)calloc((size_t)n_total, sizeof(double));
    double* z = (double*)malloc(sizeof(double) * (size_t)p);
    for (int64_t i = 0; i < n_total; ++i) g[i] = in_fit(mask, i) ? y[i] - sigmoid(eta[i]) : 0.0;
    or_zscan(n_total, p, X, ldx, mask, c, s, keep, g, z);
    double zmax = 0.0;
    for (int64_t j = 0; j < p; ++j)
        if (keep[j] && fabs(z[j]) * (double)n > zmax) zmax = fabs(z[j]) * (double)n;
    double nl = (double)n * lambda;
    double scale = zmax > nl ? zmax : nl;
    double primal = (double)n * or_logistic_objective(n_total, mask, y, eta, p, beta, lambda);
    double dual = 0.0;
    for (int64_t i = 0; i < n_total; ++i)
        if (in_fit(mask, i)) dual -= negent(y[i] - nl * g[i] / scale);
    free(g);
    free(z);
    return primal > 0.0 ? (primal - dual) / primal : 0.0;
}

/*
 * The safe rule paired with the strong rule for logistic regression.  The rule the paper names (Slores) is not
 * printed in it; this one plays its part with the same inputs and cost as BEDPP: the gap-safe sphere around
 * the dual point known exactly at lambda_max (beta = 0, b0 = logit(y-bar), theta_max = (y - y-bar)/(n lambda_max)),
 * evaluated at lambda.  f_i has f_i'' <= 1/4, so the dual is 4 (n lambda)^2-strongly concave and the dual
 * optimum lies within r = sqrt(G / 2) / (n lambda) of theta_max, G the gap of (logit(y-bar), 0) and theta_max
 * at lambda.  With ||x~_j||_2 = sqrt(n), j is discarded when |x~_j' theta_max| + r sqrt(n) < 1, i.e.
 *   |a_j| < lambda_max (1 - sqrt(G / (2 n)) / lambda),   a_j = x~_j' (y - y-bar) / n.
 * G depends on lambda only through rho = lambda / lambda_max (closed form over the n1 ones and n0 zeros).
 * Returns that threshold on |a_j|; or_logistic_discard applies it.
 */
double or_logistic_safe_threshold(int64_t n, int64_t n1, double lambda_max, double lambda) {
    double yb = (double)n1 / (double)n;
    double n0 = (double)(n - n1);
    double P = -((double)n1 * log(yb) + n0 * log(1.0 - yb));
    double rho = lambda / lambda_max;
    if (rho > 1.0) rho = 1.0;
    double D = -((double)n1 * negent(1.0 - rho * (1.0 - yb)) + n0 * negent(rho * yb));
    double G = P - D;
    if (G < 0.0) G = 0.0;
    return lambda_max * (1.0 - sqrt(G / (2.0 * (double)n)) / lambda);
}

int64_t or_logistic_discard(int64_t p, const double* a, const uint8_t* keep, double thr, uint8_t* discard) {
    int64_t cnt = 0;
    for (int64_t j = 0; j < p; ++j) {
        discard[j] = (!keep[j] || fabs(a[j]) < thr) ? 1 : 0;
        cnt += discard[j];
    }
    return cnt;
}

/*
 * The logistic lasso path with warm starts, the strong rule on z of the previous lambda and the
 * post-convergence check over every kept feature, as for the linear path.  Each solve is iteratively
 * reweighted least squares with cyclic coordinate descent on its quadratic model (the pathwise method the
 * package builds on): weights w_i = pi_i (1 - pi_i) (at least 1e-5), working residual r_i = (y_i - pi_i) / w_i,
 * coordinate step beta_j' = S(sum_i w_i x~_ij r_i / n + v_j beta_j, lambda) / v_j with v_j = sum_i w_i x~_ij^2 / n,
 * intercept step sum_i w_i r_i / sum_i w_i; inner sweeps until the largest change is below tol, outer
 * iterations until an iteration changes no coefficient (intercept included) by tol or more.
 * beta is p x K, b0 has K entries (standardized scale).  Returns 0, 1 (not converged) or 2 (bad input,
 * e.g. y not in {0, 1} or constant on the fitted rows).
 */
int or_fit_path_logistic(int64_t n_total, int64_t p, const double* X, int64_t ldx, const uint8_t* mask,
                         const double* y, int64_t K, double ratio, int screen, double tol, int64_t max_iter,
                         double* c, double* s, uint8_t* keep, double* lambda, double* beta, double* b0out,
                         or_path_stats* st, int64_t* k_done) {
    *k_done = 0;
    if (p <= 0 || K <= 0) return 2;
    int64_t n = or_standardize(n_total, p, X, ldx, mask, c, s, keep);
    if (n <= 0) return 2;
    int64_t n1 = 0;
    for (int64_t i = 0; i < n_total; ++i) {
        if (!in_fit(mask, i)) continue;
        if (y[i] != 0.0 && y[i] != 1.0) return 2;
        n1 += y[i] == 1.0;
    }
    if (n1 == 0 || n1 == n) return 2;
    double yb = (double)n1 / (double)n;
    double* ym = (double*)calloc((size_t)n_total, sizeof(double));
    double* eta = (double*)calloc((size_t)n_total, sizeof(double));
    double* w = (double*)calloc((size_t)n_total, sizeof(double));
    double* r = (double*)calloc((size_t)n_total, sizeof(double));
    double* g = (double*)calloc((size_t)n_total, sizeof(double));
    double* a = (double*)calloc((size_t)p, sizeof(double));
    double* z = (double*)calloc((size_t)p, sizeof(double));
    double* zprev = (double*)calloc((size_t)p, sizeof(double));
    double* bcur = (double*)calloc((size_t)p, sizeof(double));
    uint8_t* inE = (uint8_t*)calloc((size_t)p, 1);
    uint8_t* disc = (uint8_t*)calloc((size_t)p, 1);
    int status = 0;
    for (int64_t i = 0; i < n_total; ++i) ym[i] = in_fit(mask, i) ? y[i] - yb : 0.0;
    or_zscan(n_total, p, X, ldx, mask, c, s, keep, ym, a);
    double lmax = 0.0;
    for (int64_t j = 0; j < p; ++j)
        if (keep[j] && fabs(a[j]) > lmax) lmax = fabs(a[j]);
    or_lambda_grid(lmax, ratio, K, lambda);
    double b0 = log(yb / (1.0 - yb));
    for (int64_t i = 0; i < n_total; ++i) eta[i] = in_fit(mask, i) ? b0 : 0.0;
    memcpy(zprev, a, sizeof(double) * (size_t)p);

    for (int64_t k = 0; k < K; ++k) {
        double lk = lambda[k];
        int64_t sweeps_k = 0, viol_k = 0, rounds_k = 0, nE = 0;
        if (lk < lmax) {
            double thr = 2.0 * lk - (k > 0 ? lambda[k - 1] : lmax);
            for (int64_t j = 0; j < p; ++j) {
                if (!keep[j]) inE[j] = 0;
                else if (screen == OR_SCREEN_NONE) inE[j] = 1;
                else if (screen == OR_SCREEN_ACTIVE) inE[j] = bcur[j] != 0.0;
                else inE[j] = (bcur[j] != 0.0 || fabs(zprev[j]) >= thr) ? 1 : 0;
            }
            for (;;) {
                nE = 0;
                for (int64_t j = 0; j < p; ++j) nE += inE[j];
                /* IRLS over E */
                int64_t it = 0;
                for (;;) {
                    double wsum = 0.0;
                    for (int64_t i = 0; i < n_total; ++i) {
                        if (!in_fit(mask, i)) continue;
                        double pi = sigmoid(eta[i]);
                        double wi = pi * (1.0 - pi);
                        if (wi < 1e-5) wi = 1e-5;
                        w[i] = wi;
                        r[i] = (y[i] - pi) / wi;
                        wsum += wi;
                    }
                    double outer_max = 0.0;
                    for (int64_t sweep = 1;; ++sweep) {
                        double mx = 0.0;
                        /* intercept */
                        double num = 0.0;
                        for (int64_t i = 0; i < n_total; ++i)
                            if (in_fit(mask, i)) num += w[i] * r[i];
                        double d0 = num / wsum;
                        if (d0 != 0.0) {
                            b0 += d0;
                            for (int64_t i = 0; i < n_total; ++i)
                                if (in_fit(mask, i)) {
                                    r[i] -= d0;
                                    eta[i] += d0;
                                }
                        }
                        if (fabs(d0) > mx) mx = fabs(d0);
                        for (int64_t j = 0; j < p; ++j) {
                            if (!inE[j]) continue;
                            const double* x = X + j * ldx;
                            double xwr = 0.0, xwx = 0.0;
                            for (int64_t i = 0; i < n_total; ++i) {
                                if (!in_fit(mask, i)) continue;
                                double xt = (x[i] - c[j]) / s[j];
                                xwr += w[i] * xt * r[i];
                                xwx += w[i] * xt * xt;
                            }
                            xwr /= (double)n;
                            xwx /= (double)n;
                            double bnew = soft_threshold(xwr + xwx * bcur[j], lk) / xwx;
                            double dlt = bnew - bcur[j];
                            if (dlt != 0.0) {
                                for (int64_t i = 0; i < n_total; ++i) {
                                    if (!in_fit(mask, i)) continue;
                                    double xt = (x[i] - c[j]) / s[j];
                                    r[i] -= dlt * xt;
                                    eta[i] += dlt * xt;
                                }
                                bcur[j] = bnew;
                            }
                            if (fabs(dlt) > mx) mx = fabs(dlt);
                        }
                        ++sweeps_k;
                        if (mx > outer_max) outer_max = mx;
                        if (mx < tol) break;
                        if (sweeps_k > max_iter) {
                            status = 1;
                            goto done;
                        }
                    }
                    ++it;
                    if (outer_max < tol) break;
                    if (it > max_iter) {
                        status = 1;
                        goto done;
                    }
                }
                rounds_k += 1;
                for (int64_t i = 0; i < n_total; ++i) g[i] = in_fit(mask, i) ? y[i] - sigmoid(eta[i]) : 0.0;
                or_zscan(n_total, p, X, ldx, mask, c, s, keep, g, z);
                int64_t nv = 0;
                for (int64_t j = 0; j < p; ++j)
                    if (keep[j] && !inE[j] && fabs(z[j]) > lk) {
                        inE[j] = 1;
                        ++nv;
                    }
                viol_k += nv;
                if (nv == 0) break;
            }
            memcpy(zprev, z, sizeof(double) * (size_t)p);
        }
        memcpy(beta + k * p, bcur, sizeof(double) * (size_t)p);
        b0out[k] = b0;
        if (st) {
            int64_t nact = 0;
            for (int64_t j = 0; j < p; ++j) nact += bcur[j] != 0.0;
            if (st->sweeps) st->sweeps[k] = sweeps_k;
            if (st->n_strong) st->n_strong[k] = nE;
            if (st->n_viol) st->n_viol[k] = viol_k;
            if (st->n_rounds) st->n_rounds[k] = rounds_k;
            if (st->n_active) st->n_active[k] = nact;
            if (st->n_safe)
                st->n_safe[k] = p - or_logistic_discard(p, a, keep, or_logistic_safe_threshold(n, n1, lmax, lk), disc);
            if (st->rss) st->rss[k] = 0.0;
            if (st->obj) st->obj[k] = or_logistic_objective(n_total, mask, y, eta, p, bcur, lk);
            if (st->gap) st->gap[k] = or_logistic_gap(n_total, p, X, ldx, mask, c, s, keep, y, eta, bcur, lk);
        }
        *k_done = k + 1;
    }
done:
    free(ym);
    free(eta);
    free(w);
    free(r);
    free(g);
    free(a);
    free(z);
    free(zprev);
    free(bcur);
    free(inE);
    free(disc);
    return status;
}

/*
 * Screening network used by the learned form: 4 inputs -> H (ReLU) -> H (ReLU)
 * -> 1 logit -> logistic.  Parameter vector layout:
 *   W1[H][4], b1[H], W2[H][H], b2[H], w3[H], b3.
 * The paper has no such network; this is the plain definition of the model
 * the GPU form trains, so its outputs and gradients can be checked.
 */
static double relu(double x) { return x > 0.0 ? x : 0.0; }

static void mlp_one(int64_t H, const double* f, const double* P, double* h1, double* h2, double* logit) {
    const double* W1 = P;
    const double* b1 = W1 + H * 4;
    const double* W2 = b1 + H;
    const double* b2 = W2 + H * H;
    const double* w3 = b2 + H;
    const double* b3 = w3 + H;
    for (int64_t u = 0; u < H; ++u) {
        double acc = b1[u];
        for (int64_t q = 0; q < 4; ++q) acc += W1[u * 4 + q] * f[q];
        h1[u] = relu(acc);
    }
    for (int64_t u = 0; u < H; ++u) {
        double acc = b2[u];
        for (int64_t q = 0; q < H; ++q) acc += W2[u * H + q] * h1[q];
        h2[u] = relu(acc);
    }
    double o = b3[0];
    for (int64_t u = 0; u < H; ++u) o += w3[u] * h2[u];
    *logit = o;
}

void or_mlp_forward(int64_t m, int64_t H, const double* feat, const double* params, double* prob) {
    double* h1 = (double*)malloc(sizeof(double) * (size_t)H);
    double* h2 = (double*)malloc(sizeof(double) * (size_t)H);
    for (int64_t t = 0; t < m; ++t) {
        double o;
        mlp_one(H, feat + t * 4, params, h1, h2, &o);
        prob[t] = 1.0 / (1.0 + exp(-o));
    }
    free(h1);
    free(h2);
}

/*
 * Mean binary cross-entropy over m rows, L = (1/m) sum [log(1 + e^o) - y o],
 * and its gradient with respect to every parameter (back-propagation through
 * the layers above, written out per layer).
 */
double or_mlp_loss_grad(int64_t m, int64_t H, const double* feat, const double* label, const double* params,
                        double* grad) {
    int64_t np = H * H + 7 * H + 1;
    memset(grad, 0, sizeof(double) * (size_t)np);
    double* g_W1 = grad;
    double* g_b1 = g_W1 + H * 4;
    double* g_W2 = g_b1 + H;
    double* g_b2 = g_W2 + H * H;
    double* g_w3 = g_b2 + H;
    double* g_b3 = g_w3 + H;
    const double* W2 = params + H * 4 + H;
    const double* w3 = W2 + H * H + H;
    double* h1 = (double*)malloc(sizeof(double) * (size_t)H);
    double* h2 = (double*)malloc(sizeof(double) * (size_t)H);
    double* d2 = (double*)malloc(sizeof(double) * (size_t)H);
    double* d1 = (double*)malloc(sizeof(double) * (size_t)H);
    double loss = 0.0;
    for (int64_t t = 0; t < m; ++t) {
        const double* f = feat + t * 4;
        double o;
        mlp_one(H, f, params, h1, h2, &o);
        double y = label[t];
        double sp = o > 0.0 ? o + log1p(exp(-o)) : log1p(exp(o));
        loss += sp - y * o;
        double dout = (1.0 / (1.0 + exp(-o)) - y) / (double)m;
        g_b3[0] += dout;
        for (int64_t u = 0; u < H; ++u) {
            g_w3[u] += dout * h2[u];
            d2[u] = h2[u] > 0.0 ? dout * w3[u] : 0.0;
        }
        for (int64_t u = 0; u < H; ++u) {
            g_b2[u] += d2[u];
            for (int64_t q = 0; q < H; ++q) g_W2[u * H + q] += d2[u] * h1[q];
        }
        for (int64_t q = 0; q < H; ++q) {
            double acc = 0.0;
            for (int64_t u = 0; u < H; ++u) acc += W2[u * H + q] * d2[u];
            d1[q] = h1[q] > 0.0 ? acc : 0.0;
        }
        for (int64_t u = 0; u < H; ++u) {
            g_b1[u] += d1[u];
            for (int64_t q = 0; q < 4; ++q) g_W1[u * 4 + q] += d1[u] * f[q];
        }
    }
    free(h1);
    free(h2);
    free(d2);
    free(d1);
    return loss / (double)m;
}
