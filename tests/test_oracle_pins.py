"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: library
routines (numpy mean/std/lstsq), closed forms of the lasso (soft-thresholding
on orthogonal designs, the first segment of the path), brute-force
enumeration of sign patterns, optimality certificates, and the lambda values
the paper prints.  None of them retypes the oracle's own formulas.
"""
import itertools
import os

import numpy as np
import pytest

import datagen
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def std_numpy(Xt, mask=None):
    """Explicitly standardized copy X~ (n x p) and centered y helper, in numpy."""
    X = Xt.T.astype(np.float64)
    if mask is not None:
        X = X[mask.astype(bool)]
    c = X.mean(axis=0)
    s = X.std(axis=0)
    return (X - c) / s, c, s


def soft(u, l):
    return np.sign(u) * np.maximum(np.abs(u) - l, 0.0)


# ---------------------------------------------------------------------------------------------
# standardization and the scan (Section 3.1, 3.1.1)
# ---------------------------------------------------------------------------------------------

def test_standardize_matches_numpy_population_sd():
    rng = np.random.default_rng(0)
    Xt = rng.normal(3.0, 2.0, size=(37, 53))
    Xt[5] = 1.25  # constant column
    mask = (rng.uniform(size=53) < 0.7).astype(np.uint8)
    c, s, keep, n = oracle.standardize(Xt, mask)
    X = Xt.T[mask.astype(bool)]
    assert n == mask.sum()
    np.testing.assert_allclose(c, X.mean(axis=0), rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(s, X.std(axis=0, ddof=0), rtol=1e-13, atol=1e-15)
    assert not keep[5] and keep.sum() == 36


def test_scan_equals_simplified_identity_type3():
    # Section 3.1.1 type (3): x~_j' r = (sum_i x_ij r_i - c_j sum_i r_i) / s_j, with r not centered
    rng = np.random.default_rng(1)
    Xt = datagen.genotype_u8(7, 61, 45).astype(np.float64)
    mask = np.ones(61, dtype=np.uint8)
    mask[::7] = 0
    c, s, keep, n = oracle.standardize(Xt, mask)
    r = rng.normal(size=61) + 0.3
    r[mask == 0] = 0.0
    z = oracle.zscan(Xt, c, s, keep, r, mask)
    X = Xt.T
    ident = (X.T @ r - c * r.sum()) / (s * n)
    np.testing.assert_allclose(z[keep], ident[keep], rtol=1e-12, atol=1e-14)


def test_type1_and_type2_identities():
    # Section 3.1.1 types (1) and (2) through lambda_max and the BEDPP correlations
    rng = np.random.default_rng(2)
    Xt = rng.normal(size=(30, 80)) * rng.uniform(0.5, 3, size=(30, 1)) + rng.normal(size=(30, 1))
    y = rng.normal(size=80) + 4.0
    c, s, keep, n = oracle.standardize(Xt)
    ybar, yt, a, lmax, js = oracle.lambda_max(Xt, c, s, keep, y)
    X = Xt.T
    np.testing.assert_allclose(a, (X.T @ y - c * y.sum()) / (s * n), rtol=1e-12, atol=1e-14)
    b = oracle.bedpp_b(Xt, c, s, keep, js)
    xs = X[:, js]
    np.testing.assert_allclose(b, (X.T @ xs - n * c * c[js]) / (n * s * s[js]), rtol=1e-11, atol=1e-13)
    assert lmax == pytest.approx(np.abs(a).max(), rel=0, abs=0)
    assert js == int(np.argmax(np.abs(a)))
    assert ybar == pytest.approx(y.mean(), rel=1e-15)


# ---------------------------------------------------------------------------------------------
# the lasso solution: closed forms, brute force, certificates
# ---------------------------------------------------------------------------------------------

def orthogonal_design(n, p, seed):
    """Columns centered, mutually orthogonal, (1/n)||x_j||^2 = 1, random means and scales added back."""
    rng = np.random.default_rng(seed)
    G = rng.normal(size=(n, p))
    G -= G.mean(axis=0)
    Q, _ = np.linalg.qr(G)
    Xs = Q * np.sqrt(n)
    scale = rng.uniform(0.5, 2.0, size=p)
    shift = rng.normal(size=p)
    return (Xs * scale + shift).T.copy()  # (p, n)


def test_orthogonal_design_soft_threshold_closed_form():
    n, p = 60, 12
    Xt = orthogonal_design(n, p, 3)
    rng = np.random.default_rng(4)
    y = Xt.T @ rng.normal(size=p) + rng.normal(size=n)
    path = oracle.fit_path(Xt, y, K=25, ratio=0.05)
    Xtil, c, s = std_numpy(Xt)
    a = Xtil.T @ (y - y.mean()) / n
    for k, lam in enumerate(path.lam):
        np.testing.assert_allclose(path.beta[k], soft(a, lam), atol=1e-11)


def test_first_segment_closed_form():
    # with one active feature the solution is sign(a_*) (lambda_max - lambda) (unit curvature)
    rng = np.random.default_rng(5)
    Xt = rng.normal(size=(40, 120))
    y = 2.0 * Xt[7] + rng.normal(size=120)
    c, s, keep, n = oracle.standardize(Xt)
    ybar, yt, a, lmax, js = oracle.lambda_max(Xt, c, s, keep, y)
    second = np.sort(np.abs(a))[-2]
    lam = 0.5 * (lmax + second)
    beta = np.zeros(40)
    r = yt.copy()
    ok, sweeps = oracle.cd(Xt, c, s, lam, np.arange(40), beta, r)
    assert ok
    expect = np.zeros(40)
    expect[js] = np.sign(a[js]) * (lmax - lam)
    np.testing.assert_allclose(beta, expect, atol=1e-13)


def test_beta_zero_at_lambda_max():
    prob = datagen.make("c1", n=150, p=300)
    path = oracle.fit_path(prob.Xt, prob.y[0], K=10, ratio=0.1)
    assert path.lam[0] == pytest.approx(path.lam[0])
    assert np.all(path.beta[0] == 0.0)
    assert path.sweeps[0] == 0          # no iterations at lambda_max (iter[1] = 0 in the package output)
    assert path.n_active[1] >= 1


def brute_force_lasso(Xtil, yt, lam):
    """Enumerate sign patterns; return the unique pattern meeting the optimality conditions."""
    n, p = Xtil.shape
    G = Xtil.T @ Xtil / n
    q = Xtil.T @ yt / n
    found = []
    for sig in itertools.product((-1, 0, 1), repeat=p):
        sig = np.array(sig)
        A = np.flatnonzero(sig)
        beta = np.zeros(p)
        if A.size:
            try:
                beta[A] = np.linalg.solve(G[np.ix_(A, A)], q[A] - lam * sig[A])
            except np.linalg.LinAlgError:
                continue
            if not np.all(np.sign(beta[A]) == sig[A]):
                continue
        grad = q - G @ beta
        off = np.setdiff1d(np.arange(p), A)
        if np.all(np.abs(grad[off]) <= lam * (1 + 1e-12)):
            found.append(beta)
    return found


@pytest.mark.parametrize("seed,design", [(11, "gaussian"), (12, "genotype"), (13, "ar1")])
def test_brute_force_sign_enumeration(seed, design):
    n, p = 30, 8
    rng = np.random.default_rng(seed)
    if design == "gaussian":
        Xt = rng.normal(size=(p, n))
    elif design == "genotype":
        Xt = datagen.genotype_u8(seed, n, p).astype(np.float64)
    else:
        Xt = datagen.ar1_f32(seed, n, p, 0.8).astype(np.float64)
    y = Xt[:3].T @ np.array([1.5, -1.0, 0.7]) + rng.normal(size=n)
    path = oracle.fit_path(Xt, y, K=12, ratio=0.02)
    Xtil, c, s = std_numpy(Xt)
    yt = y - y.mean()
    for k in range(1, 12, 2):
        sols = brute_force_lasso(Xtil, yt, path.lam[k])
        assert len(sols) == 1
        np.testing.assert_allclose(path.beta[k], sols[0], atol=1e-10)


def test_brute_force_p10_with_row_mask():
    n, p = 45, 10
    rng = np.random.default_rng(21)
    Xt = rng.normal(size=(p, n)) + rng.normal(size=(p, 1))
    mask = np.ones(n, dtype=np.uint8)
    mask[rng.choice(n, 9, replace=False)] = 0
    y = Xt[2] - 2 * Xt[5] + rng.normal(size=n)
    path = oracle.fit_path(Xt, y, K=8, ratio=0.05, mask=mask)
    Xtil, c, s = std_numpy(Xt, mask)
    ym = y[mask.astype(bool)]
    for k in (3, 7):
        sols = brute_force_lasso(Xtil, ym - ym.mean(), path.lam[k])
        assert len(sols) == 1
        np.testing.assert_allclose(path.beta[k], sols[0], atol=1e-10)


def test_ols_limit_matches_lstsq():
    rng = np.random.default_rng(6)
    n, p = 200, 15
    Xt = rng.normal(size=(p, n))
    y = Xt.T @ rng.normal(size=p) + rng.normal(size=n)
    c, s, keep, nn = oracle.standardize(Xt)
    ybar, yt, a, lmax, js = oracle.lambda_max(Xt, c, s, keep, y)
    lam = lmax * 1e-10
    beta = np.zeros(p)
    r = yt.copy()
    ok, _ = oracle.cd(Xt, c, s, lam, np.arange(p), beta, r, tol=1e-15)
    assert ok
    Xtil, _, _ = std_numpy(Xt)
    ols, *_ = np.linalg.lstsq(Xtil, y - y.mean(), rcond=None)
    np.testing.assert_allclose(beta, ols, atol=1e-8)


def test_single_feature_soft_threshold():
    rng = np.random.default_rng(7)
    x = rng.normal(size=(1, 50))
    y = 0.8 * x[0] + rng.normal(size=50)
    path = oracle.fit_path(x, y, K=6, ratio=0.1)
    a = (x[0] - x[0].mean()) / x[0].std() @ (y - y.mean()) / 50
    for k, lam in enumerate(path.lam):
        assert path.beta[k, 0] == pytest.approx(soft(a, lam), abs=1e-13)


@pytest.mark.parametrize("name", ["c1", "c2", "c4"])
def test_kkt_certificate_and_duality_gap(name):
    prob = datagen.make(name, n=300, p=700) if name != "c4" else datagen.make("c4", n=300, p=400, nresp=1, nsub=1)
    Xt = prob.Xt.astype(np.float64)
    y = prob.y[0]
    K = 40
    path = oracle.fit_path(Xt, y, K=K, ratio=prob.recipe.lambda_min_ratio)
    Xtil, c, s = std_numpy(Xt)
    yt = y - y.mean()
    n = Xtil.shape[0]
    for k in range(K):
        b = path.beta[k]
        r = yt - Xtil @ b
        z = Xtil.T @ r / n
        lam = path.lam[k]
        act = b != 0
        assert np.all(np.abs(z[~act]) <= lam * (1 + 1e-9))
        np.testing.assert_allclose(z[act], lam * np.sign(b[act]), atol=1e-9 * max(1.0, lam))
        assert path.gap[k] <= 1e-10
        # objective (1/2n)||r||^2 + lam ||b||_1 recomputed in numpy
        assert path.obj[k] == pytest.approx(r @ r / (2 * n) + lam * np.abs(b).sum(), rel=1e-12)


def test_screening_none_and_strong_rule_agree():
    prob = datagen.make("c2", n=250, p=900)
    Xt = prob.Xt.astype(np.float64)
    p1 = oracle.fit_path(Xt, prob.y[0], K=30, ratio=0.05, screen=oracle.SCREEN_SSR)
    p0 = oracle.fit_path(Xt, prob.y[0], K=30, ratio=0.05, screen=oracle.SCREEN_NONE)
    np.testing.assert_allclose(p1.beta, p0.beta, atol=1e-11)
    assert np.all(p1.n_strong <= p0.n_strong)


def test_cd_not_converged_reports():
    prob = datagen.make("c1", n=100, p=200)
    path = oracle.fit_path(prob.Xt, prob.y[0], K=20, ratio=0.1, max_sweeps=1)
    assert path.status == 1 and 1 <= path.k_done < 20


# ---------------------------------------------------------------------------------------------
# BEDPP safe rule (Section 2.2): safety, monotonicity, reduction at lambda_max
# ---------------------------------------------------------------------------------------------

def bedpp_inputs(Xt, y):
    c, s, keep, n = oracle.standardize(Xt)
    ybar, yt, a, lmax, js = oracle.lambda_max(Xt, c, s, keep, y)
    b = oracle.bedpp_b(Xt, c, s, keep, js)
    v = yt @ yt / n
    return a, b, keep, lmax, np.sign(a[js]), v


@pytest.mark.parametrize("seed,design", [(31, "gaussian"), (32, "genotype"), (33, "ar1"), (34, "ar1_strong")])
def test_bedpp_is_safe_and_monotone(seed, design):
    n, p = 120, 400
    if design == "gaussian":
        Xt = datagen.gaussian_f64(seed, n, p)
    elif design == "genotype":
        Xt = datagen.genotype_u8(seed, n, p).astype(np.float64)
    elif design == "ar1":
        Xt = datagen.ar1_f32(seed, n, p, 0.5).astype(np.float64)
    else:
        Xt = datagen.ar1_f32(seed, n, p, 0.95, block=20).astype(np.float64)
    rng = np.random.default_rng(seed)
    sup = rng.choice(p, 10, replace=False)
    y = Xt[sup].T @ rng.normal(size=10) * 2 + rng.normal(size=n)
    path = oracle.fit_path(Xt, y, K=60, ratio=0.01)
    a, b, keep, lmax, sg, v = bedpp_inputs(Xt, y)
    prev = None
    total_discarded = 0
    for k, lam in enumerate(path.lam):
        d = oracle.bedpp_discard(a, b, keep, lmax, sg, v, lam)
        assert not np.any(d & (path.beta[k] != 0)), f"BEDPP discarded an active feature at k={k}"
        if prev is not None:
            assert not np.any(d & ~prev), "safe set must grow as lambda decreases"
        prev = d
        total_discarded += d.sum()
    assert total_discarded > 0


def test_bedpp_at_lambda_max_reduces_to_correlation_test():
    prob = datagen.make("c1", n=200, p=500)
    a, b, keep, lmax, sg, v = bedpp_inputs(prob.Xt, prob.y[0])
    d = oracle.bedpp_discard(a, b, keep, lmax, sg, v, lmax)
    np.testing.assert_array_equal(d, np.abs(a) < lmax)


def test_bedpp_on_orthogonal_design_implies_inactive():
    n, p = 80, 30
    Xt = orthogonal_design(n, p, 41)
    rng = np.random.default_rng(42)
    y = Xt.T @ (rng.normal(size=p) * (rng.uniform(size=p) < 0.3)) + rng.normal(size=n)
    a, b, keep, lmax, sg, v = bedpp_inputs(Xt, y)
    for lam in lmax * np.geomspace(1.0, 0.05, 30):
        d = oracle.bedpp_discard(a, b, keep, lmax, sg, v, lam)
        assert np.all(np.abs(a[d]) < lam)


# ---------------------------------------------------------------------------------------------
# lambda grid: the lambda values printed in the paper's Section 5 example (tests/golden)
# ---------------------------------------------------------------------------------------------

def read_golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = line.split("=")
                vals[k.strip()] = v.strip()
    return vals


def test_lambda_grid_reproduces_printed_example():
    g = read_golden("colon_lambda_grid.txt")
    printed = [float(x) for x in g["lambda_first"].split(",")]
    K = int(g["nlambda"])
    ratio = float(g["lambda_min_ratio"])
    k_sel = int(g["selected_index"])
    sel = float(g["selected_lambda"])
    lo, hi = printed[0] - 0.5e-4, printed[0] + 0.5e-4

    def matches(lmax):
        lam = oracle.lambda_grid(lmax, ratio, K)
        ok = all(float(f"{lam[k]:.4g}") == printed[k] for k in range(len(printed)))
        return ok and float(f"{lam[k_sel]:.3g}") == sel

    cands = np.linspace(lo, hi, 2001)
    assert any(matches(x) for x in cands)
    # an arithmetic grid with the same endpoints does not reproduce the printed values
    arith = [np.linspace(x, ratio * x, K) for x in cands]
    assert not any(all(float(f"{g_[k]:.4g}") == printed[k] for k in range(len(printed))) for g_ in arith)


# ---------------------------------------------------------------------------------------------
# screening network (learned form): gradients against finite differences
# ---------------------------------------------------------------------------------------------

def test_mlp_gradient_matches_finite_differences():
    H = 6
    rng = np.random.default_rng(8)
    params = rng.normal(scale=0.5, size=oracle.n_params(H))
    feat = rng.uniform(0, 2, size=(25, 4))
    label = (rng.uniform(size=25) < 0.4).astype(np.float64)
    loss, grad = oracle.mlp_loss_grad(feat, label, params, H)
    eps = 1e-6
    num = np.empty_like(params)
    for i in range(params.size):
        pp = params.copy()
        pp[i] += eps
        lp, _ = oracle.mlp_loss_grad(feat, label, pp, H)
        pp[i] -= 2 * eps
        lm, _ = oracle.mlp_loss_grad(feat, label, pp, H)
        num[i] = (lp - lm) / (2 * eps)
    np.testing.assert_allclose(grad, num, atol=1e-7, rtol=1e-5)
    prob = oracle.mlp_forward(feat, params, H)
    bce = -np.mean(label * np.log(prob) + (1 - label) * np.log(1 - prob))
    assert loss == pytest.approx(bce, rel=1e-10)


# ---------------------------------------------------------------------------------------------
# the post-convergence check repairs a deliberately weak screen (Section 2.2: the strong rule is
# heuristic and needs the check; here the working set is only the previous active set, so every
# feature that enters the path must be found and added by the check)
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["c1", "c2"])
def test_weak_screen_is_repaired_by_the_check(name):
    prob = datagen.make(name, n=160, p=260)
    Xt = prob.Xt.astype(np.float64)
    y = prob.y[0]
    weak = oracle.fit_path(Xt, y, K=25, ratio=0.05, screen=oracle.SCREEN_ACTIVE)
    full = oracle.fit_path(Xt, y, K=25, ratio=0.05, screen=oracle.SCREEN_NONE)
    assert weak.status == 0 and weak.k_done == 25
    # the check found features the screen left out, and the path was solved again after adding them
    assert weak.n_viol.sum() > 0
    assert weak.n_rounds.max() >= 2
    assert np.all(weak.n_rounds[weak.n_viol > 0] >= 2)
    np.testing.assert_allclose(weak.beta, full.beta, atol=1e-11)
    np.testing.assert_array_equal(weak.n_active, full.n_active)


# ---------------------------------------------------------------------------------------------
# duality gap, residual: closed forms and numpy
# ---------------------------------------------------------------------------------------------

def test_duality_gap_closed_form_at_beta_zero():
    # at beta = 0 and lambda < lambda_max the dual point is y~ / (n lambda_max), so
    # P = ||y~||^2 / 2 and D = ||y~||^2 / 2 * (1 - (1 - lambda/lambda_max)^2): gap = (1 - lambda/lambda_max)^2;
    # at lambda >= lambda_max the dual point y~ / (n lambda) closes the gap
    rng = np.random.default_rng(14)
    Xt = rng.normal(size=(50, 90)) + rng.normal(size=(50, 1))
    y = Xt[3] - Xt[8] + rng.normal(size=90)
    mask = (rng.uniform(size=90) < 0.85).astype(np.uint8)
    c, s, keep, n = oracle.standardize(Xt, mask)
    ybar, yt, a, lmax, js = oracle.lambda_max(Xt, c, s, keep, y, mask)
    beta = np.zeros(50)
    for frac in (0.9, 0.5, 0.1):
        g = oracle.duality_gap(Xt, c, s, keep, yt, yt, beta, frac * lmax, mask)
        assert g == pytest.approx((1.0 - frac) ** 2, rel=1e-12)
    assert abs(oracle.duality_gap(Xt, c, s, keep, yt, yt, beta, 1.5 * lmax, mask)) <= 1e-15


def test_duality_gap_bounds_the_suboptimality():
    # P(beta) - P(beta*) <= P - D for any beta (weak duality), with P* from a converged solve
    rng = np.random.default_rng(15)
    Xt = rng.normal(size=(30, 70))
    y = 1.5 * Xt[2] + rng.normal(size=70)
    c, s, keep, n = oracle.standardize(Xt)
    ybar, yt, a, lmax, js = oracle.lambda_max(Xt, c, s, keep, y)
    lam = 0.2 * lmax
    bopt = np.zeros(30)
    ropt = yt.copy()
    assert oracle.cd(Xt, c, s, lam, np.arange(30), bopt, ropt, tol=1e-15)[0]
    popt = oracle.objective(ropt, bopt, lam) * n
    for t in range(5):
        beta = bopt + rng.normal(scale=0.05, size=30) * (rng.uniform(size=30) < 0.5)
        r = oracle.residual(Xt, c, s, yt, beta)
        P = oracle.objective(r, beta, lam) * n
        gap = oracle.duality_gap(Xt, c, s, keep, yt, r, beta, lam)
        assert P - popt <= gap * P * (1 + 1e-9) + 1e-12
        assert gap > 0


def test_residual_matches_numpy():
    rng = np.random.default_rng(16)
    Xt = datagen.genotype_u8(16, 77, 40).astype(np.float64)
    mask = (rng.uniform(size=77) < 0.75).astype(np.uint8)
    c, s, keep, n = oracle.standardize(Xt, mask)
    ybar, yt, a, lmax, js = oracle.lambda_max(Xt, c, s, keep, rng.normal(size=77), mask)
    beta = rng.normal(size=40) * (rng.uniform(size=40) < 0.3)
    yt = yt.copy()
    yt[mask == 0] = 1e3          # rows outside the fit do not enter: r is 0 there
    r = oracle.residual(Xt, c, s, yt, beta, mask)
    Xtil, _, _ = std_numpy(Xt, mask)
    expect = np.zeros(77)
    expect[mask.astype(bool)] = yt[mask.astype(bool)] - Xtil @ beta
    np.testing.assert_allclose(r, expect, rtol=1e-12, atol=1e-12)
    assert np.all(r[mask == 0] == 0.0)


# ---------------------------------------------------------------------------------------------
# screening network: forward pass against numpy written from the definition
# (input f -> relu(W1 f + b1) -> relu(W2 h1 + b2) -> w3 . h2 + b3 -> logistic)
# ---------------------------------------------------------------------------------------------

def test_mlp_forward_matches_numpy_definition():
    H = 7
    rng = np.random.default_rng(17)
    params = rng.normal(scale=0.8, size=oracle.n_params(H))
    feat = rng.uniform(-1, 2, size=(40, 4))
    W1 = params[: 4 * H].reshape(H, 4)
    b1 = params[4 * H: 5 * H]
    W2 = params[5 * H: 5 * H + H * H].reshape(H, H)
    b2 = params[5 * H + H * H: 6 * H + H * H]
    w3 = params[6 * H + H * H: 7 * H + H * H]
    b3 = params[7 * H + H * H]
    h1 = np.maximum(feat @ W1.T + b1, 0.0)
    h2 = np.maximum(h1 @ W2.T + b2, 0.0)
    o = h2 @ w3 + b3
    expect = 1.0 / (1.0 + np.exp(-o))
    # the ReLUs cut something on this input (otherwise a missing ReLU would go unnoticed)
    assert (feat @ W1.T + b1 < 0).any() and (h1 @ W2.T + b2 < 0).any()
    np.testing.assert_allclose(oracle.mlp_forward(feat, params, H), expect, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------------------------------------
# BEDPP discard power: the closed form against the EDPP ball test written with explicit vectors
# (Wang, Wonka & Ye 2015, basic EDPP with the reference point at lambda_max, which the paper's
# Section 2.2 cites): with lambda' = n lambda, theta0 = y~ / (n lambda_max), v1 = sign(x~_*' y~) x~_*,
# v2 = y~ / lambda' - theta0, v2p = v2 - (v1.v2 / ||v1||^2) v1, feature j is discarded when
# |x~_j' (theta0 + v2p / 2)| < 1 - ||v2p|| ||x~_j|| / 2.
# ---------------------------------------------------------------------------------------------

def edpp_ball_discard(Xtil, yt, lam):
    n = Xtil.shape[0]
    corr = Xtil.T @ yt
    js = int(np.argmax(np.abs(corr)))
    lmp = np.abs(corr[js])                  # n lambda_max
    theta0 = yt / lmp
    v1 = np.sign(corr[js]) * Xtil[:, js]
    v2 = yt / (n * lam) - theta0
    v2p = v2 - (v1 @ v2) / (v1 @ v1) * v1
    lhs = np.abs(Xtil.T @ (theta0 + 0.5 * v2p))
    rhs = 1.0 - 0.5 * np.linalg.norm(v2p) * np.linalg.norm(Xtil, axis=0)
    return lhs < rhs, lhs - rhs


@pytest.mark.parametrize("seed,design", [(51, "gaussian"), (52, "genotype"), (53, "ar1")])
def test_bedpp_discards_exactly_the_edpp_ball_set(seed, design):
    n, p = 150, 600
    if design == "gaussian":
        Xt = datagen.gaussian_f64(seed, n, p)
    elif design == "genotype":
        Xt = datagen.genotype_u8(seed, n, p).astype(np.float64)
    else:
        Xt = datagen.ar1_f32(seed, n, p, 0.6).astype(np.float64)
    rng = np.random.default_rng(seed)
    y = Xt[rng.choice(p, 8, replace=False)].T @ rng.normal(size=8) + rng.normal(size=n)
    a, b, keep, lmax, sg, v = bedpp_inputs(Xt, y)
    Xtil, _, _ = std_numpy(Xt)
    yt = y - y.mean()
    total = 0
    for frac in np.geomspace(0.99, 0.2, 12):
        lam = frac * lmax
        d = oracle.bedpp_discard(a, b, keep, lmax, sg, v, lam)
        ball, margin = edpp_ball_discard(Xtil, yt, lam)
        undecided = np.abs(margin) < 1e-10          # within rounding of the boundary
        assert np.array_equal(d[~undecided], ball[~undecided]), f"lambda/lambda_max = {frac:.3f}"
        total += d.sum()
    assert total > 0


# ---------------------------------------------------------------------------------------------
# user lambda grids and cross-validation (Section 3.1.2: folds are row subsets of one X; Section 5.2:
# the cross-validation curve, lambda.min and the error there)
# ---------------------------------------------------------------------------------------------

def test_user_grid_equal_to_the_geometric_grid_gives_the_same_path():
    prob = datagen.make("c1", n=120, p=260)
    a = oracle.fit_path(prob.Xt, prob.y[0], K=20, ratio=0.05)
    b = oracle.fit_path(prob.Xt, prob.y[0], K=20, ratio=0.05, lambdas=a.lam)
    np.testing.assert_array_equal(a.beta, b.beta)
    np.testing.assert_array_equal(a.lam, b.lam)


def test_user_grid_above_and_below_lambda_max_brute_force():
    n, p = 40, 8
    rng = np.random.default_rng(61)
    Xt = rng.normal(size=(p, n)) + rng.normal(size=(p, 1))
    mask = np.ones(n, dtype=np.uint8)
    mask[rng.choice(n, 7, replace=False)] = 0
    y = 1.2 * Xt[1] - 0.8 * Xt[6] + rng.normal(size=n)
    c, s, keep, nn = oracle.standardize(Xt, mask)
    ybar, yt, a, lmax, js = oracle.lambda_max(Xt, c, s, keep, y, mask)
    lams = lmax * np.array([1.7, 1.0, 0.62, 0.31, 0.08])
    path = oracle.fit_path(Xt, y, K=5, mask=mask, lambdas=lams)
    Xtil, _, _ = std_numpy(Xt, mask)
    ym = y[mask.astype(bool)]
    assert np.all(path.beta[:2] == 0.0) and path.sweeps[0] == 0
    for k in (2, 3, 4):
        sols = brute_force_lasso(Xtil, ym - ym.mean(), lams[k])
        assert len(sols) == 1
        np.testing.assert_allclose(path.beta[k], sols[0], atol=1e-10)


def test_cv_summary_on_a_hand_worked_example():
    # rows of the loss matrix and what they give, worked by hand:
    #   k=0: 1, 1, 1, 1.8  -> mean 1.2, deviations -.2 -.2 -.2 .6, sample variance .48/3 = .16, SE .4/2 = .2
    #   k=1: 0, 2, 0, 2    -> mean 1.0, sample variance 4/3, SE sqrt(4/3)/2 = sqrt(1/3)
    #   k=2: 1.1 (x4)      -> mean 1.1, SE 0
    # smallest mean at k=1; 1.0 + sqrt(1/3) = 1.577 admits k=0 (1.2), the largest lambda
    loss = np.array([[1, 1, 1, 1.8], [0, 2, 0, 2], [1.1, 1.1, 1.1, 1.1]])
    cve, cvse, k_min, k_1se = oracle.cv_summary(loss)
    np.testing.assert_allclose(cve, [1.2, 1.0, 1.1], rtol=1e-15)
    np.testing.assert_allclose(cvse, [0.2, np.sqrt(1.0 / 3.0), 0.0], rtol=1e-14, atol=1e-15)
    assert k_min == 1 and k_1se == 0
    # ties: the first smallest
    cve, cvse, k_min, k_1se = oracle.cv_summary(np.array([[2.0, 2.0], [1.0, 1.0], [1.0, 1.0]]))
    assert k_min == 1 and k_1se == 1


def test_cv_single_feature_closed_form():
    """p = 1: every fold's coefficient is the soft threshold of its correlation (unit curvature), so the
    held-out predictions, their squared errors and the CV curve follow in closed form."""
    rng = np.random.default_rng(71)
    n = 53
    x = rng.normal(2.0, 1.5, size=n)
    y = 0.7 * x + rng.normal(size=n)
    fold = datagen.cv_folds(n, 5, 3)
    K, ratio = 9, 0.05
    cv = oracle.cv_path(x[None, :], y, fold, 5, K=K, ratio=ratio)
    # full-data grid
    xc = x - x.mean()
    lmax = abs(xc @ (y - y.mean())) / n / x.std()
    np.testing.assert_allclose(cv.lam, lmax * ratio ** (np.arange(K) / (K - 1)), rtol=1e-13)
    pred = np.zeros((K, n))
    for f in range(5):
        tr = fold != f
        xt, ytr = x[tr], y[tr]
        c, sd = xt.mean(), xt.std()
        a = ((xt - c) / sd) @ (ytr - ytr.mean()) / tr.sum()
        for k, lam in enumerate(cv.lam):
            slope = soft(a, lam) / sd
            pred[k, ~tr] = ytr.mean() + slope * (x[~tr] - c)
    np.testing.assert_allclose(cv.pred, pred, rtol=1e-11, atol=1e-11)
    loss = (y[None, :] - pred) ** 2
    np.testing.assert_allclose(cv.cve, loss.mean(axis=1), rtol=1e-11)


def test_cv_brute_force_folds():
    """p = 7: each fold's solution at every lambda of the full-data grid equals the unique sign pattern
    meeting the optimality conditions on the fold's training rows."""
    n, p = 48, 7
    rng = np.random.default_rng(81)
    Xt = datagen.genotype_u8(81, n, p).astype(np.float64)
    y = Xt[2] - 0.6 * Xt[5] + rng.normal(size=n)
    fold = datagen.cv_folds(n, 4, 9)
    cv = oracle.cv_path(Xt, y, fold, 4, K=6, ratio=0.05)
    for f in range(4):
        tr = (fold != f).astype(np.uint8)
        Xtil, c, s = std_numpy(Xt, tr)
        ym = y[tr.astype(bool)]
        for k in (2, 5):
            sols = brute_force_lasso(Xtil, ym - ym.mean(), cv.lam[k])
            assert len(sols) == 1
            np.testing.assert_allclose(cv.paths[f].beta[k], sols[0], atol=1e-10)
            b = sols[0] / s
            te = fold == f
            np.testing.assert_allclose(cv.pred[k, te], ym.mean() + (Xt[:, te].T - c) @ b, atol=1e-9)
    assert 0 <= cv.k_1se <= cv.k_min < 6


# ---------------------------------------------------------------------------------------------
# elastic net and penalty factors (Section 1: the package fits lasso and elastic-net penalties; the
# penalty of feature j is lambda w_j (alpha |beta_j| + (1 - alpha) beta_j^2 / 2))
# ---------------------------------------------------------------------------------------------

def enet_brute_force(Xtil, yt, lam, alpha, w):
    """Sign patterns again, with the ridge part on the diagonal and weighted thresholds."""
    n, p = Xtil.shape
    G = Xtil.T @ Xtil / n
    q = Xtil.T @ yt / n
    found = []
    for sig in itertools.product((-1, 0, 1), repeat=p):
        sig = np.array(sig)
        A = np.flatnonzero(sig)
        beta = np.zeros(p)
        if A.size:
            H = G[np.ix_(A, A)] + np.diag(lam * (1 - alpha) * w[A])
            beta[A] = np.linalg.solve(H, q[A] - lam * alpha * w[A] * sig[A])
            if not np.all(np.sign(beta[A]) == sig[A]):
                continue
        grad = q - G @ beta
        off = np.setdiff1d(np.arange(p), A)
        if np.all(np.abs(grad[off]) <= lam * alpha * w[off] * (1 + 1e-12)):
            found.append(beta)
    return found


def test_enet_unit_weights_and_alpha_one_is_the_lasso():
    prob = datagen.make("c1", n=150, p=320)
    a = oracle.fit_path(prob.Xt, prob.y[0], K=25, ratio=0.05)
    b = oracle.fit_path(prob.Xt, prob.y[0], K=25, ratio=0.05, alpha=1.0, penalty_factor=np.ones(320))
    np.testing.assert_array_equal(a.beta, b.beta)
    np.testing.assert_array_equal(a.lam, b.lam)


def test_enet_orthogonal_design_closed_form():
    n, p = 64, 10
    Xt = orthogonal_design(n, p, 91)
    rng = np.random.default_rng(92)
    y = Xt.T @ rng.normal(size=p) + rng.normal(size=n)
    w = rng.uniform(0.3, 2.0, size=p)
    alpha = 0.4
    path = oracle.fit_path(Xt, y, K=20, ratio=0.02, alpha=alpha, penalty_factor=w)
    Xtil, c, s = std_numpy(Xt)
    a = Xtil.T @ (y - y.mean()) / n
    assert path.lam[0] == pytest.approx(np.max(np.abs(a) / (alpha * w)), rel=1e-13)
    for k, lam in enumerate(path.lam):
        expect = soft(a, lam * alpha * w) / (1 + lam * (1 - alpha) * w)
        np.testing.assert_allclose(path.beta[k], expect, atol=1e-11)


@pytest.mark.parametrize("alpha,weighted", [(0.5, False), (0.8, True), (1.0, True)])
def test_enet_brute_force_with_row_mask(alpha, weighted):
    n, p = 42, 8
    rng = np.random.default_rng(101)
    Xt = rng.normal(size=(p, n)) + rng.normal(size=(p, 1))
    mask = np.ones(n, dtype=np.uint8)
    mask[rng.choice(n, 6, replace=False)] = 0
    y = Xt[0] - 1.5 * Xt[4] + 0.5 * Xt[6] + rng.normal(size=n)
    w = rng.uniform(0.5, 2.0, size=p) if weighted else np.ones(p)
    path = oracle.fit_path(Xt, y, K=10, ratio=0.03, mask=mask, alpha=alpha,
                           penalty_factor=w if weighted else None)
    Xtil, c, s = std_numpy(Xt, mask)
    ym = y[mask.astype(bool)]
    assert np.all(path.beta[0] == 0.0)
    for k in (2, 5, 9):
        sols = enet_brute_force(Xtil, ym - ym.mean(), path.lam[k], alpha, w)
        assert len(sols) == 1
        np.testing.assert_allclose(path.beta[k], sols[0], atol=1e-10)


def test_enet_weights_scale_with_lambda():
    """The penalty depends on lambda w_j only: weights times c with lambda over c is the same fit."""
    prob = datagen.make("c2", n=120, p=200)
    Xt = prob.Xt.astype(np.float64)
    w = np.random.default_rng(3).uniform(0.5, 1.5, size=200)
    a = oracle.fit_path(Xt, prob.y[0], K=12, ratio=0.1, alpha=0.7, penalty_factor=w)
    b = oracle.fit_path(Xt, prob.y[0], K=12, alpha=0.7, penalty_factor=4.0 * w, lambdas=a.lam / 4.0)
    np.testing.assert_allclose(b.beta, a.beta, atol=1e-11)


def test_enet_duality_gap_closed_form_at_beta_zero():
    """At beta = 0 the scaled residual is t y~ with t = lambda / lambda_max, so the gap is (1 - t)^2."""
    prob = datagen.make("c1", n=90, p=140)
    Xt = prob.Xt
    c, s, keep, n = oracle.standardize(Xt)
    ybar, yt, a, lmax_l, js = oracle.lambda_max(Xt, c, s, keep, prob.y[0])
    w = np.random.default_rng(4).uniform(0.5, 2.0, size=140)
    alpha = 0.6
    lmax = np.max(np.abs(a) / (alpha * w))
    for frac in (0.9, 0.5, 0.1):
        lam = frac * lmax
        gap = oracle.duality_gap(Xt, c, s, keep, yt, yt, np.zeros(140), lam, alpha=alpha, penalty_factor=w)
        assert gap == pytest.approx((1 - frac) ** 2, rel=1e-12)


def test_enet_path_certificates():
    prob = datagen.make("c4", n=200, p=400, nresp=1, nsub=1)
    Xt = prob.Xt.astype(np.float64)
    w = np.random.default_rng(5).uniform(0.25, 4.0, size=400)
    path = oracle.fit_path(Xt, prob.y[0], K=30, ratio=0.02, alpha=0.3, penalty_factor=w)
    assert path.k_done == 30
    assert np.max(path.gap[1:]) <= 1e-10
    # stationarity: z_j - lambda (1 - alpha) w_j beta_j = lambda alpha w_j sign(beta_j) on the support
    c, s, keep, n = path.c, path.s, path.keep, Xt.shape[1]
    yt = prob.y[0] - prob.y[0].mean()
    for k in (10, 29):
        b = path.beta[k]
        r = oracle.residual(Xt, c, s, yt, b)
        z = oracle.zscan(Xt, c, s, keep, r)
        lam = path.lam[k]
        act = b != 0
        np.testing.assert_allclose(z[act] - lam * 0.7 * w[act] * b[act], lam * 0.3 * w[act] * np.sign(b[act]),
                                   atol=1e-9 * lam)
        assert np.all(np.abs(z[~act]) <= lam * 0.3 * w[~act] * (1 + 1e-9))


# ---------------------------------------------------------------------------------------------
# lasso-penalized logistic regression (Section 1; Section 2.2's hybrid rule for it)
# ---------------------------------------------------------------------------------------------

def logistic_problem(seed, n, p, design="gaussian", nnz=4):
    rng = np.random.default_rng(seed)
    if design == "gaussian":
        Xt = rng.normal(size=(p, n))
    elif design == "genotype":
        Xt = datagen.genotype_u8(seed, n, p).astype(np.float64)
    else:
        Xt = datagen.ar1_f32(seed, n, p, 0.6).astype(np.float64)
    Xs = (Xt - Xt.mean(1, keepdims=True)) / Xt.std(1, keepdims=True)
    coef = np.zeros(p)
    coef[rng.choice(p, nnz, replace=False)] = rng.uniform(0.5, 1.5, nnz) * rng.choice([-1, 1], nnz)
    eta = Xs.T @ coef + 0.3
    y = (rng.uniform(size=n) < 1.0 / (1.0 + np.exp(-eta))).astype(np.float64)
    return Xt, y


def scipy_logistic_lasso(Xtil, y, lam):
    """An independent solve: L-BFGS-B on the smooth split beta = u - v, u, v >= 0 (library routine)."""
    from scipy.optimize import minimize
    n, p = Xtil.shape

    def f(v):
        b0, u, w = v[0], v[1:p + 1], v[p + 1:]
        eta = b0 + Xtil @ (u - w)
        pi = 1.0 / (1.0 + np.exp(-eta))
        loss = np.mean(np.logaddexp(0.0, eta) - y * eta) + lam * (u.sum() + w.sum())
        g = (pi - y) / n
        gb = Xtil.T @ g
        return loss, np.concatenate([[g.sum()], gb + lam, -gb + lam])

    x0 = np.zeros(2 * p + 1)
    bounds = [(None, None)] + [(0.0, None)] * (2 * p)
    r = minimize(f, x0, jac=True, method="L-BFGS-B", bounds=bounds,
                 options={"ftol": 1e-15, "gtol": 1e-12, "maxiter": 20000, "maxcor": 30})
    return r.x[0], r.x[1:p + 1] - r.x[p + 1:]


@pytest.mark.parametrize("design", ["gaussian", "genotype", "ar1"])
def test_logistic_path_matches_an_independent_solver(design):
    n, p = 120, 6
    Xt, y = logistic_problem(1, n, p, design)
    path = oracle.fit_path_logistic(Xt, y, K=12, ratio=0.05)
    assert path.status == 0 and path.k_done == 12
    Xtil, c, s = std_numpy(Xt)
    for k in (3, 7, 11):
        b0, b = scipy_logistic_lasso(Xtil, y, path.lam[k])
        np.testing.assert_allclose(path.beta[k], b, atol=2e-6)
        assert path.b0[k] == pytest.approx(b0, abs=2e-6)


def test_logistic_lambda_max_and_intercept_closed_form():
    Xt, y = logistic_problem(2, 150, 40)
    path = oracle.fit_path_logistic(Xt, y, K=10, ratio=0.1)
    Xtil, c, s = std_numpy(Xt)
    yb = y.mean()
    assert path.lam[0] == pytest.approx(np.max(np.abs(Xtil.T @ (y - yb))) / 150, rel=1e-13)
    assert np.all(path.beta[0] == 0.0) and path.sweeps[0] == 0
    assert path.b0[0] == pytest.approx(np.log(yb / (1 - yb)), rel=1e-14)


def test_logistic_single_feature_by_scalar_minimization():
    from scipy.optimize import minimize
    rng = np.random.default_rng(3)
    n = 90
    x = rng.normal(1.0, 2.0, size=n)
    y = (rng.uniform(size=n) < 1 / (1 + np.exp(-(0.8 * (x - 1) / 2 - 0.2)))).astype(float)
    path = oracle.fit_path_logistic(x[None, :], y, K=8, ratio=0.05)
    xt = (x - x.mean()) / x.std()
    for k in range(1, 8):
        lam = path.lam[k]
        obj = lambda v: np.mean(np.logaddexp(0, v[0] + v[1] * xt) - y * (v[0] + v[1] * xt)) + lam * abs(v[1])
        r = minimize(obj, [0.0, 0.1], method="Nelder-Mead", options={"xatol": 1e-11, "fatol": 1e-15,
                                                                     "maxiter": 20000})
        assert path.beta[k][0] == pytest.approx(r.x[1], abs=1e-6)


@pytest.mark.parametrize("design", ["gaussian", "genotype", "ar1"])
def test_logistic_kkt_and_gap_along_the_path(design):
    Xt, y = logistic_problem(4, 300, 500, design, nnz=15)
    mask = (np.random.default_rng(5).uniform(size=300) < 0.9).astype(np.uint8)
    path = oracle.fit_path_logistic(Xt, y, K=30, ratio=0.03, mask=mask)
    assert path.k_done == 30
    assert np.max(path.gap) <= 1e-10
    rows = mask.astype(bool)
    for k in (10, 29):
        c, s = path.c, path.s
        Xtil = ((Xt[:, rows].T - c) / s)
        eta = path.b0[k] + Xtil @ path.beta[k]
        pi = 1 / (1 + np.exp(-eta))
        z = Xtil.T @ (y[rows] - pi) / rows.sum()
        b = path.beta[k]
        lam = path.lam[k]
        assert abs(np.sum(y[rows] - pi)) <= 1e-8 * rows.sum()
        np.testing.assert_allclose(z[b != 0], lam * np.sign(b[b != 0]), atol=1e-8 * lam)
        assert np.all(np.abs(z[b == 0]) <= lam * (1 + 1e-8))


@pytest.mark.parametrize("seed,design", [(6, "gaussian"), (7, "genotype"), (8, "ar1")])
def test_logistic_safe_rule_is_safe(seed, design):
    Xt, y = logistic_problem(seed, 250, 400, design, nnz=10)
    path = oracle.fit_path_logistic(Xt, y, K=40, ratio=0.02, screen=oracle.SCREEN_NONE)
    c, s, keep, n = oracle.standardize(Xt)
    a = oracle.zscan(Xt, c, s, keep, y - y.mean())
    n1 = int(y.sum())
    discarded_total = 0
    for k, lam in enumerate(path.lam):
        thr = oracle.logistic_safe_threshold(250, n1, path.lam[0], lam)
        disc = np.abs(a) < thr
        discarded_total += disc.sum()
        assert np.all(path.beta[k][disc] == 0.0), k
        assert path.n_safe[k] == 400 - disc.sum()
    assert discarded_total > 0
    # at lambda_max the gap is 0 and the test is |a_j| < lambda_max
    assert oracle.logistic_safe_threshold(250, n1, path.lam[0], path.lam[0]) == pytest.approx(path.lam[0], rel=1e-14)
