"""Elastic net and penalty factors (Section 1: the package fits lasso and elastic-net penalties) against
the FP64 oracle: whole paths to the same bar as the lasso (max |d beta| <= 1e-6, relative objective <=
1e-8, equal active-set sizes), through each coordinate-descent form: the multi-workgroup covariance solve
(one threshold, alpha < 1 without weights), the single-workgroup covariance solve (per-coordinate
thresholds), and the residual form (reached by lowering the covariance limit)."""
import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_1701_05936_amd as bl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def check_path(res, ref, K):
    assert res.k_done == K
    np.testing.assert_allclose(res.lam, ref.lam, rtol=1e-12)
    d = np.abs(res.beta.cpu().numpy() - ref.beta).max()
    rd = np.abs((res.obj - ref.obj) / ref.obj).max()
    print(f"max|d beta| {d:.2e}, max RD {rd:.2e}, largest working set {res.n_strong.max()}, "
          f"active at the end {res.n_active[-1]}", flush=True)
    assert d <= 1e-6
    assert rd <= 1e-8
    np.testing.assert_array_equal(res.n_active, ref.n_active)
    np.testing.assert_array_equal(res.n_safe, ref.n_safe)


CASES = {
    # name: (recipe, n, p, storage, masked, alpha, weighted)
    "gauss_alpha05": ("c1", 900, 2600, np.float64, False, 0.5, False),
    "geno_alpha07_weighted_masked": ("c2", 700, 1800, np.float64, True, 0.7, True),
    "ar1_f32_alpha1_weighted": ("c4", 600, 1500, np.float32, False, 1.0, True),
    "ar1_f32_alpha02_masked": ("c4", 650, 1400, np.float32, True, 0.2, False),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_enet_path_matches_oracle(gpu_ctx, name):
    rec, n, p, dt, masked, alpha, weighted = CASES[name]
    prob = datagen.make(rec, n=n, p=p, nresp=1, nsub=1) if rec == "c4" else datagen.make(rec, n=n, p=p)
    Xh = prob.Xt.astype(dt)
    y = prob.y[0]
    rng = np.random.default_rng(n + p)
    mask = (rng.uniform(size=n) < 0.85).astype(np.uint8) if masked else None
    w = rng.uniform(0.3, 3.0, size=p) if weighted else None
    K, ratio = 40, 0.01
    ref = oracle.fit_path(Xh.astype(np.float64), y, K=K, ratio=ratio, tol=1e-13, mask=mask, alpha=alpha,
                          penalty_factor=w)
    print(f"{name}:", flush=True)
    res = bl.fit_path(gpu_ctx, to_dev(Xh), to_dev(y), nlambda=K, lambda_min_ratio=ratio, tol=1e-10,
                      row_mask=to_dev(mask) if masked else None, alpha=alpha,
                      penalty_factor=to_dev(w) if weighted else None)
    check_path(res, ref, K)
    assert res.lambda_max == pytest.approx(ref.lam[0], rel=1e-12)


@pytest.mark.parametrize("weighted", [False, True])
def test_enet_residual_form_matches_oracle(weighted):
    n, p = 700, 1200
    prob = datagen.make("c1", n=n, p=p)
    w = np.random.default_rng(8).uniform(0.5, 2.0, size=p) if weighted else None
    K, ratio = 25, 0.02
    ref = oracle.fit_path(prob.Xt, prob.y[0], K=K, ratio=ratio, tol=1e-13, alpha=0.6, penalty_factor=w)
    with bl.Context(0) as ctx:
        ctx.set_limits(cov_max=16)
        res = bl.fit_path(ctx, to_dev(prob.Xt), to_dev(prob.y[0]), nlambda=K, lambda_min_ratio=ratio, tol=1e-10,
                          alpha=0.6, penalty_factor=to_dev(w) if weighted else None)
    check_path(res, ref, K)


def test_enet_with_the_active_set_rule_is_repaired(gpu_ctx):
    prob = datagen.make("c1", n=300, p=800)
    w = np.random.default_rng(9).uniform(0.5, 2.0, size=800)
    K, ratio = 25, 0.05
    ref = oracle.fit_path(prob.Xt, prob.y[0], K=K, ratio=ratio, tol=1e-13, alpha=0.5, penalty_factor=w,
                          screen=oracle.SCREEN_ACTIVE)
    res = bl.fit_path(gpu_ctx, to_dev(prob.Xt), to_dev(prob.y[0]), nlambda=K, lambda_min_ratio=ratio, tol=1e-10,
                      alpha=0.5, penalty_factor=to_dev(w), rule=bl.SCREEN_ACTIVE)
    check_path(res, ref, K)
    assert res.n_viol.sum() > 0 and res.rounds.max() >= 2


def test_enet_rejects_what_it_cannot_do(gpu_ctx):
    prob = datagen.make("c2", n=128, p=300)
    X8 = to_dev(prob.Xt.astype(np.int8))
    y = to_dev(prob.y[0])
    with pytest.raises(bl.BLError) as e:
        bl.fit_path(gpu_ctx, X8, y, nlambda=10, alpha=0.5, precision=bl.PREC_I8X4)
    assert e.value.status == bl.BL_ERR_UNSUPPORTED
    w = np.ones(300)
    w[7] = 0.0
    with pytest.raises(bl.BLError) as e:
        bl.fit_path(gpu_ctx, X8, y, nlambda=10, penalty_factor=to_dev(w))
    assert e.value.status == bl.BL_ERR_INVALID
    with pytest.raises(bl.BLError) as e:
        bl.fit_path(gpu_ctx, X8, y, nlambda=10, alpha=1.5)
    assert e.value.status == bl.BL_ERR_INVALID
