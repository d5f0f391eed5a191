"""Lasso-penalized logistic regression (family BL_FAMILY_BINOMIAL) against the FP64 oracle.

The oracle solves each lambda by IRLS with coordinate descent; the GPU by majorization with the lasso
coordinate descent on its Gram pool.  Both reach the unique solution, so coefficients agree to the
stopping tolerances (max |d beta| <= 1e-6, relative objective <= 1e-8), with equal active-set sizes and
equal safe-rule survivor counts.
"""
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


def binary_response(Xt, seed, nnz=10):
    rng = np.random.default_rng(seed)
    p, n = Xt.shape
    Xs = (Xt - Xt.mean(1, keepdims=True)) / Xt.std(1, keepdims=True)
    coef = np.zeros(p)
    idx = rng.choice(p, nnz, replace=False)
    coef[idx] = rng.uniform(0.4, 1.2, nnz) * rng.choice([-1, 1], nnz)
    eta = Xs.T @ coef - 0.4
    return (rng.uniform(size=n) < 1 / (1 + np.exp(-eta))).astype(np.float64)


CASES = {
    # name: (recipe, n, p, dtype, masked, rule)
    "gauss_f64_hybrid": ("c1", 500, 1500, np.float64, False, bl.SCREEN_SSR_BEDPP),
    "geno_f64_masked_hybrid": ("c2", 600, 2000, np.float64, True, bl.SCREEN_SSR_BEDPP),
    "ar1_f32_ssr": ("c4", 450, 1200, np.float32, False, bl.SCREEN_SSR),
    "gauss_f64_active": ("c1", 300, 700, np.float64, True, bl.SCREEN_ACTIVE),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_logistic_path_matches_oracle(gpu_ctx, name):
    rec, n, p, dt, masked, rule = CASES[name]
    prob = datagen.make(rec, n=n, p=p, nresp=1, nsub=1) if rec == "c4" else datagen.make(rec, n=n, p=p)
    Xh = prob.Xt.astype(dt)
    X64 = Xh.astype(np.float64)
    y = binary_response(X64, n + p)
    mask = (np.random.default_rng(p).uniform(size=n) < 0.85).astype(np.uint8) if masked else None
    K, ratio = 30, 0.05
    screen = {bl.SCREEN_SSR_BEDPP: oracle.SCREEN_SSR, bl.SCREEN_SSR: oracle.SCREEN_SSR,
              bl.SCREEN_ACTIVE: oracle.SCREEN_ACTIVE}[rule]
    ref = oracle.fit_path_logistic(X64, y, K=K, ratio=ratio, tol=1e-12, mask=mask, screen=screen)
    assert ref.k_done == K
    res = bl.fit_path(gpu_ctx, to_dev(Xh), to_dev(y), nlambda=K, lambda_min_ratio=ratio, rule=rule, tol=1e-11,
                      row_mask=to_dev(mask) if masked else None, family=bl.FAMILY_BINOMIAL)
    assert res.k_done == K
    np.testing.assert_allclose(res.lam, ref.lam, rtol=1e-12)
    d = np.abs(res.beta.cpu().numpy() - ref.beta).max()
    rd = np.abs((res.obj - ref.obj) / ref.obj).max()
    print(f"{name}: max|d beta| {d:.2e}, max RD {rd:.2e}, active at the end {res.n_active[-1]}, violations "
          f"{res.n_viol.sum()}, sweeps {res.sweeps.sum()}, {res.time_ms:.0f} ms", flush=True)
    assert d <= 1e-6
    assert rd <= 1e-8
    np.testing.assert_array_equal(res.n_active, ref.n_active)
    icpt, _ = ref.original_scale()
    np.testing.assert_allclose(res.intercept, icpt, atol=1e-6)
    if rule == bl.SCREEN_SSR_BEDPP:
        np.testing.assert_array_equal(res.n_safe, ref.n_safe)
        assert res.n_safe[1] < p   # the safe rule discards at the top of the path
    if rule == bl.SCREEN_ACTIVE:
        assert res.n_viol.sum() > 0 and res.rounds.max() >= 2


def test_logistic_host_path_equals_device_path(gpu_ctx):
    prob = datagen.make("c2", n=700, p=6000)
    X64 = prob.Xt.astype(np.float64)
    y = to_dev(binary_response(X64, 5))
    kw = dict(nlambda=25, lambda_min_ratio=0.05, tol=1e-10, family=bl.FAMILY_BINOMIAL)
    dev = bl.fit_path(gpu_ctx, to_dev(X64), y, **kw)
    host, st = bl.fit_path_host(gpu_ctx, torch.from_numpy(X64).pin_memory(), y, panel_cols=700, **kw)
    assert torch.equal(host.beta, dev.beta)
    np.testing.assert_array_equal(host.obj, dev.obj)


def test_logistic_rejects_bad_responses(gpu_ctx):
    prob = datagen.make("c1", n=80, p=50)
    Xd = to_dev(prob.Xt)
    y = binary_response(prob.Xt, 1)
    bad = y.copy()
    bad[4] = 2.0
    with pytest.raises(bl.BLError) as e:
        bl.fit_path(gpu_ctx, Xd, to_dev(bad), nlambda=5, family=bl.FAMILY_BINOMIAL)
    assert e.value.status == bl.BL_ERR_INVALID
    with pytest.raises(bl.BLError) as e:
        bl.fit_path(gpu_ctx, Xd, to_dev(np.ones(80)), nlambda=5, family=bl.FAMILY_BINOMIAL)
    assert e.value.status == bl.BL_ERR_INVALID
    with pytest.raises(bl.BLError) as e:
        bl.fit_path(gpu_ctx, Xd, to_dev(y), nlambda=5, family=bl.FAMILY_BINOMIAL, alpha=0.5)
    assert e.value.status == bl.BL_ERR_UNSUPPORTED
