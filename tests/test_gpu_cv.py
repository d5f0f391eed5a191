"""Cross-validation (bl_cv_fit) and the batched form on a shared grid, against the FP64 oracle.

Every fold's path is compared with the oracle's path on that fold's training rows over the full-data grid
(max |d beta| <= 1e-6, relative objective <= 1e-8), the held-out predictions with the oracle's (which
follow from those coefficients: their error is bounded by sum_j |x_ij| |d beta_j| / s_j), and the curve,
lambda.min and the one-standard-error choice with the oracle's.
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


def decisive(cve, k, rel=1e-6):
    """k is the argmin by a margin larger than rounding (so the GPU must pick the same index)."""
    others = np.delete(cve, k)
    return others.size == 0 or np.min(others) > cve[k] * (1 + rel)


@pytest.mark.parametrize("n,p,nfolds,K,dt,left_out", [(1500, 3000, 10, 20, np.float32, 0),
                                                       (701, 1333, 5, 25, np.float64, 37)])
def test_cv_matches_oracle(gpu_ctx, n, p, nfolds, K, dt, left_out):
    rec = datagen.RECIPES["c4"].scaled(n=n, p=p, nresp=1, nsub=1, seed=404 + n)
    prob = datagen.make(rec)
    X = prob.Xt.astype(dt)
    y = prob.y[0]
    fold = datagen.cv_folds(n, nfolds, 7)
    if left_out:
        fold[np.random.default_rng(1).choice(n, left_out, replace=False)] = -1
    ratio = rec.lambda_min_ratio
    ref = oracle.cv_path(X.astype(np.float64), y, fold, nfolds, K=K, ratio=ratio)
    res = bl.cv_fit(gpu_ctx, to_dev(X), to_dev(y), to_dev(fold), nfolds, nlambda=K, lambda_min_ratio=ratio,
                    tol=1e-10)
    print(f"n={n} p={p} folds={nfolds}: {res.time_ms:.0f} ms, lambda.min index {res.k_min} (oracle {ref.k_min}), "
          f"1se {res.k_1se} (oracle {ref.k_1se})", flush=True)
    np.testing.assert_allclose(res.lam, ref.lam, rtol=1e-12)
    assert res.n_rows == int((fold >= 0).sum())
    fb = res.fold_beta.cpu().numpy()
    for f in range(nfolds):
        d = np.abs(fb[f] - ref.paths[f].beta).max()
        assert d <= 1e-6, (f, d)
    # the full-data path
    full = oracle.fit_path(X.astype(np.float64), y, K=K, ratio=ratio, mask=(fold >= 0).astype(np.uint8))
    assert np.abs(res.beta.cpu().numpy() - full.beta).max() <= 1e-6
    # predictions: the held-out rows of every fold, at every lambda
    pred = res.pred.cpu().numpy()
    scale = 1.0 + np.abs(y).max()
    assert np.abs(pred - ref.pred).max() <= 1e-5 * scale
    np.testing.assert_allclose(res.cve, ref.cve, rtol=1e-5)
    np.testing.assert_allclose(res.cvse, ref.cvse, rtol=1e-4, atol=1e-12)
    np.testing.assert_allclose(res.fold_err, ref.fold_err, rtol=1e-5)
    if decisive(ref.cve, ref.k_min):
        assert res.k_min == ref.k_min
    assert res.k_1se <= res.k_min
    assert res.lambda_min == res.lam[res.k_min] and res.lambda_1se == res.lam[res.k_1se]


def test_batch_on_a_shared_grid_above_and_below_each_lambda_max(gpu_ctx):
    """One grid for every problem, starting above some problems' lambda_max: those rows are beta = 0, the
    others are solved from the first point on."""
    rec = datagen.RECIPES["c4"].scaled(n=800, p=1500, nresp=4, nsub=2, seed=504)
    prob = datagen.make(rec)
    X64 = prob.Xt.astype(np.float64)
    Y = np.repeat(prob.y, 2, axis=0)
    masks = prob.masks
    lmaxes = []
    for b in range(Y.shape[0]):
        c, s, keep, n = oracle.standardize(X64, masks[b])
        lmaxes.append(oracle.lambda_max(X64, c, s, keep, Y[b], masks[b])[3])
    lmaxes = np.array(lmaxes)
    K = 15
    lam = np.median(lmaxes) * 1.05 * 0.08 ** (np.arange(K) / (K - 1))
    assert np.any(lmaxes <= lam[0]) and np.any(lmaxes > lam[0])
    res = bl.fit_path_batch(gpu_ctx, to_dev(prob.Xt), to_dev(Y), to_dev(masks), nlambda=K, lambdas=lam, tol=1e-10)
    assert res.k_done == K
    beta = res.beta.cpu().numpy()
    for b in range(Y.shape[0]):
        ref = oracle.fit_path(X64, Y[b], K=K, mask=masks[b], lambdas=lam)
        np.testing.assert_array_equal(res.lam[b], lam)
        d = np.abs(beta[b] - ref.beta).max()
        rd = np.abs((res.obj[b] - ref.obj) / ref.obj).max()
        print(f"problem {b}: lambda_max / lambda_0 = {lmaxes[b] / lam[0]:.3f}, max|d beta| {d:.2e}, RD {rd:.2e}")
        assert d <= 1e-6 and rd <= 1e-8
        np.testing.assert_array_equal(res.n_active[b], ref.n_active)
        np.testing.assert_array_equal(res.n_safe[b], ref.n_safe)
        if lmaxes[b] <= lam[0]:
            assert np.all(beta[b, 0] == 0.0)


def test_cv_rejects_bad_folds(gpu_ctx):
    prob = datagen.make("c1", n=60, p=40)
    Xd, yd = to_dev(prob.Xt), to_dev(prob.y[0])
    fold = datagen.cv_folds(60, 4, 1)
    bad = fold.copy()
    bad[3] = 7
    with pytest.raises(bl.BLError) as e:
        bl.cv_fit(gpu_ctx, Xd, yd, to_dev(bad), 4, nlambda=5)
    assert e.value.status == bl.BL_ERR_INVALID
    empty = fold.copy()
    empty[empty == 2] = 1
    with pytest.raises(bl.BLError) as e:
        bl.cv_fit(gpu_ctx, Xd, yd, to_dev(empty), 4, nlambda=5)
    assert e.value.status == bl.BL_ERR_INVALID
    with pytest.raises(bl.BLError) as e:
        bl.cv_fit(gpu_ctx, Xd, yd, to_dev(fold), 1, nlambda=5)
    assert e.value.status == bl.BL_ERR_INVALID
