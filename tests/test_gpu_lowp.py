"""Precision form: int8 genotype codes on BF16 matrix cores.

The BF16 scan must stay within the error bound it reports for every column,
and whole paths must meet the FP64 accuracy target with the same active sets
as the FP64 path (decisions near a threshold are re-taken in FP64).
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


def padded_codes(Xt, ld):
    p, n = Xt.shape
    out = np.full((p, ld), 2, dtype=np.int8)   # padding rows hold codes that must not be read as data
    out[:, :n] = Xt
    return out


@pytest.mark.parametrize("n,ld,p,masked", [(2000, 2000, 3000, False), (1990, 2000, 1237, False),
                                            (1500, 1504, 2100, True), (130, 144, 70, False)])
def test_bf16_scan_within_its_bound(gpu_ctx, n, ld, p, masked):
    Xt = datagen.genotype_u8(42 + n, n, p).astype(np.int8)
    X64 = Xt.astype(np.float64)
    rng = np.random.default_rng(n)
    mask = (rng.uniform(size=n) < 0.85).astype(np.uint8) if masked else None
    c, s, keep, nn = oracle.standardize(X64, mask)
    r = rng.normal(size=n) * 3 + 0.1
    r[rng.uniform(size=n) < 0.05] *= 1e-6          # tiny residuals exercise the piece split
    if mask is not None:
        r[mask == 0] = 0.0
    z_exact = oracle.zscan(X64, c, s, keep, r, mask)
    cols = np.flatnonzero(keep).astype(np.int32)
    z, err = bl.scan(gpu_ctx, to_dev(padded_codes(Xt, ld)), to_dev(c), to_dev(s), to_dev(r), to_dev(cols),
                     precision=bl.PREC_BF16X3, row_mask=to_dev(mask) if masked else None, n_total=n, want_err=True)
    z, err = z.cpu().numpy()[cols], err.cpu().numpy()[cols]
    dev = np.abs(z - z_exact[cols])
    ratio = np.max(dev / err)
    print(f"n={n} p={p}: max |z~ - z| = {dev.max():.3e}, max bound = {err.max():.3e}, max ratio {ratio:.3f}")
    assert ratio <= 1.0
    # the bound is tight enough to be useful: far below the spread of z
    assert np.max(err) < 1e-4 * np.max(np.abs(z_exact))
    zf = bl.scan(gpu_ctx, to_dev(padded_codes(Xt, ld)), to_dev(c), to_dev(s), to_dev(r), to_dev(cols),
                 precision=bl.PREC_FP64, row_mask=to_dev(mask) if masked else None, n_total=n).cpu().numpy()
    np.testing.assert_allclose(zf[cols], z_exact[cols], atol=1e-12 * np.abs(z_exact).max())


def test_bf16_scan_rejects_what_it_cannot_do(gpu_ctx):
    Xt = datagen.genotype_u8(1, 64, 20)
    c, s, keep, n = oracle.standardize(Xt.astype(np.float64))
    cols = torch.arange(20, dtype=torch.int32, device=DEV)
    r = to_dev(np.ones(64))
    with pytest.raises(bl.BLError) as e:
        bl.scan(gpu_ctx, to_dev(Xt.astype(np.float64)), to_dev(c), to_dev(s), r, cols, precision=bl.PREC_BF16X3)
    assert e.value.status == bl.BL_ERR_UNSUPPORTED
    with pytest.raises(bl.BLError) as e:   # leading dimension not a multiple of 16
        bl.scan(gpu_ctx, to_dev(padded_codes(Xt.astype(np.int8), 70)), to_dev(c), to_dev(s), r, cols,
                precision=bl.PREC_BF16X3, n_total=64)
    assert e.value.status == bl.BL_ERR_UNSUPPORTED


@pytest.mark.parametrize("n,p,masked", [(1600, 4000, False), (1211, 2500, True)])
def test_precision_path_matches_oracle_with_fp64_active_sets(gpu_ctx, n, p, masked):
    rec = datagen.RECIPES["c3"].scaled(n=n, p=p)
    prob = datagen.make(rec)
    Xt = prob.Xt.astype(np.int8)
    ld = (n + 15) // 16 * 16
    mask = (np.random.default_rng(p).uniform(size=n) < 0.9).astype(np.uint8) if masked else None
    K, ratio = 40, rec.lambda_min_ratio
    ref = oracle.fit_path(Xt.astype(np.float64), prob.y[0], K=K, ratio=ratio, tol=1e-13, mask=mask)
    Xd = to_dev(padded_codes(Xt, ld))
    kw = dict(nlambda=K, lambda_min_ratio=ratio, tol=1e-10, n_total=n,
              row_mask=to_dev(mask) if masked else None)
    lp = bl.fit_path(gpu_ctx, Xd, to_dev(prob.y[0]), precision=bl.PREC_BF16X3, **kw)
    hp = bl.fit_path(gpu_ctx, Xd, to_dev(prob.y[0]), precision=bl.PREC_FP64, **kw)
    assert lp.k_done == K
    bl_ = lp.beta.cpu().numpy()
    assert np.abs(bl_ - ref.beta).max() <= 1e-6
    assert np.abs((lp.obj - ref.obj) / ref.obj).max() <= 1e-8
    # every screening and check decision equals the FP64 path's, and the solves start from the same
    # exact gradients, so the coefficients are the FP64 path's bit for bit (same active sets a fortiori)
    assert torch.equal(lp.beta, hp.beta)
    np.testing.assert_array_equal(lp.n_strong, hp.n_strong)
    np.testing.assert_array_equal(lp.n_active, ref.n_active)
    assert lp.n_recheck.sum() > 0
