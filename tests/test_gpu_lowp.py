"""Precision forms: int8 genotype codes on BF16 or on int8 matrix cores.

Each matrix-core scan must stay within the error bound it reports for every
column, and whole paths must meet the FP64 accuracy target with the same active
sets as the FP64 path (decisions near a threshold are re-taken in FP64).
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


FORMS = [pytest.param(bl.PREC_BF16X3, id="bf16x3"), pytest.param(bl.PREC_I8X4, id="i8x4")]


@pytest.mark.parametrize("prec", FORMS)
@pytest.mark.parametrize("n,ld,p,masked", [(2000, 2000, 3000, False), (1990, 2000, 1237, False),
                                            (1500, 1504, 2100, True), (130, 144, 70, False)])
def test_matrix_core_scan_within_its_bound(gpu_ctx, n, ld, p, masked, prec):
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
                     precision=prec, row_mask=to_dev(mask) if masked else None, n_total=n, want_err=True)
    z, err = z.cpu().numpy()[cols], err.cpu().numpy()[cols]
    dev = np.abs(z - z_exact[cols])
    ratio = np.max(dev / err)
    print(f"n={n} p={p}: max |z~ - z| = {dev.max():.3e}, max bound = {err.max():.3e}, max ratio {ratio:.3f}")
    assert ratio <= 1.0
    # the bound is tight enough to be useful: far below the spread of z (int8 pieces: 4 x 7 bits of max|r|)
    assert np.max(err) < (1e-4 if prec == bl.PREC_BF16X3 else 1e-6) * np.max(np.abs(z_exact))
    zf = bl.scan(gpu_ctx, to_dev(padded_codes(Xt, ld)), to_dev(c), to_dev(s), to_dev(r), to_dev(cols),
                 precision=bl.PREC_FP64, row_mask=to_dev(mask) if masked else None, n_total=n).cpu().numpy()
    np.testing.assert_allclose(zf[cols], z_exact[cols], atol=1e-12 * np.abs(z_exact).max())


@pytest.mark.parametrize("prec", FORMS)
def test_matrix_core_scan_rejects_what_it_cannot_do(gpu_ctx, prec):
    Xt = datagen.genotype_u8(1, 64, 20)
    c, s, keep, n = oracle.standardize(Xt.astype(np.float64))
    cols = torch.arange(20, dtype=torch.int32, device=DEV)
    r = to_dev(np.ones(64))
    with pytest.raises(bl.BLError) as e:
        bl.scan(gpu_ctx, to_dev(Xt.astype(np.float64)), to_dev(c), to_dev(s), r, cols, precision=prec)
    assert e.value.status == bl.BL_ERR_UNSUPPORTED
    with pytest.raises(bl.BLError) as e:   # leading dimension not a multiple of 16
        bl.scan(gpu_ctx, to_dev(padded_codes(Xt.astype(np.int8), 70)), to_dev(c), to_dev(s), r, cols,
                precision=prec, n_total=64)
    assert e.value.status == bl.BL_ERR_UNSUPPORTED
    with pytest.raises(bl.BLError) as e:
        bl.scan(gpu_ctx, to_dev(Xt.astype(np.int8)), to_dev(c), to_dev(s), r, cols, precision=7)
    assert e.value.status == bl.BL_ERR_INVALID


@pytest.mark.parametrize("n,p", [(70001, 40), (140001, 9)])
def test_i8_scan_full_code_range_past_one_int32_chunk(gpu_ctx, n, p):
    """Codes over the whole int8 range and more rows than one int32 sum holds (65,536).  Column 0 is
    -128 on all rows but one and 95% of the residual sits at 127 = 127 s_1 (s_1 = 1), so its first-piece
    sum reaches -128 * 127 * 133,000 < -2^31 over 140,001 rows: exact only with the per-chunk flush."""
    rng = np.random.default_rng(n + p)
    Xt = rng.integers(-128, 128, size=(p, n), dtype=np.int64).astype(np.int8)
    Xt[0, :] = -128
    Xt[0, -1] = 127
    Xt[1, :] = np.where(np.arange(n) % 2 == 0, 127, -128)
    X64 = Xt.astype(np.float64)
    c, s, keep, nn = oracle.standardize(X64)
    assert keep.all()
    r = rng.normal(size=n)
    r[: int(0.95 * n)] = 127.0
    z_exact = oracle.zscan(X64, c, s, keep, r)
    cols = np.flatnonzero(keep).astype(np.int32)
    z, err = bl.scan(gpu_ctx, to_dev(padded_codes(Xt, (n + 15) // 16 * 16)), to_dev(c), to_dev(s), to_dev(r),
                     to_dev(cols), precision=bl.PREC_I8X4, n_total=n, want_err=True)
    z, err = z.cpu().numpy()[cols], err.cpu().numpy()[cols]
    dev = np.abs(z - z_exact[cols])
    print(f"n={n}: max |z~ - z| = {dev.max():.3e}, max bound = {err.max():.3e}")
    assert np.all(dev <= err)
    # columns 0 and 1 have |c_j| >> s_j, which widens their bound by ||x_j||_2 / (sqrt(n) s_j); the rest are tight
    assert np.max(err[2:]) < 1e-6 * np.max(np.abs(z_exact))


def test_i8_scan_of_a_zero_residual_is_zero(gpu_ctx):
    Xt = datagen.genotype_u8(5, 300, 50).astype(np.int8)
    c, s, keep, n = oracle.standardize(Xt.astype(np.float64))
    cols = np.flatnonzero(keep).astype(np.int32)
    z, err = bl.scan(gpu_ctx, to_dev(padded_codes(Xt, 304)), to_dev(c), to_dev(s), to_dev(np.zeros(300)),
                     to_dev(cols), precision=bl.PREC_I8X4, n_total=300, want_err=True)
    assert torch.count_nonzero(z).item() == 0
    assert torch.count_nonzero(err).item() == 0


@pytest.mark.parametrize("prec", FORMS)
@pytest.mark.parametrize("n,p,masked", [(1600, 4000, False), (1211, 2500, True)])
def test_precision_path_matches_oracle_with_fp64_active_sets(gpu_ctx, n, p, masked, prec):
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
    lp = bl.fit_path(gpu_ctx, Xd, to_dev(prob.y[0]), precision=prec, **kw)
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
