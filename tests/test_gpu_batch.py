"""Batched form: many problems (responses x cross-validation row subsets) over one X.

Every problem's path is compared with the FP64 oracle run on that problem alone
(its response, its row mask), to the same bar as the plain path: max |d beta|
<= 1e-6 and relative objective difference <= 1e-8 on the problem's own
standardized scale, equal active-set sizes and BEDPP survivor counts.
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


def check_against_oracle(res, X64, Y, masks, K, ratio, problems, check_safe=True):
    assert res.k_done == K
    beta = res.beta.cpu().numpy()
    for b in problems:
        ref = oracle.fit_path(X64, Y[b], K=K, ratio=ratio, tol=1e-13, mask=None if masks is None else masks[b])
        assert ref.k_done == K
        np.testing.assert_allclose(res.lam[b], ref.lam, rtol=1e-12)
        d = np.abs(beta[b] - ref.beta).max()
        rd = np.abs((res.obj[b] - ref.obj) / ref.obj).max()
        print(f"problem {b}: max|d beta| {d:.2e}, max RD {rd:.2e}, active at end {ref.n_active[-1]}")
        assert d <= 1e-6, b
        assert rd <= 1e-8, b
        np.testing.assert_array_equal(res.n_active[b], ref.n_active)
        icpt, _ = ref.original_scale()
        np.testing.assert_allclose(res.intercept[b], icpt, atol=1e-6 * max(1.0, abs(ref.ybar)))
        if check_safe:
            np.testing.assert_array_equal(res.n_safe[b], ref.n_safe)


def cv_problem(n, p, nresp, nsub, seed_shift=0):
    rec = datagen.RECIPES["c4"].scaled(n=n, p=p, nresp=nresp, nsub=nsub, seed=104 + seed_shift)
    prob = datagen.make(rec)
    X32 = prob.Xt                     # (p, n) float32
    Y = np.repeat(prob.y, nsub, axis=0)   # problem b = t * nsub + s uses response t
    masks = prob.masks
    return rec, X32, Y, masks


@pytest.mark.parametrize("n,p,nresp,nsub,K", [(1500, 4000, 8, 2, 20), (643, 1111, 32, 2, 12)])
def test_batch_matches_oracle_per_problem(gpu_ctx, n, p, nresp, nsub, K):
    rec, X32, Y, masks = cv_problem(n, p, nresp, nsub)
    ratio = rec.lambda_min_ratio
    res = bl.fit_path_batch(gpu_ctx, to_dev(X32), to_dev(Y), to_dev(masks), nlambda=K, lambda_min_ratio=ratio,
                            tol=1e-10)
    B = Y.shape[0]
    problems = range(B)   # every problem, 64 at the second shape
    check_against_oracle(res, X32.astype(np.float64), Y, masks, K, ratio, problems)


@pytest.mark.parametrize("rule", [bl.SCREEN_NONE, bl.SCREEN_SSR, bl.SCREEN_BEDPP, bl.SCREEN_SSR_BEDPP])
def test_batch_all_rules_f64_all_rows(gpu_ctx, rule):
    rec = datagen.RECIPES["c1"].scaled(n=420, p=1300)
    Xt = datagen.design(rec)
    Y = np.stack([datagen.response(rec, Xt, t) for t in range(5)])
    K, ratio = 25, 0.05
    res = bl.fit_path_batch(gpu_ctx, to_dev(Xt), to_dev(Y), None, nlambda=K, lambda_min_ratio=ratio, rule=rule,
                            tol=1e-10)
    check_against_oracle(res, Xt, Y, None, K, ratio, range(5),
                         check_safe=rule in (bl.SCREEN_BEDPP, bl.SCREEN_SSR_BEDPP))
    assert (res.sweeps[:, 0] == 0).all() and (res.n_active[:, 0] == 0).all()


def test_batch_shared_masks_match_oracle(gpu_ctx):
    """Problems with the same row mask (several responses on one cross-validation fold) share its column
    statistics, one pass of X per distinct mask: three masks over twelve problems, each against the oracle."""
    rec, X32, Y, masks = cv_problem(800, 1700, 6, 2, seed_shift=11)
    masks = masks[np.arange(12) % 3]
    K, ratio = 12, rec.lambda_min_ratio
    res = bl.fit_path_batch(gpu_ctx, to_dev(X32), to_dev(Y), to_dev(masks), nlambda=K, lambda_min_ratio=ratio,
                            tol=1e-10)
    check_against_oracle(res, X32.astype(np.float64), Y, masks, K, ratio, range(12))


def test_batch_equals_single_problem_batches(gpu_ctx):
    """A problem's path does not depend on which other problems share the batch."""
    rec, X32, Y, masks = cv_problem(900, 1500, 4, 2, seed_shift=7)
    Xd = to_dev(X32)
    K = 15
    full = bl.fit_path_batch(gpu_ctx, Xd, to_dev(Y), to_dev(masks), nlambda=K, lambda_min_ratio=0.1, tol=1e-10)
    for b in (0, 5):
        one = bl.fit_path_batch(gpu_ctx, Xd, to_dev(Y[b:b + 1]), to_dev(masks[b:b + 1]), nlambda=K,
                                lambda_min_ratio=0.1, tol=1e-10)
        np.testing.assert_allclose(one.beta[0].cpu().numpy(), full.beta[b].cpu().numpy(), atol=1e-9)
        np.testing.assert_array_equal(one.n_active[0], full.n_active[b])


def test_graph_replayed_steps_equal_eager_launches(gpu_ctx):
    """The screening kernels of every lambda step replayed from the captured graph give the eagerly
    launched results bit for bit; the autotuned scan width is one of the candidates."""
    rec, X32, Y, masks = cv_problem(800, 1700, 5, 2, seed_shift=11)
    Xd, Yd, Md = to_dev(X32), to_dev(Y), to_dev(masks)
    g = bl.fit_path_batch(gpu_ctx, Xd, Yd, Md, nlambda=20, lambda_min_ratio=0.1, tol=1e-10)
    e = bl.fit_path_batch(gpu_ctx, Xd, Yd, Md, nlambda=20, lambda_min_ratio=0.1, tol=1e-10, eager=True)
    assert torch.equal(g.beta, e.beta)
    np.testing.assert_array_equal(g.n_strong, e.n_strong)
    np.testing.assert_array_equal(g.n_safe, e.n_safe)
    assert g.scan_cols in (64, 128, 256)


def test_batch_is_deterministic(gpu_ctx):
    rec, X32, Y, masks = cv_problem(700, 900, 6, 2, seed_shift=3)
    Xd, Yd, Md = to_dev(X32), to_dev(Y), to_dev(masks)
    r1 = bl.fit_path_batch(gpu_ctx, Xd, Yd, Md, nlambda=12, lambda_min_ratio=0.1, tol=1e-10)
    r2 = bl.fit_path_batch(gpu_ctx, Xd, Yd, Md, nlambda=12, lambda_min_ratio=0.1, tol=1e-10)
    assert torch.equal(r1.beta, r2.beta)
    np.testing.assert_array_equal(r1.obj, r2.obj)


def test_batch_rejects_invalid_inputs(gpu_ctx):
    rec, X32, Y, masks = cv_problem(200, 150, 2, 2)
    Xd, Yd = to_dev(X32), to_dev(Y)
    with pytest.raises(bl.BLError) as e:      # more than 64 problems
        bl.fit_path_batch(gpu_ctx, Xd, to_dev(np.tile(Y, (17, 1))), None, nlambda=5)
    assert e.value.status == bl.BL_ERR_INVALID
    bad = masks.copy()
    bad[1] = 0                                # a problem without rows
    with pytest.raises(bl.BLError) as e:
        bl.fit_path_batch(gpu_ctx, Xd, Yd, to_dev(bad), nlambda=5)
    assert e.value.status == bl.BL_ERR_INVALID
    with pytest.raises(bl.BLError) as e:      # int8 storage is the precision form's, not the batch's
        bl.fit_path_batch(gpu_ctx, to_dev(np.zeros((150, 200), dtype=np.int8)), Yd, None, nlambda=5)
    assert e.value.status == bl.BL_ERR_UNSUPPORTED
    with pytest.raises(bl.BLError) as e:
        bl.fit_path_batch(gpu_ctx, Xd, Yd, None, nlambda=0)
    assert e.value.status == bl.BL_ERR_INVALID


@pytest.mark.parametrize("prec", [bl.PREC_BF16X3, bl.PREC_BF16X2])
@pytest.mark.parametrize("n,p,nresp,nsub,K,ratio", [(1500, 4000, 8, 2, 20, None), (1037, 2222, 32, 2, 15, None),
                                                    (701, 40000, 8, 2, 6, 0.3)])
def test_batch_bf16_scans_equal_fp64_scans(gpu_ctx, n, p, nresp, nsub, K, ratio, prec):
    """The BF16 matrix-core check scans (f32 X, three or two pieces of x and r) re-take every decision within
    their error bound on the FP64 scan and start each solve from FP64 gradients: the same coefficients as the
    FP64 scans, bit for bit.  The scan splits its column list evenly over the workgroups the device holds at
    once: lists shorter than one 128-column tile per workgroup are cut by rows throughout (the first two
    shapes); 40,000 columns (every column survives BEDPP from the third step on) give every workgroup a whole
    tile and cut the tiles left over by rows."""
    rec, X32, Y, masks = cv_problem(n, p, nresp, nsub, seed_shift=7)
    ratio = ratio or rec.lambda_min_ratio
    Xd, Yd, Md = to_dev(X32), to_dev(Y), to_dev(masks)
    kw = dict(nlambda=K, lambda_min_ratio=ratio, tol=1e-10)
    r64 = bl.fit_path_batch(gpu_ctx, Xd, Yd, Md, **kw)
    rbf = bl.fit_path_batch(gpu_ctx, Xd, Yd, Md, precision=prec, **kw)
    assert rbf.k_done == K
    assert torch.equal(rbf.beta, r64.beta)
    np.testing.assert_array_equal(rbf.obj, r64.obj)
    np.testing.assert_array_equal(rbf.n_strong, r64.n_strong)
    check_against_oracle(rbf, X32.astype(np.float64), Y, masks, K, ratio, [0, Y.shape[0] - 1])
    with pytest.raises(bl.BLError) as e:
        bl.fit_path_batch(gpu_ctx, to_dev(X32.astype(np.float64)), Yd, Md, precision=prec, **kw)
    assert e.value.status == bl.BL_ERR_UNSUPPORTED


def test_autotune_cache_file(tmp_path, monkeypatch):
    """BL_AUTOTUNE_CACHE: the first context times the scan variants on this shape and appends its pick; a new
    context reads it back (no second line) and the two runs give the same coefficients."""
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("BL_AUTOTUNE_CACHE", str(path))
    rec, X32, Y, masks = cv_problem(700, 1300, 4, 2, seed_shift=9)
    Xd, Yd, Md = to_dev(X32), to_dev(Y), to_dev(masks)
    kw = dict(nlambda=8, lambda_min_ratio=rec.lambda_min_ratio, tol=1e-10)
    with bl.Context(0) as c1:
        r1 = bl.fit_path_batch(c1, Xd, Yd, Md, **kw)
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("bscan ") and lines[0].split()[3:5] == ["700", "1300"]
    with bl.Context(0) as c2:
        r2 = bl.fit_path_batch(c2, Xd, Yd, Md, **kw)
    assert path.read_text().splitlines() == lines
    assert r2.scan_cols == r1.scan_cols
    assert torch.equal(r1.beta, r2.beta)
