"""Paths the product can take that ordinary inputs do not reach, each against the FP64 oracle.

- The post-convergence repair: a screen that keeps only the previous active set (rule ACTIVE)
  leaves every entering feature to the check, which must add it back and re-solve (Section 2.2:
  a heuristic screen is made exact by the check).  Covered for the FP64 scan, both precision
  forms, the batched form, and the learned rule with a network that rejects nearly every
  candidate.  Each asserts violations were found and repaired (rounds >= 2) and that the path
  still equals the oracle's.
- The scan that reads r from global memory (n_total above 10,240 rows), f32 and f64, masked.
- The residual-form and single-workgroup coordinate descent, reached by lowering the context's
  covariance and helper limits.
- Resuming a path at lambda index 50 from a saved coefficient row and residual: bit-identical
  to the uninterrupted path.
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


def check_path(res, ref, K):
    assert res.k_done == K
    np.testing.assert_allclose(res.lam, ref.lam, rtol=1e-12)
    d = np.abs(res.beta.cpu().numpy() - ref.beta).max()
    rd = np.abs((res.obj - ref.obj) / ref.obj).max()
    print(f"max|d beta| {d:.2e}, max RD {rd:.2e}, violations {res.n_viol.sum()} (oracle {ref.n_viol.sum()}), "
          f"max rounds {res.rounds.max()}", flush=True)
    assert d <= 1e-6
    assert rd <= 1e-8
    np.testing.assert_array_equal(res.n_active, ref.n_active)


def repair_was_exercised(res, ref):
    assert res.n_viol.sum() > 0 and res.rounds.max() >= 2
    assert ref.n_viol.sum() > 0 and ref.n_rounds.max() >= 2
    # features entering at a lambda are found at the first check there on both sides; a feature within
    # rounding of the threshold at a later round may be counted on one side only
    same = np.mean(res.n_viol == ref.n_viol)
    assert same >= 0.9, same


ACTIVE_CASES = {
    # name: (recipe, n, p, storage dtype, masked)
    "gauss_f64": ("c1", 333, 1037, np.float64, False),
    "geno_f64_masked": ("c2", 900, 1500, np.float64, True),
    "ar1_f32_masked": ("c4", 700, 1200, np.float32, True),
}


@pytest.mark.parametrize("name", sorted(ACTIVE_CASES))
def test_active_set_screen_is_repaired_by_the_check(gpu_ctx, name):
    rec, n, p, dt, masked = ACTIVE_CASES[name]
    prob = datagen.make(rec, n=n, p=p, nresp=1, nsub=1) if rec == "c4" else datagen.make(rec, n=n, p=p)
    Xh = prob.Xt.astype(dt)
    mask = (np.random.default_rng(n).uniform(size=n) < 0.8).astype(np.uint8) if masked else None
    y = prob.y[0]
    K, ratio = 30, 0.05
    ref = oracle.fit_path(Xh.astype(np.float64), y, K=K, ratio=ratio, tol=1e-13, mask=mask,
                          screen=oracle.SCREEN_ACTIVE)
    print(f"{name}:", flush=True)
    res = bl.fit_path(gpu_ctx, to_dev(Xh), to_dev(y), nlambda=K, lambda_min_ratio=ratio, rule=bl.SCREEN_ACTIVE,
                      tol=1e-10, row_mask=to_dev(mask) if masked else None)
    check_path(res, ref, K)
    repair_was_exercised(res, ref)
    # BEDPP survivor counts equal the oracle's predicate
    np.testing.assert_array_equal(res.n_safe, ref.n_safe)


@pytest.mark.parametrize("prec", [bl.PREC_BF16X3, bl.PREC_I8X4], ids=["bf16x3", "i8x4"])
def test_active_set_screen_precision_forms(gpu_ctx, prec):
    n, p = 1216, 1900
    Xt = datagen.make("c2", n=n, p=p)
    X8 = Xt.Xt.astype(np.int8)
    y = Xt.y[0]
    K, ratio = 30, 0.05
    ref = oracle.fit_path(X8.astype(np.float64), y, K=K, ratio=ratio, tol=1e-13, screen=oracle.SCREEN_ACTIVE)
    Xd, yd = to_dev(X8), to_dev(y)
    kw = dict(nlambda=K, lambda_min_ratio=ratio, rule=bl.SCREEN_ACTIVE, tol=1e-10)
    r64 = bl.fit_path(gpu_ctx, Xd, yd, precision=bl.PREC_FP64, **kw)
    rlo = bl.fit_path(gpu_ctx, Xd, yd, precision=prec, **kw)
    check_path(rlo, ref, K)
    repair_was_exercised(rlo, ref)
    # every decision near a threshold is re-taken in FP64: the same path bit for bit
    assert torch.equal(rlo.beta, r64.beta)
    np.testing.assert_array_equal(rlo.n_viol, r64.n_viol)
    np.testing.assert_array_equal(rlo.rounds, r64.rounds)


def test_active_set_screen_batched(gpu_ctx):
    rec = datagen.RECIPES["c4"].scaled(n=900, p=1400, nresp=4, nsub=2, seed=204)
    prob = datagen.make(rec)
    X32 = prob.Xt
    Y = np.repeat(prob.y, 2, axis=0)
    masks = prob.masks
    K, ratio = 20, rec.lambda_min_ratio
    res = bl.fit_path_batch(gpu_ctx, to_dev(X32), to_dev(Y), to_dev(masks), nlambda=K, lambda_min_ratio=ratio,
                            rule=bl.SCREEN_ACTIVE, tol=1e-10)
    assert res.k_done == K
    beta = res.beta.cpu().numpy()
    X64 = X32.astype(np.float64)
    for b in range(Y.shape[0]):
        ref = oracle.fit_path(X64, Y[b], K=K, ratio=ratio, tol=1e-13, mask=masks[b], screen=oracle.SCREEN_ACTIVE)
        d = np.abs(beta[b] - ref.beta).max()
        rd = np.abs((res.obj[b] - ref.obj) / ref.obj).max()
        print(f"problem {b}: max|d beta| {d:.2e}, RD {rd:.2e}, violations {res.n_viol[b].sum()}, "
              f"max rounds {res.rounds[b].max()}", flush=True)
        assert d <= 1e-6 and rd <= 1e-8
        np.testing.assert_array_equal(res.n_active[b], ref.n_active)
        assert res.n_viol[b].sum() > 0 and res.rounds[b].max() >= 2


def test_learned_rule_with_a_rejecting_network_is_repaired(gpu_ctx):
    """An untrained network with a threshold near 1 turns away almost every strong-rule candidate; the
    check must bring back every one that enters, and the path must still be the hybrid rule's."""
    prob = datagen.make("c5", n=600, p=1500)
    Xt, y = prob.Xt, prob.y[0]
    K, ratio = 30, 0.05
    P = to_dev(bl.mlp_init(3))
    ref = oracle.fit_path(Xt.astype(np.float64), y, K=K, ratio=ratio, tol=1e-13)
    res = bl.fit_path(gpu_ctx, to_dev(Xt), to_dev(y), nlambda=K, lambda_min_ratio=ratio, rule=bl.SCREEN_LEARNED,
                      mlp=P, mlp_tau=0.999, tol=1e-10)
    check_path(res, ref, K)
    assert res.n_viol.sum() > 0 and res.rounds.max() >= 2


@pytest.mark.parametrize("dt", [np.float64, np.float32], ids=["f64", "f32"])
def test_path_with_residual_in_global_memory(gpu_ctx, dt):
    """n_total above 10,240 rows: the scan reads r from global memory instead of LDS."""
    n, p = 16000, 700
    prob = datagen.make("c1", n=n, p=p)
    Xh = prob.Xt.astype(dt)
    mask = (np.random.default_rng(16).uniform(size=n) < 0.9).astype(np.uint8)
    y = prob.y[0]
    K, ratio = 25, 0.05
    ref = oracle.fit_path(Xh.astype(np.float64), y, K=K, ratio=ratio, tol=1e-13, mask=mask)
    res = bl.fit_path(gpu_ctx, to_dev(Xh), to_dev(y), nlambda=K, lambda_min_ratio=ratio, tol=1e-10,
                      row_mask=to_dev(mask))
    check_path(res, ref, K)
    np.testing.assert_array_equal(res.n_safe, ref.n_safe)
    # the check scan itself, element by element, at this height
    c, s, keep, nn = oracle.standardize(Xh.astype(np.float64), mask)
    rng = np.random.default_rng(2)
    r = rng.normal(size=n) + 0.3
    r[mask == 0] = 0.0
    oz = oracle.zscan(Xh.astype(np.float64), c, s, keep, r, mask)
    cols = np.flatnonzero(keep).astype(np.int32)
    z = bl.scan(gpu_ctx, to_dev(Xh), to_dev(c), to_dev(s), to_dev(r), to_dev(cols), row_mask=to_dev(mask))
    np.testing.assert_allclose(z.cpu().numpy()[cols], oz[cols], atol=1e-12 * np.abs(oz).max())


@pytest.mark.parametrize("limits,what", [((8, -1), "residual"), ((0, 12), "few helpers"),
                                         ((0, 0), "single-workgroup")])
def test_cd_fallbacks_match_oracle(limits, what):
    """Lowered limits send working sets to the residual-form solve (cov_max 8) or, with the helper count
    capped below what a set needs, to the single-workgroup covariance solve."""
    n, p, m_set = 800, 2200, 1500
    prob = datagen.make("c1", n=n, p=p)
    Xt = prob.Xt
    oc, os_, ok, on = oracle.standardize(Xt)
    oy, oyt, oa, olm, ojs = oracle.lambda_max(Xt, oc, os_, ok, prob.y[0])
    cset = np.sort(np.argsort(-np.abs(oa))[:m_set]).astype(np.int32)
    lam = 0.15 * olm
    ob, orr = np.zeros(p), oyt.copy()
    conv, osw = oracle.cd(Xt, oc, os_, lam, cset.astype(np.int64), ob, orr, tol=1e-11)
    assert conv
    with bl.Context(0) as ctx:
        lim0 = ctx.limits()
        assert lim0["resident"] >= 2 and lim0["cd_helpers"] == min(255, lim0["resident"] - 1)
        ctx.set_limits(*limits)
        print(f"{what}: limits {ctx.limits()}", flush=True)
        bd, rd = to_dev(np.zeros(p)), to_dev(oyt.copy())
        sw = bl.cd_solve(ctx, to_dev(Xt), to_dev(oc), to_dev(os_), lam, to_dev(cset), bd, rd, tol=1e-11)
        assert abs(sw - osw) <= 1
        np.testing.assert_allclose(bd.cpu().numpy(), ob, atol=1e-9)
        np.testing.assert_allclose(rd.cpu().numpy(), orr, atol=1e-8 * np.abs(oyt).max())
        # a whole path through the same fallback
        K, ratio = 25, 0.05
        ref = oracle.fit_path(Xt, prob.y[0], K=K, ratio=ratio, tol=1e-13)
        res = bl.fit_path(ctx, to_dev(Xt), to_dev(prob.y[0]), nlambda=K, lambda_min_ratio=ratio, tol=1e-10)
        check_path(res, ref, K)
        with pytest.raises(bl.BLError) as e:
            ctx.set_limits(0, lim0["resident"])
        assert e.value.status == bl.BL_ERR_INVALID


@pytest.mark.parametrize("with_r", [True, False], ids=["saved_residual", "recomputed_residual"])
def test_resume_at_lambda_50(gpu_ctx, with_r):
    prob = datagen.make("c2", n=1000, p=2500)
    X64 = prob.Xt.astype(np.float64)
    Xd, yd = to_dev(X64), to_dev(prob.y[0])
    K, k0 = 100, 50
    full = bl.fit_path(gpu_ctx, Xd, yd, nlambda=K, lambda_min_ratio=0.05, tol=1e-10)
    lam = full.lam.copy()
    r_saved = torch.zeros(prob.Xt.shape[1], dtype=torch.float64, device=DEV)
    first = bl.fit_path(gpu_ctx, Xd, yd, nlambda=k0, lambdas=lam[:k0], tol=1e-10, r_out=r_saved)
    assert torch.equal(first.beta, full.beta[:k0])
    rest = bl.fit_path(gpu_ctx, Xd, yd, nlambda=K, lambdas=lam, tol=1e-10, k_start=k0,
                       beta_init=first.beta[k0 - 1].contiguous(), r_init=r_saved if with_r else None)
    assert rest.k_done == K
    if with_r:
        assert torch.equal(rest.beta[k0:], full.beta[k0:])
        np.testing.assert_array_equal(rest.obj[k0:], full.obj[k0:])
        np.testing.assert_array_equal(rest.sweeps[k0:], full.sweeps[k0:])
    else:
        assert (rest.beta[k0:] - full.beta[k0:]).abs().max().item() <= 1e-9
    np.testing.assert_array_equal(rest.n_active[k0:], full.n_active[k0:])
    ref = oracle.fit_path(X64, prob.y[0], K=K, ratio=0.05, tol=1e-13)
    assert np.abs(rest.beta[k0:].cpu().numpy() - ref.beta[k0:]).max() <= 1e-6


def test_resume_rejects_what_it_cannot_do(gpu_ctx):
    prob = datagen.make("c1", n=100, p=200)
    Xd, yd = to_dev(prob.Xt), to_dev(prob.y[0])
    with pytest.raises(bl.BLError) as e:
        bl.fit_path(gpu_ctx, Xd, yd, nlambda=10, k_start=5)
    assert e.value.status == bl.BL_ERR_INVALID
    with pytest.raises(bl.BLError) as e:
        bl.fit_path(gpu_ctx, Xd, yd, nlambda=10, k_start=10, beta_init=torch.zeros(200, dtype=torch.float64,
                                                                                    device=DEV))
    assert e.value.status == bl.BL_ERR_INVALID
    with pytest.raises(bl.BLError) as e:
        bl.fit_path(gpu_ctx, Xd, yd, nlambda=10, k_start=4, beta_init=torch.zeros(200, dtype=torch.float64,
                                                                                   device=DEV),
                    rule=bl.SCREEN_LEARNED, mlp=to_dev(bl.mlp_init(0)), mlp_tau=0.5)
    assert e.value.status == bl.BL_ERR_UNSUPPORTED
