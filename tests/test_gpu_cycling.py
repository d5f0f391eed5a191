"""Active-set cycling in the plain path's solves (Section 3.1.1: the descent iterates over the nonzero
coefficients), against the FP64 oracle's plain cyclic descent over the working set.

Both stop on the same rule (a sweep over the whole working set that changes no coefficient by tol), so
their paths agree to the solve tolerance.  Each case lowers the context's cycle_min so that every working
set of at least 8 features cycles, and checks the path against the oracle, against the same path with
cycling turned off (the coordinate updates of both are printed).  The covariance solve in its
multi-workgroup and single-workgroup forms and the residual-form solve are each reached through the
context's limits; the repair loop, the elastic net and a row mask ride along.
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


def path_with(ctx, limits, Xd, yd, **kw):
    ctx.set_limits(**limits)
    ctx.profile(True)
    res = bl.fit_path(ctx, Xd, yd, **kw)
    updates = ctx.profile_get(bl.PROF_CD)["units"]
    ctx.profile(False)
    return res, updates


CASES = {
    # name: (recipe, n, p, dtype, masked, extra limits, fit options)
    "multi_f64": ("c2", 900, 6000, np.float64, False, {}, {}),
    "multi_f32_masked": ("c4", 1100, 5000, np.float32, True, {}, {}),
    "single_workgroup": ("c1", 700, 4000, np.float64, False, {"cd_helpers": 0}, {}),
    "residual_form": ("c1", 600, 3000, np.float64, True, {"cov_max": 8}, {}),
    "repair_active_rule": ("c2", 800, 5000, np.float64, False, {}, {"rule": bl.SCREEN_ACTIVE}),
    "elastic_net": ("c4", 900, 4000, np.float32, False, {}, {"alpha": 0.7}),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_cycling_matches_oracle(name):
    rec, n, p, dt, masked, lim, extra = CASES[name]
    prob = datagen.make(rec, n=n, p=p, nresp=1, nsub=1) if rec == "c4" else datagen.make(rec, n=n, p=p)
    X = prob.Xt.astype(dt)
    y = prob.y[0]
    mask = (np.random.default_rng(n).uniform(size=n) < 0.85).astype(np.uint8) if masked else None
    K, ratio = 30, 0.05
    alpha = extra.get("alpha", 1.0)
    screen = oracle.SCREEN_ACTIVE if extra.get("rule") == bl.SCREEN_ACTIVE else oracle.SCREEN_SSR
    ref = oracle.fit_path(X.astype(np.float64), y, K=K, ratio=ratio, mask=mask, tol=1e-13, screen=screen,
                          alpha=alpha)
    kw = dict(nlambda=K, lambda_min_ratio=ratio, tol=1e-10, row_mask=None if mask is None else to_dev(mask), **extra)
    Xd, yd = to_dev(X), to_dev(y)
    with bl.Context(0) as ctx:
        cyc, u_cyc = path_with(ctx, dict(cycle_min=8, **lim), Xd, yd, **kw)
        assert ctx.limits()["cycle_min"] == 8
        plain, u_plain = path_with(ctx, dict(cycle_min=-1), Xd, yd, **kw)
        assert ctx.limits()["cycle_min"] == -1
    d = np.abs(cyc.beta.cpu().numpy() - ref.beta).max()
    rd = np.abs((cyc.obj - ref.obj) / ref.obj).max()
    dp = (cyc.beta - plain.beta).abs().max().item()
    print(f"{name}: max|d beta| {d:.2e} vs oracle, {dp:.2e} vs no cycling, RD {rd:.2e}; coordinate updates "
          f"{u_cyc:.0f} cycling, {u_plain:.0f} not; sweeps {cyc.sweeps.sum()} vs {plain.sweeps.sum()}, "
          f"violations {cyc.n_viol.sum()}", flush=True)
    assert cyc.k_done == K
    np.testing.assert_allclose(cyc.lam, ref.lam, rtol=1e-12)
    assert d <= 1e-6 and rd <= 1e-8 and dp <= 1e-6
    np.testing.assert_array_equal(cyc.n_active, ref.n_active)
    np.testing.assert_array_equal(cyc.n_active, plain.n_active)
    if extra.get("rule") == bl.SCREEN_ACTIVE:
        assert cyc.n_viol.sum() > 0 and cyc.rounds.max() >= 2


def test_cycle_limit_is_checked(gpu_ctx):
    with pytest.raises(bl.BLError) as e:
        gpu_ctx.set_limits(cycle_min=-2)
    assert e.value.status == bl.BL_ERR_INVALID
    assert gpu_ctx.limits()["cycle_min"] == -1   # off unless asked for
