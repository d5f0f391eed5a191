"""The path with X in host memory (bl_fit_path_host), streamed in column panels.

The streamed path runs the same kernels over the same bytes as the path with X in device memory, so its
results are compared bit for bit with that path (and, once, with the oracle); the counters show that
panels without BEDPP survivors were never moved.
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


def pinned(a):
    return torch.from_numpy(np.ascontiguousarray(a)).pin_memory()


def same_path(a, b):
    assert a.k_done == b.k_done
    assert torch.equal(a.beta, b.beta)
    np.testing.assert_array_equal(a.obj, b.obj)
    np.testing.assert_array_equal(a.n_safe, b.n_safe)
    np.testing.assert_array_equal(a.n_strong, b.n_strong)
    np.testing.assert_array_equal(a.sweeps, b.sweeps)
    np.testing.assert_array_equal(a.n_viol, b.n_viol)


CASES = {
    # name: (recipe, n, p, dtype, masked, panel_cols, rule)
    "geno_f64": ("c2", 1200, 20000, np.float64, False, 1500, bl.SCREEN_SSR_BEDPP),
    "geno_i8_masked": ("c2", 1104, 15000, np.int8, True, 1024, bl.SCREEN_SSR_BEDPP),
    "ar1_f32_masked_ssr": ("c4", 900, 9000, np.float32, True, 1000, bl.SCREEN_SSR),
    "gauss_f64_active": ("c1", 500, 6000, np.float64, False, 777, bl.SCREEN_ACTIVE),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_host_path_equals_device_path(gpu_ctx, name):
    rec, n, p, dt, masked, pc, rule = CASES[name]
    prob = datagen.make(rec, n=n, p=p, nresp=1, nsub=1) if rec == "c4" else datagen.make(rec, n=n, p=p)
    Xh = prob.Xt.astype(dt)
    y = to_dev(prob.y[0])
    mask = to_dev((np.random.default_rng(n).uniform(size=n) < 0.85).astype(np.uint8)) if masked else None
    kw = dict(nlambda=40, lambda_min_ratio=0.05, rule=rule, tol=1e-10, row_mask=mask)
    dev = bl.fit_path(gpu_ctx, to_dev(Xh), y, **kw)
    host, st = bl.fit_path_host(gpu_ctx, pinned(Xh), y, panel_cols=pc, **kw)
    print(f"{name}: {st}, device {dev.time_ms:.0f} ms, host {host.time_ms:.0f} ms", flush=True)
    same_path(host, dev)
    assert st["panel_cols"] == pc
    if rule != bl.SCREEN_SSR:
        assert st["panels_skipped"] > 0   # early lambda values: panels without BEDPP survivors stay put
    # the two set-up passes move every panel once at least
    npan = (p + pc - 1) // pc
    assert st["panels_streamed"] >= 2 * npan


def test_host_path_matches_oracle_and_pageable_memory(gpu_ctx):
    prob = datagen.make("c1", n=400, p=3000)
    K, ratio = 30, 0.05
    ref = oracle.fit_path(prob.Xt, prob.y[0], K=K, ratio=ratio, tol=1e-13)
    # pageable host memory (no pinning): slower copies, same results
    host, st = bl.fit_path_host(gpu_ctx, torch.from_numpy(prob.Xt.copy()), to_dev(prob.y[0]), nlambda=K,
                                lambda_min_ratio=ratio, tol=1e-10, panel_cols=640)
    assert np.abs(host.beta.cpu().numpy() - ref.beta).max() <= 1e-6
    assert np.abs((host.obj - ref.obj) / ref.obj).max() <= 1e-8
    np.testing.assert_array_equal(host.n_active, ref.n_active)


def test_host_path_resume_and_elastic_net(gpu_ctx):
    prob = datagen.make("c2", n=700, p=5000)
    X64 = prob.Xt.astype(np.float64)
    y = to_dev(prob.y[0])
    full = bl.fit_path(gpu_ctx, to_dev(X64), y, nlambda=40, lambda_min_ratio=0.05, tol=1e-10)
    r_saved = torch.zeros(700, dtype=torch.float64, device=DEV)
    first, _ = bl.fit_path_host(gpu_ctx, pinned(X64), y, nlambda=20, lambdas=full.lam[:20], tol=1e-10,
                                r_out=r_saved, panel_cols=900)
    rest, _ = bl.fit_path_host(gpu_ctx, pinned(X64), y, nlambda=40, lambdas=full.lam, tol=1e-10, k_start=20,
                               beta_init=first.beta[19].contiguous(), r_init=r_saved, panel_cols=900)
    assert torch.equal(rest.beta[20:], full.beta[20:])
    with pytest.raises(bl.BLError) as e:
        bl.fit_path_host(gpu_ctx, pinned(X64), y, nlambda=40, lambdas=full.lam, k_start=20,
                         beta_init=first.beta[19].contiguous())
    assert e.value.status == bl.BL_ERR_UNSUPPORTED
    w = to_dev(np.random.default_rng(1).uniform(0.5, 2.0, size=5000))
    de = bl.fit_path(gpu_ctx, to_dev(X64), y, nlambda=30, lambda_min_ratio=0.05, tol=1e-10, alpha=0.6,
                     penalty_factor=w)
    he, _ = bl.fit_path_host(gpu_ctx, pinned(X64), y, nlambda=30, lambda_min_ratio=0.05, tol=1e-10, alpha=0.6,
                             penalty_factor=w, panel_cols=1111)
    same_path(he, de)
    with pytest.raises(bl.BLError) as e:
        bl.fit_path_host(gpu_ctx, pinned(prob.Xt.astype(np.int8)), y, nlambda=10, precision=bl.PREC_I8X4)
    assert e.value.status == bl.BL_ERR_UNSUPPORTED
