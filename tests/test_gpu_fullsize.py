"""Full-size parity in the launch configurations bench.py times (CD tolerance 1e-10 here, 1e-8 there, except
the learned form's path, certified at bench.py's 1e-8): the
plain path on the 5,000 x 500,000 genotype design (FP64, 20 GB), the precision form on the 10,000 x
2,000,000 genotype design (int8, 20 GB), the batched form on the 20,000 x 200,000 AR(1) design (64
problems) and the learned form on the 5,000 x 1,000,000 block-AR(1) design (float32, 20 GB).

The oracle cannot run these paths whole in seconds, so the checks use what the oracle computes column by
column: sampled column statistics, lambda_max over every column (in chunks), and KKT certificates of the
GPU coefficients at sampled lambda values, with the standardization, the residual and z computed by the
oracle over every column, in chunks.
"""
import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_1701_05936_amd as bl
from conftest import progress

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
CHUNK = 25_000


def log(msg):
    progress(f"[fullsize] {msg}")


def chunked(Xt, fn):
    """fn(block of columns as float64, offset) over all columns in chunks."""
    p = Xt.shape[0]
    out = []
    for j0 in range(0, p, CHUNK):
        out.append(fn(np.ascontiguousarray(Xt[j0:j0 + CHUNK], dtype=np.float64), j0))
        if (j0 // CHUNK) % 10 == 9:
            log(f"  columns {j0 + CHUNK} of {p}")
    return out


def kkt_residuals(Xt, c, s, keep, yt, beta, lam, mask=None):
    """max over inactive kept j of |z_j| / lam - 1, and max over active j of |z_j - lam sign(beta_j)| / lam."""
    act = np.flatnonzero(beta)
    r = yt.copy()
    for j in act:   # residual from the active columns only, in FP64
        xj = (Xt[j].astype(np.float64) - c[j]) / s[j]
        if mask is not None:
            xj = xj * mask
        r -= beta[j] * xj
    zs = chunked(Xt, lambda blk, j0: oracle.zscan(blk, c[j0:j0 + len(blk)], s[j0:j0 + len(blk)],
                                                  keep[j0:j0 + len(blk)], r, mask))
    z = np.concatenate(zs)
    inactive = keep & (beta == 0)
    out_viol = np.max(np.abs(z[inactive])) / lam - 1.0
    on_act = np.max(np.abs(z[act] - lam * np.sign(beta[act]))) / lam if act.size else 0.0
    return out_viol, on_act


@pytest.fixture(scope="module")
def c2_full(gpu_ctx):
    rec = datagen.RECIPES["c2"]
    log("generating c2 at full size ...")
    Xt = datagen.design(rec)                 # (p, n) uint8 codes
    y = datagen.response(rec, Xt, 0)
    Xd = torch.from_numpy(Xt).to(DEV).to(torch.float64)
    res = bl.fit_path(gpu_ctx, Xd, torch.from_numpy(y).to(DEV), nlambda=rec.nlambda,
                      lambda_min_ratio=rec.lambda_min_ratio, rule=bl.SCREEN_SSR_BEDPP, tol=1e-10)
    log(f"GPU path: {res.time_ms:.0f} ms, {res.n_active[-1]} active at the end")
    beta = res.beta.cpu().numpy()
    c, s, keep = res.center.cpu().numpy(), res.scale.cpu().numpy(), res.keep.cpu().numpy().astype(bool)
    del Xd
    torch.cuda.empty_cache()
    return rec, Xt, y, res, beta, c, s, keep


def test_c2_full_standardization_and_lambda_max(c2_full):
    rec, Xt, y, res, beta, c, s, keep = c2_full
    rng = np.random.default_rng(0)
    cols = np.sort(rng.choice(Xt.shape[0], 300, replace=False))
    oc, os_, okeep, n = oracle.standardize(Xt[cols].astype(np.float64))
    np.testing.assert_allclose(c[cols], oc, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(s[cols], os_, rtol=1e-13)
    np.testing.assert_array_equal(keep[cols], okeep.astype(bool))
    # lambda_max and j* over every column, chunk by chunk
    best, bj = -1.0, -1
    for part, j0 in zip(chunked(Xt, lambda blk, j0: oracle.lambda_max(blk, c[j0:j0 + len(blk)], s[j0:j0 + len(blk)],
                                                                        keep[j0:j0 + len(blk)], y)[2]),
                        range(0, Xt.shape[0], CHUNK)):
        a = np.where(keep[j0:j0 + part.size], np.abs(part), -1.0)
        j = int(np.argmax(a))
        if a[j] > best:
            best, bj = float(a[j]), j0 + j
    log(f"lambda_max {res.lambda_max:.15g} vs oracle {best:.15g}, j* {res.jstar} vs {bj}")
    assert abs(res.lambda_max - best) <= 1e-12 * best
    assert res.jstar == bj
    assert res.k_done == rec.nlambda


@pytest.mark.parametrize("k", [20, 60, 99])
def test_c2_full_kkt_certificate(c2_full, k):
    rec, Xt, y, res, beta, c, s, keep = c2_full
    yt = y - y.mean()
    lam = res.lam[k]
    out_v, on_a = kkt_residuals(Xt, c, s, keep, yt, beta[k], lam)
    log(f"k={k}: lambda {lam:.6g}, active {np.count_nonzero(beta[k])}, max inactive |z|/lambda - 1 = {out_v:.2e}, "
        f"max active |z - lambda sign| / lambda = {on_a:.2e}")
    # CD stops at max |d beta| < 1e-10: the optimality conditions hold to about that order in z
    assert out_v <= 1e-6
    assert on_a <= 1e-6


@pytest.fixture(scope="module")
def c4_full(gpu_ctx):
    rec = datagen.RECIPES["c4"]
    log("generating c4 at full size ...")
    prob = datagen.make(rec)
    Y = np.repeat(prob.y, rec.nsub, axis=0)
    Xd = torch.from_numpy(prob.Xt).to(DEV)
    Yd, Md = torch.from_numpy(Y).to(DEV), torch.from_numpy(prob.masks).to(DEV)
    kw = dict(nlambda=rec.nlambda, lambda_min_ratio=rec.lambda_min_ratio, rule=bl.SCREEN_SSR_BEDPP, tol=1e-10)
    res = bl.fit_path_batch(gpu_ctx, Xd, Yd, Md, **kw)
    log(f"GPU batch: {res.time_ms:.0f} ms for {Y.shape[0]} problems")
    # the BF16 check-scan forms, the configuration bench.py times (two pieces) and three pieces
    same = {}
    for name, prec in (("bf16x2", bl.PREC_BF16X2), ("bf16x3", bl.PREC_BF16X3)):
        rb = bl.fit_path_batch(gpu_ctx, Xd, Yd, Md, precision=prec, **kw)
        same[name] = bool(torch.equal(rb.beta, res.beta)) and rb.k_done == res.k_done
        log(f"GPU batch, {name} check scans: {rb.time_ms:.0f} ms, coefficients bit-identical: {same[name]}")
        del rb
    beta = res.beta.cpu().numpy()
    del Xd
    torch.cuda.empty_cache()
    return rec, prob, Y, res, beta, same


def test_c4_full_bf16_check_scans_equal_fp64(c4_full):
    """At the benchmarked shape the BF16 matrix-core check scans (two and three pieces) take every decision
    the FP64 scans take: all 64 problems' coefficients are the same bits."""
    assert c4_full[5] == {"bf16x2": True, "bf16x3": True}


@pytest.mark.parametrize("b,k", [(0, 49), (37, 25)])
def test_c4_full_kkt_certificate(c4_full, b, k):
    rec, prob, Y, res, beta, _ = c4_full
    Xt, mask = prob.Xt, prob.masks[b]
    # the problem's own standardization by the oracle, chunk by chunk
    st = chunked(Xt, lambda blk, j0: oracle.standardize(blk, mask)[:3])
    c = np.concatenate([t[0] for t in st])
    s = np.concatenate([t[1] for t in st])
    keep = np.concatenate([t[2] for t in st]).astype(bool)
    y = Y[b]
    yt = np.where(mask > 0, y - y[mask > 0].mean(), 0.0)
    lam = res.lam[b, k]
    out_v, on_a = kkt_residuals(Xt, c, s, keep, yt, beta[b, k], lam, mask)
    log(f"problem {b}, k={k}: rows {int(mask.sum())}, active {np.count_nonzero(beta[b, k])}, "
        f"inactive {out_v:.2e}, active {on_a:.2e}")
    assert out_v <= 1e-6
    assert on_a <= 1e-6


def oracle_stats(Xt, mask=None):
    """The oracle's column statistics over every column, chunk by chunk."""
    st = chunked(Xt, lambda blk, j0: oracle.standardize(blk, mask)[:3])
    return (np.concatenate([t[0] for t in st]), np.concatenate([t[1] for t in st]),
            np.concatenate([t[2] for t in st]).astype(bool))


@pytest.fixture(scope="module")
def c3_full(gpu_ctx):
    rec = datagen.RECIPES["c3"]
    log("generating c3 at full size ...")
    Xt = datagen.design(rec)                 # (p, n) uint8 codes
    y = datagen.response(rec, Xt, 0)
    Xd = torch.from_numpy(Xt.view(np.int8)).to(DEV)
    yd = torch.from_numpy(y).to(DEV)
    kw = dict(nlambda=rec.nlambda, lambda_min_ratio=rec.lambda_min_ratio, rule=bl.SCREEN_SSR_BEDPP, tol=1e-10)
    lp = bl.fit_path(gpu_ctx, Xd, yd, precision=bl.PREC_I8X4, **kw)
    bp = bl.fit_path(gpu_ctx, Xd, yd, precision=bl.PREC_BF16X3, **kw)
    bp.beta = bp.beta.cpu()
    hp = bl.fit_path(gpu_ctx, Xd, yd, precision=bl.PREC_FP64, **kw)
    log(f"int8 form {lp.time_ms:.0f} ms, BF16 form {bp.time_ms:.0f} ms, FP64 scans {hp.time_ms:.0f} ms, "
        f"{lp.n_active[-1]} active at the end, {int(lp.n_recheck.sum())} / {int(bp.n_recheck.sum())} FP64 rechecks")
    del Xd
    torch.cuda.empty_cache()
    log("oracle column statistics of c3 ...")
    stats = oracle_stats(Xt)
    return rec, Xt, y, lp, bp, hp, stats


def test_c3_full_precision_forms_equal_fp64_path(c3_full):
    """The int8 and the BF16 matrix-core scans take every decision the FP64 scans take: identical
    coefficients."""
    rec, Xt, y, lp, bp, hp, stats = c3_full
    assert lp.k_done == rec.nlambda and bp.k_done == rec.nlambda and hp.k_done == rec.nlambda
    assert torch.equal(lp.beta, hp.beta)
    assert torch.equal(bp.beta, hp.beta.cpu())
    for form in (lp, bp):
        np.testing.assert_array_equal(form.n_active, hp.n_active)
        np.testing.assert_array_equal(form.n_strong, hp.n_strong)


@pytest.mark.parametrize("k", [30, 99])
def test_c3_full_kkt_certificate(c3_full, k):
    rec, Xt, y, lp, bp, hp, (c, s, keep) = c3_full
    beta = lp.beta[k].cpu().numpy()
    lam = lp.lam[k]
    out_v, on_a = kkt_residuals(Xt, c, s, keep, y - y.mean(), beta, lam)
    log(f"c3 k={k}: lambda {lam:.6g}, active {np.count_nonzero(beta)}, max inactive |z|/lambda - 1 over all "
        f"columns = {out_v:.2e}, max active |z - lambda sign| / lambda = {on_a:.2e}")
    assert out_v <= 1e-6
    assert on_a <= 1e-6


@pytest.fixture(scope="module")
def c5_full(gpu_ctx):
    """The learned form on the full c5 design over its whole 100-lambda grid, with a network trained on 10
    recorded strong-rule paths (first 60 lambda values) of a 10,000-column design of the same recipe.  The
    path runs at the CD tolerance bench.py times it at (1e-8): the certificate is of the timed configuration."""
    rec = datagen.RECIPES["c5"]
    depth = 60
    full = rec.nlambda
    step = rec.lambda_min_ratio ** (1.0 / (rec.nlambda - 1))
    tr = rec.scaled(p=10_000, seed=rec.seed + 1000, nresp=10)
    tp = datagen.make(tr)
    Xtr = torch.from_numpy(tp.Xt).to(DEV)
    cap = 4_000_000
    feat = torch.zeros((cap, 4), dtype=torch.float32, device=DEV)
    lab = torch.zeros(cap, dtype=torch.float32, device=DEV)
    n_rec = 0
    for t in range(tr.nresp):
        ytr = torch.from_numpy(tp.y[t]).to(DEV)
        lmax = bl.fit_path(gpu_ctx, Xtr, ytr, nlambda=1, want_beta=False).lambda_max
        r = bl.fit_path(gpu_ctx, Xtr, ytr, nlambda=depth, lambdas=lmax * step ** np.arange(depth),
                        rule=bl.SCREEN_SSR_BEDPP, tol=1e-8, rec_feat=feat[n_rec:], rec_label=lab[n_rec:],
                        want_beta=False)
        n_rec += r.n_recorded
        log(f"c5 training path {t + 1} of {tr.nresp}: {r.n_recorded} records")
    P = torch.from_numpy(bl.mlp_init(1)).to(DEV)
    info = bl.mlp_train(gpu_ctx, feat[:n_rec].contiguous(), lab[:n_rec].contiguous(), P, epochs=10, batch=8192,
                        lr=2e-3, seed=5, target_recall=0.995)
    del Xtr, feat, lab
    log(f"trained on {n_rec} records: recall {info['recall']:.4f}, tau {info['tau']:.4g}")
    log("generating c5 at full size ...")
    Xt = datagen.design(rec)                 # (p, n) float32
    y = datagen.response(rec, Xt, 0)
    Xd = torch.from_numpy(Xt).to(DEV)
    yd = torch.from_numpy(y).to(DEV)
    lmax = bl.fit_path(gpu_ctx, Xd, yd, nlambda=1, want_beta=False).lambda_max
    res = bl.fit_path(gpu_ctx, Xd, yd, nlambda=full, lambda_min_ratio=rec.lambda_min_ratio,
                      rule=bl.SCREEN_LEARNED, mlp=P, mlp_tau=info["tau"], tol=1e-8)
    log(f"learned path: {res.time_ms:.0f} ms, {res.n_active[-1]} active at the end, "
        f"{int(res.n_viol.sum())} violations repaired, working sets {int(res.n_strong.sum())}")
    del Xd
    torch.cuda.empty_cache()
    log("oracle column statistics of c5 ...")
    stats = oracle_stats(Xt)
    return rec, Xt, y, res, stats


@pytest.mark.parametrize("k", [30, 59, 80, 99])
def test_c5_full_learned_kkt_certificate(c5_full, k):
    rec, Xt, y, res, (c, s, keep) = c5_full
    assert res.k_done == rec.nlambda
    beta = res.beta[k].cpu().numpy()
    lam = res.lam[k]
    out_v, on_a = kkt_residuals(Xt, c, s, keep, y - y.mean(), beta, lam)
    log(f"c5 k={k}: lambda {lam:.6g}, active {np.count_nonzero(beta)}, max inactive |z|/lambda - 1 over all "
        f"columns = {out_v:.2e}, max active |z - lambda sign| / lambda = {on_a:.2e}")
    assert out_v <= 1e-6
    assert on_a <= 1e-6
