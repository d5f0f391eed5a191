"""Learned-screening form: the screening network's kernels against the oracle, its training, and the
path with the network in the loop against the oracle and against the strong rule it stands beside."""
import numpy as np
import pytest
import torch

import datagen
import oracle
import paper_1701_05936_amd as bl

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
H = bl.MLP_HIDDEN


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def params_and_features(seed, m):
    rng = np.random.default_rng(seed)
    P = bl.mlp_init(seed)
    P += rng.normal(0, 0.05, size=P.size).astype(np.float32)   # nonzero biases too
    feat = np.abs(rng.normal(0.6, 0.4, size=(m, 4))).astype(np.float32)
    feat[:, 3] = rng.uniform(0.9, 1.0, size=m).astype(np.float32)
    label = (rng.uniform(size=m) < 1 / (1 + np.exp(-4 * (feat[:, 0] - 0.8)))).astype(np.float32)
    return P, feat, label


@pytest.mark.parametrize("m", [1, 127, 1000, 4099])
def test_forward_matches_oracle(gpu_ctx, m):
    P, feat, _ = params_and_features(m, m)
    prob = bl.mlp_forward(gpu_ctx, to_dev(feat), to_dev(P)).cpu().numpy()
    ref = oracle.mlp_forward(feat.astype(np.float64), P.astype(np.float64), H)
    # FP32 evaluation of a 4-64-64-1 network: a few hundred roundings of O(1) terms
    np.testing.assert_allclose(prob, ref, rtol=0, atol=2e-5)


@pytest.mark.parametrize("m", [1, 128, 129, 1000, 5000])
def test_gradient_matches_oracle(gpu_ctx, m):
    P, feat, label = params_and_features(100 + m, m)
    loss, grad = bl.mlp_loss_grad(gpu_ctx, to_dev(feat), to_dev(label), to_dev(P))
    rloss, rgrad = oracle.mlp_loss_grad(feat.astype(np.float64), label.astype(np.float64), P.astype(np.float64), H)
    grad = grad.cpu().numpy()
    scale = np.abs(rgrad).max()
    err = np.abs(grad - rgrad).max()
    print(f"m={m}: loss {loss:.6f} vs {rloss:.6f}, max |dg| {err:.2e} of max |g| {scale:.2e}")
    assert abs(loss - rloss) <= 1e-5 * max(1.0, abs(rloss))
    assert err <= 1e-4 * scale + 1e-7


def test_one_adam_step_follows_its_definition(gpu_ctx):
    """With one step over one batch, Adam moves each parameter by lr g / (|g| + eps) (bias-corrected moments)."""
    m = 512
    P, feat, label = params_and_features(7, m)
    Pd = to_dev(P.copy())
    lr, eps = 1e-3, 1e-8
    bl.mlp_train(gpu_ctx, to_dev(feat), to_dev(label), Pd, epochs=1, batch=512, lr=lr, eps=eps, seed=3)
    _, g = oracle.mlp_loss_grad(feat.astype(np.float64), label.astype(np.float64), P.astype(np.float64), H)
    expect = P.astype(np.float64) - lr * g / (np.abs(g) + eps)
    got = Pd.cpu().numpy().astype(np.float64)
    sure = np.abs(g) > 1e-3 * np.abs(g).max()       # the sign of tiny gradients is not fixed by FP32 sums
    np.testing.assert_allclose(got[sure], expect[sure], rtol=0, atol=1e-6)


def test_training_lowers_the_loss_and_is_deterministic(gpu_ctx):
    m = 20000
    _, feat, label = params_and_features(11, m)
    fd, ld = to_dev(feat), to_dev(label)
    P0 = bl.mlp_init(5)
    runs = []
    for _ in range(2):
        Pd = to_dev(P0.copy())
        info = bl.mlp_train(gpu_ctx, fd, ld, Pd, epochs=8, batch=1024, lr=3e-3, seed=9, target_recall=0.99)
        runs.append((Pd, info))
    (P1, i1), (P2, i2) = runs
    print(i1)
    assert i1["loss_last"] < i1["loss_first"]
    assert i1["steps"] == 8 * ((m + 1023) // 1024)
    assert torch.equal(P1, P2) and i1["tau"] == i2["tau"]
    assert i1["recall"] >= 0.99
    # the trained network's loss, by the oracle, is the loss the run reports having reached
    rl, _ = oracle.mlp_loss_grad(feat.astype(np.float64), label.astype(np.float64),
                                 P1.cpu().numpy().astype(np.float64), H)
    assert rl < i1["loss_first"]


def c5_problem(seed, n=800, p=4000):
    rec = datagen.RECIPES["c5"].scaled(n=n, p=p, seed=seed)
    prob = datagen.make(rec)
    return rec, prob.Xt, prob.y[0]


def test_records_follow_their_definition(gpu_ctx):
    """Training records of an SSR path: features from the path's own |z|/lambda history, label = active."""
    rec, Xt, y = c5_problem(1105, n=300, p=2000)
    K = 30
    cap = 200000
    feat = torch.zeros((cap, 4), dtype=torch.float32, device=DEV)
    lab = torch.zeros(cap, dtype=torch.float32, device=DEV)
    res = bl.fit_path(gpu_ctx, to_dev(Xt), to_dev(y), nlambda=K, lambda_min_ratio=rec.lambda_min_ratio, tol=1e-10,
                      rec_feat=feat, rec_label=lab)
    n = res.n_recorded
    assert n > 0
    f = feat[:n].cpu().numpy()
    lb = lab[:n].cpu().numpy()
    beta = res.beta.cpu().numpy()
    lam = res.lam
    # rebuild the records from the oracle's path (same lambda grid, same definition)
    X64 = Xt.astype(np.float64)
    ref = oracle.fit_path(X64, y, K=K, ratio=rec.lambda_min_ratio, tol=1e-13)
    c, s, keep, nn = oracle.standardize(X64)
    ybar, yt, a, lmax, jstar = oracle.lambda_max(X64, c, s, keep, y)
    bb = oracle.bedpp_b(X64, c, s, keep, jstar)
    sign, v = np.sign(a[jstar]), float(yt @ yt) / nn

    def safe(lv):
        return keep & ~oracle.bedpp_discard(a, bb, keep, lmax, sign, v, lv)

    # z at lambda_m is known on the columns the path scanned there: every kept column at lambda_max,
    # the BEDPP survivors of the next lambda afterwards
    z = []
    for k in range(K):
        zk = oracle.zscan(X64, c, s, keep, oracle.residual(X64, c, s, yt, ref.beta[k]), None)
        seen = keep if k == 0 else safe(lam[min(k + 1, K - 1)])
        z.append(np.where(seen, zk, 0.0))
    rows, labels = [], []
    for k in range(3, K):
        strong = safe(lam[k]) & ((np.abs(z[k - 1]) >= 2 * lam[k] - lam[k - 1]) | (ref.beta[k - 1] != 0))
        candj = np.flatnonzero(strong & (ref.beta[k - 1] == 0))
        for j in candj:
            rows.append([abs(z[k - i][j]) / lam[k - i] for i in (1, 2, 3)] + [lam[k] / lam[k - 1]])
            labels.append(1.0 if ref.beta[k][j] != 0 else 0.0)
    rows = np.array(rows)
    print(f"{n} records, {len(rows)} rebuilt; positives {lb.sum():.0f} vs {sum(labels):.0f}")
    # the features are FP32 and the two paths stop at different tolerances: the candidate sets agree
    # except for features within rounding of the strong-rule threshold
    assert abs(n - len(rows)) <= max(2, 0.002 * len(rows))
    if n == len(rows):
        np.testing.assert_array_equal(lb, np.array(labels, dtype=np.float32))
        np.testing.assert_allclose(f[:, :3], rows[:, :3], rtol=1e-5, atol=1e-6)
        np.testing.assert_allclose(f[:, 3], rows[:, 3], rtol=1e-6)
    assert np.abs(beta - ref.beta).max() <= 1e-6


RATIO = 0.1   # the block-AR(1) problems below stay well short of n active features at this depth


@pytest.fixture(scope="module")
def trained(gpu_ctx):
    """Network trained on records of strong-rule paths over 20 block-AR(1) problems."""
    K = 50
    cap = 4_000_000
    feat = torch.zeros((cap, 4), dtype=torch.float32, device=DEV)
    lab = torch.zeros(cap, dtype=torch.float32, device=DEV)
    n = 0
    for t in range(20):
        rec, Xt, y = c5_problem(2000 + t)
        r = bl.fit_path(gpu_ctx, to_dev(Xt), to_dev(y), nlambda=K, lambda_min_ratio=RATIO, tol=1e-10,
                        rec_feat=feat[n:], rec_label=lab[n:])
        n += r.n_recorded
        print(f"training path {t}: {r.time_ms:.0f} ms, {r.n_recorded} records", flush=True)
    P = to_dev(bl.mlp_init(1))
    info = bl.mlp_train(gpu_ctx, feat[:n].contiguous(), lab[:n].contiguous(), P, epochs=30, batch=4096, lr=2e-3,
                        seed=5, target_recall=0.995)
    info["records"] = n
    info["positives"] = float(lab[:n].sum())
    print("training:", info)
    return P, info, K


def test_learned_path_matches_oracle_and_shrinks_working_sets(gpu_ctx, trained):
    P, info, K = trained
    assert info["loss_last"] < info["loss_first"]
    tot_l = tot_s = viol_l = 0
    for t in range(3):
        rec, Xt, y = c5_problem(3000 + t)
        Xd, yd = to_dev(Xt), to_dev(y)
        kw = dict(nlambda=K, lambda_min_ratio=RATIO, tol=1e-10)
        lr = bl.fit_path(gpu_ctx, Xd, yd, rule=bl.SCREEN_LEARNED, mlp=P, mlp_tau=info["tau"], **kw)
        sr = bl.fit_path(gpu_ctx, Xd, yd, rule=bl.SCREEN_SSR_BEDPP, **kw)
        ref = oracle.fit_path(Xt.astype(np.float64), y, K=K, ratio=RATIO, tol=1e-13)
        assert lr.k_done == K
        assert np.abs(lr.beta.cpu().numpy() - ref.beta).max() <= 1e-6
        assert np.abs((lr.obj - ref.obj) / ref.obj).max() <= 1e-8
        np.testing.assert_array_equal(lr.n_active, ref.n_active)
        print(f"problem {t}: working sets learned {lr.n_strong.sum()} vs strong rule {sr.n_strong.sum()}, "
              f"violations {lr.n_viol.sum()} vs {sr.n_viol.sum()}, rounds {lr.rounds.sum()} vs {sr.rounds.sum()}, "
              f"sweeps {lr.sweeps.sum()} vs {sr.sweeps.sum()}")
        tot_l += lr.n_strong.sum()
        tot_s += sr.n_strong.sum()
        viol_l += lr.n_viol.sum()
    # the gain: smaller working sets for the same solutions
    assert tot_l < tot_s


def test_learned_rule_rejects_missing_network(gpu_ctx):
    rec, Xt, y = c5_problem(7, n=100, p=300)
    with pytest.raises(bl.BLError) as e:
        bl.fit_path(gpu_ctx, to_dev(Xt), to_dev(y), nlambda=10, rule=bl.SCREEN_LEARNED)
    assert e.value.status == bl.BL_ERR_INVALID
