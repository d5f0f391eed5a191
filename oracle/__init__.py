"""Python access to the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg.  The GPU library never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c: plain FP64, no FMA contraction, no fast-math, OpenMP on column scans."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-fopenmp",
               "-std=c99", os.path.join(_HERE, "oracle.c"), "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class _Stats(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in
                ("sweeps", "n_strong", "n_viol", "n_rounds", "n_safe", "n_active", "rss", "obj", "gap")]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        i64, dbl, vp, i32 = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int
        L.or_num_threads.argtypes = []
        L.or_num_threads.restype = i32
        L.or_set_threads.argtypes = [i32]
        L.or_set_threads.restype = None
        L.or_standardize.argtypes = [i64, i64, vp, i64, vp, vp, vp, vp]
        L.or_standardize.restype = i64
        L.or_zscan.argtypes = [i64, i64, vp, i64, vp, vp, vp, vp, vp, vp]
        L.or_zscan.restype = None
        L.or_lambda_max.argtypes = [i64, i64, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        L.or_lambda_max.restype = i32
        L.or_bedpp_b.argtypes = [i64, i64, vp, i64, vp, vp, vp, vp, i64, vp]
        L.or_bedpp_b.restype = None
        L.or_bedpp_discard.argtypes = [i64, vp, vp, vp, dbl, dbl, dbl, dbl, vp]
        L.or_bedpp_discard.restype = i64
        L.or_lambda_grid.argtypes = [dbl, dbl, i64, vp]
        L.or_lambda_grid.restype = None
        L.or_cd.argtypes = [i64, i64, vp, i64, vp, vp, vp, dbl, vp, i64, vp, vp, dbl, i64, vp]
        L.or_cd.restype = i32
        L.or_residual.argtypes = [i64, i64, vp, i64, vp, vp, vp, vp, vp, vp]
        L.or_residual.restype = None
        L.or_cd_enet.argtypes = [i64, i64, vp, i64, vp, vp, vp, dbl, dbl, vp, vp, i64, vp, vp, dbl, i64, vp]
        L.or_cd_enet.restype = i32
        L.or_objective_enet.argtypes = [i64, vp, vp, i64, vp, dbl, dbl, vp]
        L.or_objective_enet.restype = dbl
        L.or_duality_gap_enet.argtypes = [i64, i64, vp, i64, vp, vp, vp, vp, vp, vp, vp, dbl, dbl, vp]
        L.or_duality_gap_enet.restype = dbl
        L.or_fit_path_enet.argtypes = [i64, i64, vp, i64, vp, vp, i64, dbl, vp, dbl, vp, i32, dbl, i64,
                                       vp, vp, vp, vp, vp, vp, vp, vp]
        L.or_fit_path_enet.restype = i32
        L.or_logistic_objective.argtypes = [i64, vp, vp, vp, i64, vp, dbl]
        L.or_logistic_objective.restype = dbl
        L.or_logistic_gap.argtypes = [i64, i64, vp, i64, vp, vp, vp, vp, vp, vp, vp, dbl]
        L.or_logistic_gap.restype = dbl
        L.or_logistic_safe_threshold.argtypes = [i64, i64, dbl, dbl]
        L.or_logistic_safe_threshold.restype = dbl
        L.or_logistic_discard.argtypes = [i64, vp, vp, dbl, vp]
        L.or_logistic_discard.restype = i64
        L.or_fit_path_logistic.argtypes = [i64, i64, vp, i64, vp, vp, i64, dbl, i32, dbl, i64,
                                           vp, vp, vp, vp, vp, vp, vp, vp]
        L.or_fit_path_logistic.restype = i32
        L.or_objective.argtypes = [i64, vp, vp, i64, vp, dbl]
        L.or_objective.restype = dbl
        L.or_duality_gap.argtypes = [i64, i64, vp, i64, vp, vp, vp, vp, vp, vp, vp, dbl]
        L.or_duality_gap.restype = dbl
        L.or_fit_path.argtypes = [i64, i64, vp, i64, vp, vp, i64, dbl, vp, i32, dbl, i64,
                                  vp, vp, vp, vp, vp, vp, ctypes.POINTER(_Stats), vp]
        L.or_fit_path.restype = i32
        L.or_mlp_forward.argtypes = [i64, i64, vp, vp, vp]
        L.or_mlp_forward.restype = None
        L.or_mlp_loss_grad.argtypes = [i64, i64, vp, vp, vp, vp]
        L.or_mlp_loss_grad.restype = dbl
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a):
    return None if a is None else a.ctypes.data


def _design(Xt):
    """Accept X as a (p, n) array (row j = column j); returns float64 (p, ld) and ld."""
    Xt = _f64(Xt)
    return Xt, Xt.shape[1]


def _mask(mask, n_total):
    if mask is None:
        return None
    m = np.ascontiguousarray(mask, dtype=np.uint8)
    assert m.shape == (n_total,)
    return m


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_threads(t: int) -> None:
    """Thread count of the oracle's OpenMP column scans."""
    _load().or_set_threads(int(t))


def standardize(Xt, mask=None):
    Xt, ld = _design(Xt)
    p, n_total = Xt.shape
    m = _mask(mask, n_total)
    c = np.empty(p)
    s = np.empty(p)
    keep = np.empty(p, dtype=np.uint8)
    n = _load().or_standardize(n_total, p, _ptr(Xt), ld, _ptr(m), _ptr(c), _ptr(s), _ptr(keep))
    return c, s, keep.astype(bool), n


def zscan(Xt, c, s, keep, r, mask=None):
    Xt, ld = _design(Xt)
    p, n_total = Xt.shape
    m = _mask(mask, n_total)
    c, s, r = _f64(c), _f64(s), _f64(r)
    k = np.ascontiguousarray(keep, dtype=np.uint8)
    z = np.empty(p)
    _load().or_zscan(n_total, p, _ptr(Xt), ld, _ptr(m), _ptr(c), _ptr(s), _ptr(k), _ptr(r), _ptr(z))
    return z


def lambda_max(Xt, c, s, keep, y, mask=None):
    Xt, ld = _design(Xt)
    p, n_total = Xt.shape
    m = _mask(mask, n_total)
    c, s, y = _f64(c), _f64(s), _f64(y)
    k = np.ascontiguousarray(keep, dtype=np.uint8)
    ybar = ctypes.c_double()
    lmax = ctypes.c_double()
    jstar = ctypes.c_int64()
    ytilde = np.empty(n_total)
    a = np.empty(p)
    rc = _load().or_lambda_max(n_total, p, _ptr(Xt), ld, _ptr(m), _ptr(c), _ptr(s), _ptr(k), _ptr(y),
                               ctypes.addressof(ybar), _ptr(ytilde), _ptr(a), ctypes.addressof(lmax),
                               ctypes.addressof(jstar))
    if rc:
        raise ValueError("lambda_max: no usable column or no rows")
    return ybar.value, ytilde, a, lmax.value, jstar.value


def bedpp_b(Xt, c, s, keep, jstar, mask=None):
    Xt, ld = _design(Xt)
    p, n_total = Xt.shape
    m = _mask(mask, n_total)
    c, s = _f64(c), _f64(s)
    k = np.ascontiguousarray(keep, dtype=np.uint8)
    b = np.empty(p)
    _load().or_bedpp_b(n_total, p, _ptr(Xt), ld, _ptr(m), _ptr(c), _ptr(s), _ptr(k), int(jstar), _ptr(b))
    return b


def bedpp_discard(a, b, keep, lambda_max, sign_star, v, lam):
    a, b = _f64(a), _f64(b)
    k = np.ascontiguousarray(keep, dtype=np.uint8)
    d = np.empty(a.size, dtype=np.uint8)
    _load().or_bedpp_discard(a.size, _ptr(a), _ptr(b), _ptr(k), lambda_max, sign_star, v, lam, _ptr(d))
    return d.astype(bool)


def lambda_grid(lambda_max, ratio, K):
    lam = np.empty(K)
    _load().or_lambda_grid(lambda_max, ratio, K, _ptr(lam))
    return lam


def _weights(w, p):
    if w is None:
        return None
    w = _f64(w)
    if w.shape != (p,) or np.any(~np.isfinite(w)) or np.any(w <= 0):
        raise ValueError("penalty weights must be p finite positive values")
    return w


def cd(Xt, c, s, lam, sset, beta, r, tol=1e-13, max_sweeps=100000, mask=None, alpha=1.0, penalty_factor=None):
    """Cyclic CD in place on beta and r; returns (converged, sweeps).  alpha < 1 or penalty_factor: the
    elastic-net step."""
    Xt, ld = _design(Xt)
    p, n_total = Xt.shape
    m = _mask(mask, n_total)
    c, s = _f64(c), _f64(s)
    sset = np.ascontiguousarray(sset, dtype=np.int64)
    assert beta.dtype == np.float64 and beta.flags.c_contiguous
    assert r.dtype == np.float64 and r.flags.c_contiguous
    sw = ctypes.c_int64()
    w = _weights(penalty_factor, p)
    if alpha == 1.0 and w is None:
        rc = _load().or_cd(n_total, p, _ptr(Xt), ld, _ptr(m), _ptr(c), _ptr(s), lam, _ptr(sset), sset.size,
                           _ptr(beta), _ptr(r), tol, max_sweeps, ctypes.addressof(sw))
    else:
        rc = _load().or_cd_enet(n_total, p, _ptr(Xt), ld, _ptr(m), _ptr(c), _ptr(s), lam, float(alpha), _ptr(w),
                                _ptr(sset), sset.size, _ptr(beta), _ptr(r), tol, max_sweeps, ctypes.addressof(sw))
    return rc == 0, sw.value


def residual(Xt, c, s, ytilde, beta, mask=None):
    Xt, ld = _design(Xt)
    p, n_total = Xt.shape
    m = _mask(mask, n_total)
    r = np.empty(n_total)
    _load().or_residual(n_total, p, _ptr(Xt), ld, _ptr(m), _ptr(_f64(c)), _ptr(_f64(s)), _ptr(_f64(ytilde)),
                        _ptr(_f64(beta)), _ptr(r))
    return r


def objective(r, beta, lam, mask=None, alpha=1.0, penalty_factor=None):
    r = _f64(r)
    m = _mask(mask, r.size)
    beta = _f64(beta)
    w = _weights(penalty_factor, beta.size)
    if alpha == 1.0 and w is None:
        return _load().or_objective(r.size, _ptr(m), _ptr(r), beta.size, _ptr(beta), lam)
    return _load().or_objective_enet(r.size, _ptr(m), _ptr(r), beta.size, _ptr(beta), lam, float(alpha), _ptr(w))


def duality_gap(Xt, c, s, keep, ytilde, r, beta, lam, mask=None, alpha=1.0, penalty_factor=None):
    Xt, ld = _design(Xt)
    p, n_total = Xt.shape
    m = _mask(mask, n_total)
    k = np.ascontiguousarray(keep, dtype=np.uint8)
    w = _weights(penalty_factor, p)
    if alpha == 1.0 and w is None:
        return _load().or_duality_gap(n_total, p, _ptr(Xt), ld, _ptr(m), _ptr(_f64(c)), _ptr(_f64(s)), _ptr(k),
                                      _ptr(_f64(ytilde)), _ptr(_f64(r)), _ptr(_f64(beta)), lam)
    return _load().or_duality_gap_enet(n_total, p, _ptr(Xt), ld, _ptr(m), _ptr(_f64(c)), _ptr(_f64(s)), _ptr(k),
                                       _ptr(_f64(ytilde)), _ptr(_f64(r)), _ptr(_f64(beta)), lam, float(alpha),
                                       _ptr(w))


@dataclass
class Path:
    lam: np.ndarray        # (K,)
    beta: np.ndarray       # (K, p) standardized scale
    c: np.ndarray
    s: np.ndarray
    keep: np.ndarray
    ybar: float
    sweeps: np.ndarray
    n_strong: np.ndarray
    n_viol: np.ndarray
    n_rounds: np.ndarray
    n_safe: np.ndarray
    n_active: np.ndarray
    rss: np.ndarray
    obj: np.ndarray
    gap: np.ndarray
    k_done: int
    status: int

    def original_scale(self):
        """Coefficients beta_j / s_j and intercept ybar - sum_j c_j beta_j / s_j, per lambda."""
        s = np.where(self.keep, self.s, 1.0)
        b = np.where(self.keep[None, :], self.beta / s[None, :], 0.0)
        icpt = self.ybar - b @ self.c
        return icpt, b


SCREEN_NONE, SCREEN_SSR, SCREEN_ACTIVE = 0, 1, 2


def fit_path(Xt, y, K=100, ratio=0.1, screen=SCREEN_SSR, tol=1e-13, max_sweeps=100000, mask=None,
             lambdas=None, alpha=1.0, penalty_factor=None) -> Path:
    """The path over the geometric grid from lambda_max, or over the decreasing grid `lambdas` (K values).
    alpha < 1 and/or penalty_factor (p positive weights): the elastic net with feature weights."""
    Xt, ld = _design(Xt)
    lam_in = None
    if lambdas is not None:
        lam_in = _f64(lambdas)
        if lam_in.size != K or np.any(np.diff(lam_in) > 0) or np.any(lam_in <= 0):
            raise ValueError("lambdas must hold K positive non-increasing values")
    p, n_total = Xt.shape
    m = _mask(mask, n_total)
    y = _f64(y)
    c, s = np.empty(p), np.empty(p)
    keep = np.empty(p, dtype=np.uint8)
    lam = np.empty(K)
    beta = np.zeros((K, p))
    ybar = ctypes.c_double()
    arr = {k: np.zeros(K, dtype=np.int64) for k in ("sweeps", "n_strong", "n_viol", "n_rounds", "n_safe", "n_active")}
    arr.update({k: np.zeros(K) for k in ("rss", "obj", "gap")})
    st = _Stats(**{k: v.ctypes.data for k, v in arr.items()})
    k_done = ctypes.c_int64()
    w = _weights(penalty_factor, p)
    rc = _load().or_fit_path_enet(n_total, p, _ptr(Xt), ld, _ptr(m), _ptr(y), K, ratio, _ptr(lam_in),
                                  float(alpha), _ptr(w), screen, tol, max_sweeps,
                             _ptr(c), _ptr(s), _ptr(keep), _ptr(lam), _ptr(beta), ctypes.addressof(ybar),
                             ctypes.byref(st), ctypes.addressof(k_done))
    if rc == 2:
        raise ValueError("fit_path: bad input")
    return Path(lam, beta, c, s, keep.astype(bool), ybar.value, k_done=k_done.value, status=rc, **arr)


def n_params(H):
    return H * H + 7 * H + 1


def mlp_forward(feat, params, H):
    feat = _f64(feat).reshape(-1, 4)
    params = _f64(params)
    assert params.size == n_params(H)
    prob = np.empty(feat.shape[0])
    _load().or_mlp_forward(feat.shape[0], H, _ptr(feat), _ptr(params), _ptr(prob))
    return prob


def mlp_loss_grad(feat, label, params, H):
    feat = _f64(feat).reshape(-1, 4)
    label = _f64(label)
    params = _f64(params)
    grad = np.empty_like(params)
    loss = _load().or_mlp_loss_grad(feat.shape[0], H, _ptr(feat), _ptr(label), _ptr(params), _ptr(grad))
    return loss, grad


# ---- cross-validation (Section 3.1.2; Section 5.2 shows its curve, lambda.min and the error there) ----

@dataclass
class CV:
    lam: np.ndarray        # (K,) the full-data grid every fold is fitted on
    pred: np.ndarray       # (K, n_total) prediction of each row by the model of its own fold (rows in no fold: 0)
    loss: np.ndarray       # (K, N) squared errors of the N rows that belong to a fold, in row order
    cve: np.ndarray        # (K,) mean of loss over the N rows
    cvse: np.ndarray       # (K,) standard error of that mean
    fold_err: np.ndarray   # (nfolds, K) mean squared error over the rows of each fold
    k_min: int
    k_1se: int
    paths: list            # the fold paths (Path)


def cv_summary(loss):
    """cve = mean over rows, cvse = sample SD over rows / sqrt(N), k_min = first smallest cve, k_1se = the
    smallest k (largest lambda) with cve[k] <= cve[k_min] + cvse[k_min]."""
    loss = np.asarray(loss, dtype=np.float64)
    N = loss.shape[1]
    cve = loss.mean(axis=1)
    cvse = loss.std(axis=1, ddof=1) / np.sqrt(N) if N > 1 else np.zeros(loss.shape[0])
    k_min = int(np.argmin(cve))
    k_1se = int(np.flatnonzero(cve <= cve[k_min] + cvse[k_min])[0])
    return cve, cvse, k_min, k_1se


def cv_path(Xt, y, fold, nfolds, K=100, ratio=0.1, tol=1e-13) -> CV:
    """K-fold cross-validation of the lasso path.  The grid comes from the full data's lambda_max; fold f is
    fitted on the rows with fold != f (a row mask, X is not copied) over that grid and predicts the rows with
    fold == f on the original scale: y^_i = intercept + sum_j x_ij beta_j / s_j.  Rows with fold < 0 are in
    no fold (neither fitted nor predicted)."""
    Xt, ld = _design(Xt)
    p, n_total = Xt.shape
    fold = np.asarray(fold, dtype=np.int64)
    y = _f64(y)
    inrows = fold >= 0
    c, s, keep, n = standardize(Xt, inrows.astype(np.uint8))
    ybar, yt, a, lmax, js = lambda_max(Xt, c, s, keep, y, inrows.astype(np.uint8))
    lam = lambda_grid(lmax, ratio, K)
    pred = np.zeros((K, n_total))
    fold_err = np.zeros((nfolds, K))
    paths = []
    for f in range(nfolds):
        train = (inrows & (fold != f)).astype(np.uint8)
        test = fold == f
        path = fit_path(Xt, y, K=K, ratio=ratio, tol=tol, mask=train, lambdas=lam)
        if path.k_done != K:
            raise RuntimeError(f"fold {f}: the oracle path stopped at {path.k_done}")
        icpt, b = path.original_scale()
        pred[:, test] = icpt[:, None] + b @ Xt[:, test]
        fold_err[f] = np.mean((y[test][None, :] - pred[:, test]) ** 2, axis=1)
        paths.append(path)
    loss = (y[inrows][None, :] - pred[:, inrows]) ** 2
    cve, cvse, k_min, k_1se = cv_summary(loss)
    return CV(lam, pred, loss, cve, cvse, fold_err, k_min, k_1se, paths)


# ---- lasso-penalized logistic regression (y in {0, 1}) ----

@dataclass
class LogisticPath:
    lam: np.ndarray
    beta: np.ndarray       # (K, p) standardized scale
    b0: np.ndarray         # (K,) intercept on the standardized scale
    c: np.ndarray
    s: np.ndarray
    keep: np.ndarray
    sweeps: np.ndarray
    n_strong: np.ndarray
    n_viol: np.ndarray
    n_rounds: np.ndarray
    n_safe: np.ndarray
    n_active: np.ndarray
    obj: np.ndarray
    gap: np.ndarray
    k_done: int
    status: int

    def original_scale(self):
        s = np.where(self.keep, self.s, 1.0)
        b = np.where(self.keep[None, :], self.beta / s[None, :], 0.0)
        return self.b0 - b @ self.c, b


def fit_path_logistic(Xt, y, K=100, ratio=0.1, screen=SCREEN_SSR, tol=1e-12, max_iter=100000, mask=None
                      ) -> LogisticPath:
    Xt, ld = _design(Xt)
    p, n_total = Xt.shape
    m = _mask(mask, n_total)
    y = _f64(y)
    c, s = np.empty(p), np.empty(p)
    keep = np.empty(p, dtype=np.uint8)
    lam = np.empty(K)
    beta = np.zeros((K, p))
    b0 = np.zeros(K)
    arr = {k: np.zeros(K, dtype=np.int64) for k in ("sweeps", "n_strong", "n_viol", "n_rounds", "n_safe", "n_active")}
    arr.update({k: np.zeros(K) for k in ("rss", "obj", "gap")})
    st = _Stats(**{k: v.ctypes.data for k, v in arr.items()})
    k_done = ctypes.c_int64()
    rc = _load().or_fit_path_logistic(n_total, p, _ptr(Xt), ld, _ptr(m), _ptr(y), K, ratio, screen, tol, max_iter,
                                      _ptr(c), _ptr(s), _ptr(keep), _ptr(lam), _ptr(beta), _ptr(b0),
                                      ctypes.byref(st), ctypes.addressof(k_done))
    if rc == 2:
        raise ValueError("fit_path_logistic: bad input")
    arr.pop("rss")
    return LogisticPath(lam, beta, b0, c, s, keep.astype(bool), k_done=k_done.value, status=rc, **arr)


def logistic_objective(y, eta, beta, lam, mask=None):
    y, eta, beta = _f64(y), _f64(eta), _f64(beta)
    m = _mask(mask, y.size)
    return _load().or_logistic_objective(y.size, _ptr(m), _ptr(y), _ptr(eta), beta.size, _ptr(beta), lam)


def logistic_gap(Xt, c, s, keep, y, eta, beta, lam, mask=None):
    Xt, ld = _design(Xt)
    p, n_total = Xt.shape
    m = _mask(mask, n_total)
    k = np.ascontiguousarray(keep, dtype=np.uint8)
    return _load().or_logistic_gap(n_total, p, _ptr(Xt), ld, _ptr(m), _ptr(_f64(c)), _ptr(_f64(s)), _ptr(k),
                                   _ptr(_f64(y)), _ptr(_f64(eta)), _ptr(_f64(beta)), lam)


def logistic_safe_threshold(n, n1, lambda_max, lam):
    return _load().or_logistic_safe_threshold(int(n), int(n1), float(lambda_max), float(lam))
