"""Python binding of libbl.so, the gfx950 pathwise-lasso library.

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/bl.h.  PyTorch supplies device
memory and the stream.  There is no fallback: if libbl.so is missing or the
device is unavailable, the calls raise.

Matrices are passed as tensors ``Xt`` of shape (p, ld): row j holds column j
of X, so the bytes are X in column-major order with leading dimension ld.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbl.so")

BL_OK, BL_ERR_INVALID, BL_ERR_NOMEM, BL_ERR_DEVICE, BL_ERR_NOT_CONVERGED, BL_ERR_UNSUPPORTED = range(6)
X_F64, X_F32, X_I8 = 0, 1, 2
SCREEN_NONE, SCREEN_SSR, SCREEN_BEDPP, SCREEN_SSR_BEDPP, SCREEN_LEARNED, SCREEN_ACTIVE = 0, 1, 2, 3, 4, 5
PREC_FP64, PREC_BF16X3, PREC_I8X4, PREC_BF16X2 = 0, 1, 2, 3
FAMILY_GAUSSIAN, FAMILY_BINOMIAL = 0, 1

_STATUS_NAMES = {0: "BL_OK", 1: "BL_ERR_INVALID", 2: "BL_ERR_NOMEM", 3: "BL_ERR_DEVICE",
                 4: "BL_ERR_NOT_CONVERGED", 5: "BL_ERR_UNSUPPORTED"}

# exported C symbols (kept in step with include/bl.h)
EXPORTS = ("bl_create", "bl_destroy", "bl_last_error", "bl_device_info", "bl_standardize", "bl_lambda_max",
           "bl_bedpp_setup", "bl_screen", "bl_cd_solve", "bl_kkt_check", "bl_scan", "bl_fit_path",
           "bl_fit_path_batch", "bl_mlp_forward", "bl_mlp_loss_grad", "bl_mlp_train", "bl_profile", "bl_profile_get",
           "bl_get_limits", "bl_set_limits", "bl_kkt_check_noalloc", "bl_cv_fit", "bl_fit_path_host")
NOALLOC_MAX_P = 4194304
MLP_HIDDEN = 64
MLP_NPARAMS = MLP_HIDDEN * MLP_HIDDEN + 7 * MLP_HIDDEN + 1
PROF_SCAN, PROF_CD, PROF_COLSTATS, PROF_GRAM, PROF_RUPDATE, PROF_RECHECK, PROF_BSCAN, PROF_SETUP = range(8)


class BLError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class _Matrix(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("xtype", ctypes.c_int32), ("n_total", ctypes.c_int64),
                ("p", ctypes.c_int64), ("ldx", ctypes.c_int64), ("row_mask", ctypes.c_void_p)]


class _ScreenState(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int64), ("rule", ctypes.c_int32), ("a", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("keep", ctypes.c_void_p), ("active", ctypes.c_void_p), ("lambda_max", ctypes.c_double),
                ("sign_star", ctypes.c_double), ("v", ctypes.c_double)]


class _KernelProfile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("total_ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("flops", ctypes.c_double), ("units", ctypes.c_double)]


class _PathOpts(ctypes.Structure):
    _fields_ = [("nlambda", ctypes.c_int32), ("lambda_min_ratio", ctypes.c_double), ("lambda_", ctypes.c_void_p),
                ("rule", ctypes.c_int32), ("tol", ctypes.c_double), ("max_sweeps", ctypes.c_int32),
                ("max_rounds", ctypes.c_int32), ("precision", ctypes.c_int32), ("mlp", ctypes.c_void_p),
                ("mlp_tau", ctypes.c_double), ("rec_feat", ctypes.c_void_p), ("rec_label", ctypes.c_void_p),
                ("rec_cap", ctypes.c_int64), ("k_start", ctypes.c_int32), ("beta_init", ctypes.c_void_p),
                ("r_init", ctypes.c_void_p), ("r_out", ctypes.c_void_p), ("alpha", ctypes.c_double),
                ("penalty_factor", ctypes.c_void_p), ("family", ctypes.c_int32)]


class _Cv(ctypes.Structure):
    _fields_ = [("nfolds", ctypes.c_int32), ("fold", ctypes.c_void_p), ("y", ctypes.c_void_p)]


class _CvResult(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_void_p), ("fold_beta", ctypes.c_void_p), ("pred", ctypes.c_void_p),
                ("lambda_", ctypes.c_void_p), ("cve", ctypes.c_void_p), ("cvse", ctypes.c_void_p),
                ("fold_err", ctypes.c_void_p), ("k_min", ctypes.c_int32), ("k_1se", ctypes.c_int32),
                ("lambda_min", ctypes.c_double), ("lambda_1se", ctypes.c_double), ("n_rows", ctypes.c_int64),
                ("k_done", ctypes.c_int32), ("time_ms", ctypes.c_double)]


class _HostStream(ctypes.Structure):
    _fields_ = [("panel_cols", ctypes.c_int64), ("panels_streamed", ctypes.c_int64),
                ("panels_skipped", ctypes.c_int64), ("bytes_streamed", ctypes.c_double)]


class _Limits(ctypes.Structure):
    _fields_ = [("cov_max", ctypes.c_int64), ("cd_helpers", ctypes.c_int32), ("resident", ctypes.c_int32),
                ("cycle_min", ctypes.c_int64)]


class _PathResult(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_void_p), ("center", ctypes.c_void_p), ("scale", ctypes.c_void_p),
                ("keep", ctypes.c_void_p), ("lambda_", ctypes.c_void_p), ("intercept", ctypes.c_void_p),
                ("rss", ctypes.c_void_p), ("obj", ctypes.c_void_p), ("sweeps", ctypes.c_void_p),
                ("rounds", ctypes.c_void_p), ("n_active", ctypes.c_void_p), ("n_strong", ctypes.c_void_p),
                ("n_safe", ctypes.c_void_p), ("n_viol", ctypes.c_void_p), ("n_scanned", ctypes.c_void_p),
                ("n_recheck", ctypes.c_void_p), ("y_mean", ctypes.c_double), ("lambda_max", ctypes.c_double), ("jstar", ctypes.c_int64),
                ("k_done", ctypes.c_int32), ("time_ms", ctypes.c_double), ("n_recorded", ctypes.c_int64)]


class _MlpTrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int32), ("batch", ctypes.c_int32), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("target_recall", ctypes.c_double)]


class _MlpTrainResult(ctypes.Structure):
    _fields_ = [("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double), ("tau", ctypes.c_double),
                ("recall", ctypes.c_double), ("neg_pass", ctypes.c_double), ("steps", ctypes.c_int64),
                ("time_ms", ctypes.c_double)]


class _Batch(ctypes.Structure):
    _fields_ = [("nprob", ctypes.c_int32), ("Y", ctypes.c_void_p), ("masks", ctypes.c_void_p),
                ("flags", ctypes.c_int32)]


class _BatchResult(ctypes.Structure):
    _fields_ = [("beta", ctypes.c_void_p), ("lambda_", ctypes.c_void_p), ("intercept", ctypes.c_void_p),
                ("rss", ctypes.c_void_p), ("obj", ctypes.c_void_p), ("sweeps", ctypes.c_void_p),
                ("rounds", ctypes.c_void_p), ("n_active", ctypes.c_void_p), ("n_strong", ctypes.c_void_p),
                ("n_safe", ctypes.c_void_p), ("n_viol", ctypes.c_void_p), ("k_done", ctypes.c_int32),
                ("time_ms", ctypes.c_double), ("scan_cols", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libbl.so and declare the C signatures.  Raises if the library is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libbl.so not built ({path}); run paper_1701_05936_amd/build.py")
    L = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    P = ctypes.POINTER
    L.bl_create.argtypes = [P(vp), ctypes.c_int, vp]
    L.bl_destroy.argtypes = [vp]
    L.bl_destroy.restype = None
    L.bl_last_error.argtypes = [vp]
    L.bl_last_error.restype = ctypes.c_char_p
    L.bl_device_info.argtypes = [vp, P(ctypes.c_int), ctypes.c_char_p, ctypes.c_int]
    L.bl_standardize.argtypes = [vp, P(_Matrix), vp, vp, vp, P(i64)]
    L.bl_lambda_max.argtypes = [vp, P(_Matrix), vp, vp, vp, vp, vp, vp, P(dbl), P(dbl), P(i64)]
    L.bl_bedpp_setup.argtypes = [vp, P(_Matrix), vp, vp, vp, vp, i64, vp, P(dbl)]
    L.bl_screen.argtypes = [vp, P(_ScreenState), dbl, dbl, vp, vp, vp, P(i64), P(i64)]
    L.bl_cd_solve.argtypes = [vp, P(_Matrix), vp, vp, dbl, vp, i64, vp, vp, dbl, i32, P(i32)]
    L.bl_kkt_check.argtypes = [vp, P(_Matrix), vp, vp, vp, dbl, vp, i64, vp, vp, vp, P(i64)]
    L.bl_kkt_check_noalloc.argtypes = [vp, P(_Matrix), vp, vp, vp, dbl, vp, i64, vp, vp, vp, P(i64)]
    L.bl_scan.argtypes = [vp, P(_Matrix), vp, vp, vp, vp, i64, i32, vp, vp]
    L.bl_fit_path.argtypes = [vp, P(_Matrix), vp, P(_PathOpts), P(_PathResult)]
    L.bl_fit_path_batch.argtypes = [vp, P(_Matrix), P(_Batch), P(_PathOpts), P(_BatchResult)]
    L.bl_mlp_forward.argtypes = [vp, vp, i64, vp, vp]
    L.bl_mlp_loss_grad.argtypes = [vp, vp, vp, i64, vp, vp, P(dbl)]
    L.bl_mlp_train.argtypes = [vp, vp, vp, i64, vp, P(_MlpTrainOpts), P(_MlpTrainResult)]
    L.bl_profile.argtypes = [vp, ctypes.c_int]
    L.bl_profile_get.argtypes = [vp, ctypes.c_int, P(_KernelProfile)]
    L.bl_cv_fit.argtypes = [vp, P(_Matrix), P(_Cv), P(_PathOpts), P(_CvResult)]
    L.bl_fit_path_host.argtypes = [vp, P(_Matrix), vp, P(_PathOpts), P(_HostStream), P(_PathResult)]
    L.bl_get_limits.argtypes = [vp, P(_Limits)]
    L.bl_set_limits.argtypes = [vp, P(_Limits)]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("bl_destroy", "bl_last_error"):
            f.restype = ctypes.c_int
    _lib = L
    return L


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


_XTYPES = {torch.float64: X_F64, torch.float32: X_F32, torch.int8: X_I8}


def matrix(Xt: torch.Tensor, n_total: int | None = None, row_mask: torch.Tensor | None = None) -> _Matrix:
    """Descriptor of X given as a (p, ld) tensor; n_total defaults to ld."""
    if Xt.dim() != 2:
        raise ValueError("Xt must be 2-D (p, ld)")
    if Xt.dtype not in _XTYPES:
        raise TypeError(f"unsupported X dtype {Xt.dtype}")
    p, ld = Xt.shape
    n_total = ld if n_total is None else int(n_total)
    if row_mask is not None and (row_mask.dtype != torch.uint8 or row_mask.numel() != n_total):
        raise ValueError("row_mask must be uint8 with n_total entries")
    return _Matrix(_ptr(Xt), _XTYPES[Xt.dtype], n_total, p, ld, _ptr(row_mask))


class Context:
    """A library context bound to one device and the current torch stream."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None):
        L = load_library()
        torch.cuda.set_device(device)
        stream = stream or torch.cuda.current_stream(device)
        self.stream = stream
        self.device = device
        h = ctypes.c_void_p()
        st = L.bl_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream))
        if st != BL_OK:
            raise BLError(st, "bl_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            load_library().bl_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _check(self, st: int):
        if st != BL_OK:
            msg = load_library().bl_last_error(self._h).decode(errors="replace")
            raise BLError(st, msg)

    @property
    def handle(self):
        return self._h

    def profile(self, enable: bool = True):
        """Enable (and reset) or disable per-kernel event timing inside bl_fit_path."""
        self._check(load_library().bl_profile(self._h, 1 if enable else 0))

    def profile_get(self, kernel: int) -> dict:
        kp = _KernelProfile()
        self._check(load_library().bl_profile_get(self._h, kernel, ctypes.byref(kp)))
        return {"launches": kp.launches, "total_ms": kp.total_ms, "bytes": kp.bytes, "flops": kp.flops,
                "units": kp.units}

    def limits(self) -> dict:
        """Coordinate-descent limits: cov_max, cd_helpers, the resident workgroup count and cycle_min."""
        lm = _Limits()
        self._check(load_library().bl_get_limits(self._h, ctypes.byref(lm)))
        return {"cov_max": lm.cov_max, "cd_helpers": lm.cd_helpers, "resident": lm.resident,
                "cycle_min": lm.cycle_min}

    def set_limits(self, cov_max: int = 0, cd_helpers: int = -1, cycle_min: int = 0):
        """Lower (or restore) the limits; 0 / -1 keep the current value (cycle_min: 0 keeps, -1 turns
        active-set cycling off)."""
        lm = _Limits(int(cov_max), int(cd_helpers), 0, int(cycle_min))
        self._check(load_library().bl_set_limits(self._h, ctypes.byref(lm)))

    def device_info(self):
        n = ctypes.c_int()
        buf = ctypes.create_string_buffer(256)
        self._check(load_library().bl_device_info(self._h, ctypes.byref(n), buf, 256))
        return n.value, buf.value.decode()


def _dev(ctx):
    return torch.device("cuda", ctx.device)


def standardize(ctx: Context, Xt, row_mask=None, n_total=None):
    M = matrix(Xt, n_total, row_mask)
    p = M.p
    c = torch.empty(p, dtype=torch.float64, device=_dev(ctx))
    s = torch.empty_like(c)
    keep = torch.empty(p, dtype=torch.uint8, device=_dev(ctx))
    n = ctypes.c_int64()
    ctx._check(load_library().bl_standardize(ctx.handle, ctypes.byref(M), _ptr(c), _ptr(s), _ptr(keep),
                                             ctypes.byref(n)))
    return c, s, keep, n.value


def lambda_max(ctx: Context, Xt, c, s, keep, y, row_mask=None, n_total=None):
    M = matrix(Xt, n_total, row_mask)
    yt = torch.empty(M.n_total, dtype=torch.float64, device=_dev(ctx))
    a = torch.empty(M.p, dtype=torch.float64, device=_dev(ctx))
    ym, lm, js = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    ctx._check(load_library().bl_lambda_max(ctx.handle, ctypes.byref(M), _ptr(c), _ptr(s), _ptr(keep), _ptr(y),
                                            _ptr(yt), _ptr(a), ctypes.byref(ym), ctypes.byref(lm), ctypes.byref(js)))
    return ym.value, yt, a, lm.value, js.value


def bedpp_setup(ctx: Context, Xt, c, s, keep, ytilde, jstar, row_mask=None, n_total=None):
    M = matrix(Xt, n_total, row_mask)
    b = torch.empty(M.p, dtype=torch.float64, device=_dev(ctx))
    v = ctypes.c_double()
    ctx._check(load_library().bl_bedpp_setup(ctx.handle, ctypes.byref(M), _ptr(c), _ptr(s), _ptr(keep),
                                             _ptr(ytilde), int(jstar), _ptr(b), ctypes.byref(v)))
    return b, v.value


def screen(ctx: Context, rule, a, b, keep, lambda_max, sign_star, v, lam, lam_prev, z_prev, active=None):
    p = keep.numel()
    st = _ScreenState(p, rule, _ptr(a), _ptr(b), _ptr(keep), _ptr(active), lambda_max, sign_star, v)
    safe = torch.empty(p, dtype=torch.uint8, device=_dev(ctx))
    strong = torch.empty_like(safe)
    ns, ne = ctypes.c_int64(), ctypes.c_int64()
    ctx._check(load_library().bl_screen(ctx.handle, ctypes.byref(st), lam, lam_prev, _ptr(z_prev), _ptr(safe),
                                        _ptr(strong), ctypes.byref(ns), ctypes.byref(ne)))
    return safe, strong, ns.value, ne.value


def cd_solve(ctx: Context, Xt, c, s, lam, cset, beta, r, tol=1e-10, max_sweeps=100000, row_mask=None,
             n_total=None):
    """In-place cyclic CD on beta and r over the int32 index tensor cset; returns sweeps."""
    M = matrix(Xt, n_total, row_mask)
    if cset.dtype != torch.int32:
        raise TypeError("cset must be int32")
    sw = ctypes.c_int32()
    ctx._check(load_library().bl_cd_solve(ctx.handle, ctypes.byref(M), _ptr(c), _ptr(s), lam,
                                          _ptr(cset) if cset.numel() else None, cset.numel(), _ptr(beta), _ptr(r),
                                          tol, max_sweeps, ctypes.byref(sw)))
    return sw.value


def kkt_check(ctx: Context, Xt, c, s, r, lam, check_set, exclude=None, z=None, row_mask=None, n_total=None):
    """z over check_set and the ascending violators {j : !exclude[j], |z_j| > lam}."""
    M = matrix(Xt, n_total, row_mask)
    if check_set.dtype != torch.int32:
        raise TypeError("check_set must be int32")
    if z is None:
        z = torch.zeros(M.p, dtype=torch.float64, device=_dev(ctx))
    viol = torch.empty(max(1, check_set.numel()), dtype=torch.int32, device=_dev(ctx))
    nv = ctypes.c_int64()
    ctx._check(load_library().bl_kkt_check(ctx.handle, ctypes.byref(M), _ptr(c), _ptr(s), _ptr(r), lam,
                                           _ptr(check_set) if check_set.numel() else None, check_set.numel(),
                                           _ptr(exclude), _ptr(z), _ptr(viol), ctypes.byref(nv)))
    return z, viol[: nv.value]


def kkt_check_noalloc(ctx: Context, Xt, c, s, r, lam, check_set, z, viol, exclude=None, row_mask=None,
                      n_total=None):
    """The check through bl_kkt_check_noalloc, which allocates nothing: z (float64 [p]) and viol (int32, at
    least max(1, len(check_set)) entries) are the caller's.  Returns the number of violators."""
    M = matrix(Xt, n_total, row_mask)
    if check_set.dtype != torch.int32 or viol.dtype != torch.int32 or viol.numel() < max(1, check_set.numel()):
        raise ValueError("check_set and viol must be int32, viol with room for every checked column")
    nv = ctypes.c_int64()
    ctx._check(load_library().bl_kkt_check_noalloc(ctx.handle, ctypes.byref(M), _ptr(c), _ptr(s), _ptr(r), lam,
                                                   _ptr(check_set) if check_set.numel() else None,
                                                   check_set.numel(), _ptr(exclude), _ptr(z), _ptr(viol),
                                                   ctypes.byref(nv)))
    return nv.value


def scan(ctx: Context, Xt, c, s, r, cols, precision=PREC_FP64, row_mask=None, n_total=None, want_err=False):
    """z over cols (and, for the matrix-core forms, the guaranteed error bound per column)."""
    M = matrix(Xt, n_total, row_mask)
    if cols.dtype != torch.int32:
        raise TypeError("cols must be int32")
    z = torch.zeros(M.p, dtype=torch.float64, device=_dev(ctx))
    err = torch.zeros(M.p, dtype=torch.float64, device=_dev(ctx)) if want_err else None
    ctx._check(load_library().bl_scan(ctx.handle, ctypes.byref(M), _ptr(c), _ptr(s), _ptr(r),
                                      _ptr(cols) if cols.numel() else None, cols.numel(), int(precision), _ptr(z),
                                      _ptr(err)))
    return (z, err) if want_err else z


@dataclass
class PathResult:
    lam: np.ndarray
    beta: torch.Tensor | None    # (K, p) device, standardized scale
    center: torch.Tensor
    scale: torch.Tensor
    keep: torch.Tensor
    intercept: np.ndarray
    rss: np.ndarray
    obj: np.ndarray
    sweeps: np.ndarray
    rounds: np.ndarray
    n_active: np.ndarray
    n_strong: np.ndarray
    n_safe: np.ndarray
    n_viol: np.ndarray
    n_scanned: np.ndarray
    n_recheck: np.ndarray
    y_mean: float
    lambda_max: float
    jstar: int
    k_done: int
    time_ms: float
    status: int
    message: str
    n_recorded: int = 0


def fit_path(ctx: Context, Xt, y, nlambda=100, lambda_min_ratio=0.1, lambdas=None, rule=SCREEN_SSR_BEDPP,
             tol=1e-8, max_sweeps=100000, max_rounds=100, row_mask=None, n_total=None, want_beta=True,
             raise_on_error=True, precision=PREC_FP64, mlp=None, mlp_tau=0.0, rec_feat=None, rec_label=None,
             k_start=0, beta_init=None, r_init=None, r_out=None, alpha=1.0, penalty_factor=None,
             family=FAMILY_GAUSSIAN) -> PathResult:
    """Whole path.  Learned rule: rule=SCREEN_LEARNED with mlp (float32 device [MLP_NPARAMS]) and mlp_tau.
    Training records: rec_feat (float32 device [cap, 4]) and rec_label (float32 device [cap]).
    Resume: k_start >= 1 with beta_init (float64 device [p], beta at lambda index k_start - 1) and
    optionally r_init (float64 device [n_total], its residual); r_out receives the final residual.
    Elastic net: alpha in (0, 1] and penalty_factor (float64 device [p], positive) or None."""
    M = matrix(Xt, n_total, row_mask)
    return _fit_path(ctx, M, y, nlambda, lambda_min_ratio, lambdas, rule, tol, max_sweeps, max_rounds, want_beta,
                     raise_on_error, precision, mlp, mlp_tau, rec_feat, rec_label, k_start, beta_init, r_init, r_out,
                     alpha, penalty_factor, None, family)


def fit_path_host(ctx: Context, Xt, y, nlambda=100, lambda_min_ratio=0.1, lambdas=None, rule=SCREEN_SSR_BEDPP,
                  tol=1e-8, max_sweeps=100000, max_rounds=100, row_mask=None, n_total=None, want_beta=True,
                  raise_on_error=True, k_start=0, beta_init=None, r_init=None, r_out=None, alpha=1.0,
                  penalty_factor=None, panel_cols=0, precision=PREC_FP64, family=FAMILY_GAUSSIAN):
    """The path with X in host memory (bl_fit_path_host): Xt is a CPU tensor (p, ld), pinned for full PCIe
    speed; y, row_mask and the outputs are on the device.  Returns (PathResult, streaming counters)."""
    if Xt.dim() != 2 or Xt.is_cuda:
        raise ValueError("Xt must be a 2-D CPU tensor (p, ld)")
    if Xt.dtype not in _XTYPES or not Xt.is_contiguous():
        raise TypeError("Xt must be a contiguous float64, float32 or int8 tensor")
    p, ld = Xt.shape
    nt = ld if n_total is None else int(n_total)
    if row_mask is not None and (row_mask.dtype != torch.uint8 or row_mask.numel() != nt):
        raise ValueError("row_mask must be uint8 with n_total entries")
    M = _Matrix(ctypes.c_void_p(Xt.data_ptr()), _XTYPES[Xt.dtype], nt, p, ld, _ptr(row_mask))
    hs = _HostStream(int(panel_cols), 0, 0, 0.0)
    res = _fit_path(ctx, M, y, nlambda, lambda_min_ratio, lambdas, rule, tol, max_sweeps, max_rounds, want_beta,
                    raise_on_error, precision, None, 0.0, None, None, k_start, beta_init, r_init, r_out, alpha,
                    penalty_factor, hs, family)
    return res, {"panel_cols": hs.panel_cols, "panels_streamed": hs.panels_streamed,
                 "panels_skipped": hs.panels_skipped, "bytes_streamed": hs.bytes_streamed}


def _fit_path(ctx, M, y, nlambda, lambda_min_ratio, lambdas, rule, tol, max_sweeps, max_rounds, want_beta,
              raise_on_error, precision, mlp, mlp_tau, rec_feat, rec_label, k_start, beta_init, r_init, r_out,
              alpha, penalty_factor, hs, family=FAMILY_GAUSSIAN) -> PathResult:
    K = int(nlambda)
    p = M.p
    dev = _dev(ctx)
    beta = torch.empty((K, p), dtype=torch.float64, device=dev) if want_beta else None
    c = torch.empty(p, dtype=torch.float64, device=dev)
    s = torch.empty_like(c)
    keep = torch.empty(p, dtype=torch.uint8, device=dev)
    host = {k: np.zeros(K) for k in ("lam", "intercept", "rss", "obj")}
    host.update({k: np.zeros(K, dtype=np.int32) for k in ("sweeps", "rounds")})
    host.update({k: np.zeros(K, dtype=np.int64) for k in ("n_active", "n_strong", "n_safe", "n_viol", "n_scanned",
                                                          "n_recheck")})
    lam_in = None
    if lambdas is not None:
        lam_in = np.ascontiguousarray(lambdas, dtype=np.float64)
        assert lam_in.size == K
    rec_cap = 0
    if rec_feat is not None:
        if rec_label is None or rec_feat.dtype != torch.float32 or rec_label.dtype != torch.float32 \
                or rec_feat.dim() != 2 or rec_feat.shape[1] != 4 or rec_label.numel() < rec_feat.shape[0]:
            raise ValueError("rec_feat (cap, 4) and rec_label (cap,) must be float32 device tensors")
        rec_cap = int(rec_feat.shape[0])
    if mlp is not None and (mlp.dtype != torch.float32 or mlp.numel() != MLP_NPARAMS):
        raise ValueError(f"mlp must be float32 with {MLP_NPARAMS} parameters")
    opts = _PathOpts(K, float(lambda_min_ratio), lam_in.ctypes.data if lam_in is not None else None, int(rule),
                     float(tol), int(max_sweeps), int(max_rounds), int(precision), _ptr(mlp), float(mlp_tau),
                     _ptr(rec_feat), _ptr(rec_label), rec_cap, int(k_start), _ptr(beta_init), _ptr(r_init),
                     _ptr(r_out), float(alpha), _ptr(penalty_factor), int(family))
    res = _PathResult(_ptr(beta), _ptr(c), _ptr(s), _ptr(keep), host["lam"].ctypes.data,
                      host["intercept"].ctypes.data, host["rss"].ctypes.data, host["obj"].ctypes.data,
                      host["sweeps"].ctypes.data, host["rounds"].ctypes.data, host["n_active"].ctypes.data,
                      host["n_strong"].ctypes.data, host["n_safe"].ctypes.data, host["n_viol"].ctypes.data,
                      host["n_scanned"].ctypes.data, host["n_recheck"].ctypes.data, 0.0, 0.0, 0, 0, 0.0, 0)
    if hs is None:
        st = load_library().bl_fit_path(ctx.handle, ctypes.byref(M), _ptr(y), ctypes.byref(opts), ctypes.byref(res))
    else:
        st = load_library().bl_fit_path_host(ctx.handle, ctypes.byref(M), _ptr(y), ctypes.byref(opts),
                                             ctypes.byref(hs), ctypes.byref(res))
    msg = load_library().bl_last_error(ctx.handle).decode(errors="replace") if st != BL_OK else ""
    if st != BL_OK and raise_on_error:
        raise BLError(st, msg)
    return PathResult(host["lam"], beta, c, s, keep, host["intercept"], host["rss"], host["obj"], host["sweeps"],
                      host["rounds"], host["n_active"], host["n_strong"], host["n_safe"], host["n_viol"],
                      host["n_scanned"], host["n_recheck"], res.y_mean, res.lambda_max, res.jstar, res.k_done, res.time_ms, st, msg,
                      res.n_recorded)


MAX_BATCH = 64


@dataclass
class BatchResult:
    lam: np.ndarray              # (B, K)
    beta: torch.Tensor | None    # (B, K, p) device, standardized scale of each problem
    intercept: np.ndarray
    rss: np.ndarray
    obj: np.ndarray
    sweeps: np.ndarray
    rounds: np.ndarray
    n_active: np.ndarray
    n_strong: np.ndarray
    n_safe: np.ndarray
    n_viol: np.ndarray
    k_done: int
    time_ms: float
    status: int
    message: str
    scan_cols: int = 0


BATCH_EAGER = 1


def fit_path_batch(ctx: Context, Xt, Y, masks=None, nlambda=100, lambda_min_ratio=0.1, rule=SCREEN_SSR_BEDPP,
                   tol=1e-8, max_sweeps=100000, max_rounds=100, n_total=None, want_beta=True,
                   raise_on_error=True, eager=False, lambdas=None, precision=PREC_FP64) -> BatchResult:
    """Batched form: B <= 64 problems over one X.  Y (B, n_total) float64 device; masks (B, n_total) uint8
    device or None (all rows in every problem)."""
    M = matrix(Xt, n_total, None)
    nt = M.n_total
    if Y.dtype != torch.float64 or Y.dim() != 2 or Y.shape[1] != nt:
        raise ValueError("Y must be float64 of shape (B, n_total)")
    B = int(Y.shape[0])
    if masks is not None and (masks.dtype != torch.uint8 or tuple(masks.shape) != (B, nt)):
        raise ValueError("masks must be uint8 of shape (B, n_total)")
    K = int(nlambda)
    p = M.p
    dev = _dev(ctx)
    beta = torch.empty((B, K, p), dtype=torch.float64, device=dev) if want_beta else None
    host = {k: np.zeros((B, K)) for k in ("lam", "intercept", "rss", "obj")}
    host.update({k: np.zeros((B, K), dtype=np.int32) for k in ("sweeps", "rounds")})
    host.update({k: np.zeros((B, K), dtype=np.int64) for k in ("n_active", "n_strong", "n_safe", "n_viol")})
    bt = _Batch(B, _ptr(Y), _ptr(masks), BATCH_EAGER if eager else 0)
    lam_in = None
    if lambdas is not None:
        lam_in = np.ascontiguousarray(lambdas, dtype=np.float64)
        assert lam_in.size == K
    opts = _PathOpts(K, float(lambda_min_ratio), lam_in.ctypes.data if lam_in is not None else None, int(rule),
                     float(tol), int(max_sweeps), int(max_rounds), int(precision))
    res = _BatchResult(_ptr(beta), *[host[k].ctypes.data for k in ("lam", "intercept", "rss", "obj", "sweeps",
                                                                  "rounds", "n_active", "n_strong", "n_safe",
                                                                  "n_viol")], 0, 0.0, 0)
    L = load_library()
    st = L.bl_fit_path_batch(ctx.handle, ctypes.byref(M), ctypes.byref(bt), ctypes.byref(opts), ctypes.byref(res))
    msg = L.bl_last_error(ctx.handle).decode(errors="replace") if st != BL_OK else ""
    if st != BL_OK and raise_on_error:
        raise BLError(st, msg)
    return BatchResult(host["lam"], beta, host["intercept"], host["rss"], host["obj"], host["sweeps"],
                       host["rounds"], host["n_active"], host["n_strong"], host["n_safe"], host["n_viol"],
                       res.k_done, res.time_ms, st, msg, res.scan_cols)


@dataclass
class CVResult:
    lam: np.ndarray              # (K,) the full-data grid
    cve: np.ndarray              # (K,) cross-validation error (mean held-out squared error)
    cvse: np.ndarray             # (K,) its standard error
    fold_err: np.ndarray         # (nfolds, K)
    k_min: int
    k_1se: int
    lambda_min: float
    lambda_1se: float
    n_rows: int
    beta: torch.Tensor | None    # (K, p) full-data path, standardized scale
    fold_beta: torch.Tensor | None   # (nfolds, K, p)
    pred: torch.Tensor | None    # (K, n_total) held-out predictions
    time_ms: float


def cv_fit(ctx: Context, Xt, y, fold, nfolds, nlambda=100, lambda_min_ratio=0.1, lambdas=None,
           rule=SCREEN_SSR_BEDPP, tol=1e-8, max_sweeps=100000, max_rounds=100, n_total=None, want_beta=True,
           want_fold_beta=True, want_pred=True) -> CVResult:
    """K-fold cross-validation (bl_cv_fit).  fold: int32 device [n_total] with values in -1..nfolds-1."""
    M = matrix(Xt, n_total, None)
    nt, p, K = M.n_total, M.p, int(nlambda)
    if fold.dtype != torch.int32 or fold.numel() != nt:
        raise ValueError("fold must be int32 with n_total entries")
    if y.dtype != torch.float64 or y.numel() != nt:
        raise ValueError("y must be float64 with n_total entries")
    dev = _dev(ctx)
    beta = torch.empty((K, p), dtype=torch.float64, device=dev) if want_beta else None
    fbeta = torch.empty((nfolds, K, p), dtype=torch.float64, device=dev) if want_fold_beta else None
    pred = torch.empty((K, nt), dtype=torch.float64, device=dev) if want_pred else None
    lam, cve, cvse = np.zeros(K), np.zeros(K), np.zeros(K)
    ferr = np.zeros((nfolds, K))
    lam_in = None
    if lambdas is not None:
        lam_in = np.ascontiguousarray(lambdas, dtype=np.float64)
        assert lam_in.size == K
    opts = _PathOpts(K, float(lambda_min_ratio), lam_in.ctypes.data if lam_in is not None else None, int(rule),
                     float(tol), int(max_sweeps), int(max_rounds), PREC_FP64)
    cvs = _Cv(int(nfolds), _ptr(fold), _ptr(y))
    res = _CvResult(_ptr(beta), _ptr(fbeta), _ptr(pred), lam.ctypes.data, cve.ctypes.data, cvse.ctypes.data,
                    ferr.ctypes.data)
    ctx._check(load_library().bl_cv_fit(ctx.handle, ctypes.byref(M), ctypes.byref(cvs), ctypes.byref(opts),
                                        ctypes.byref(res)))
    return CVResult(lam, cve, cvse, ferr, res.k_min, res.k_1se, res.lambda_min, res.lambda_1se, res.n_rows, beta,
                    fbeta, pred, res.time_ms)


# ---- screening network of the learned form ----

def mlp_init(seed: int = 0) -> np.ndarray:
    """He-initialised parameter vector (float32, layout W1[64][4], b1, W2[64][64], b2, w3, b3)."""
    rng = np.random.default_rng(seed)
    H = MLP_HIDDEN
    W1 = rng.normal(0.0, np.sqrt(2.0 / 4), size=(H, 4))
    W2 = rng.normal(0.0, np.sqrt(2.0 / H), size=(H, H))
    w3 = rng.normal(0.0, np.sqrt(1.0 / H), size=H)
    return np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), w3, np.zeros(1)]).astype(np.float32)


def _check_f32(t, name, n=None):
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32")
    if n is not None and t.numel() != n:
        raise ValueError(f"{name} must have {n} elements")


def mlp_forward(ctx: Context, feat, params):
    _check_f32(feat, "feat")
    _check_f32(params, "params", MLP_NPARAMS)
    m = feat.numel() // 4
    prob = torch.empty(m, dtype=torch.float32, device=feat.device)
    ctx._check(load_library().bl_mlp_forward(ctx.handle, _ptr(feat), m, _ptr(params), _ptr(prob)))
    return prob


def mlp_loss_grad(ctx: Context, feat, label, params):
    _check_f32(feat, "feat")
    _check_f32(label, "label")
    _check_f32(params, "params", MLP_NPARAMS)
    m = feat.numel() // 4
    grad = torch.empty(MLP_NPARAMS, dtype=torch.float32, device=feat.device)
    loss = ctypes.c_double()
    ctx._check(load_library().bl_mlp_loss_grad(ctx.handle, _ptr(feat), _ptr(label), m, _ptr(params), _ptr(grad),
                                               ctypes.byref(loss)))
    return loss.value, grad


def mlp_train(ctx: Context, feat, label, params, epochs=20, batch=4096, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
              seed=0, target_recall=0.995) -> dict:
    """Trains params (float32 device, in place); returns losses, the threshold tau and its recall."""
    _check_f32(feat, "feat")
    _check_f32(label, "label")
    _check_f32(params, "params", MLP_NPARAMS)
    m = feat.numel() // 4
    opts = _MlpTrainOpts(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps), int(seed),
                         float(target_recall))
    res = _MlpTrainResult()
    ctx._check(load_library().bl_mlp_train(ctx.handle, _ptr(feat), _ptr(label), m, _ptr(params), ctypes.byref(opts),
                                           ctypes.byref(res)))
    return {k: getattr(res, k) for k, _ in _MlpTrainResult._fields_}
