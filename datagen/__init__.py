"""Seeded synthetic lasso problems (inputs only: X, y, row subsets).

Nothing here computes any part of the lasso method.  The CPU oracle and the
GPU library both take their inputs from this module, so the two sides read
identical bytes.

Design matrices are drawn by the counter-based generator in ``gen.c`` (one
stream per column, so a column can be regenerated alone).  Coefficient
supports, values, noise and CV folds come from numpy's PCG64 generator with a
fixed seed sequence.

The workload recipes stand in for the paper's data sets (its simulated
designs of Section 4 and the genome-wide association data of Section 6, which
are not available): i.i.d. Gaussian designs, genotype codes {0,1,2} drawn as
Binomial(2, maf_j), and AR(1)-correlated designs.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libdatagen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c into libdatagen.so (gcc, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c99",
               os.path.join(_HERE, "gen.c"), "-o", _LIB_PATH + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        u64, i64, dbl = ctypes.c_uint64, ctypes.c_int64, ctypes.c_double
        vp = ctypes.c_void_p
        lib.dg_unif.argtypes = [u64, u64, u64]
        lib.dg_unif.restype = dbl
        lib.dg_normal.argtypes = [u64, u64, u64]
        lib.dg_normal.restype = dbl
        lib.dg_gaussian_f64.argtypes = [u64, i64, i64, i64, vp, i64]
        lib.dg_maf.argtypes = [u64, i64, i64, dbl, dbl, vp]
        lib.dg_genotype_u8.argtypes = [u64, i64, i64, i64, vp, vp, i64]
        lib.dg_ar1_f32.argtypes = [u64, i64, i64, dbl, i64, vp, i64]
        for f in (lib.dg_gaussian_f64, lib.dg_maf, lib.dg_genotype_u8, lib.dg_ar1_f32):
            f.restype = None
        _lib = lib
    return _lib


def unif(seed: int, stream: int, ctr: int) -> float:
    return _load().dg_unif(seed, stream, ctr)


def normal(seed: int, stream: int, ctr: int) -> float:
    return _load().dg_normal(seed, stream, ctr)


# ---------------------------------------------------------------------------
# design matrices; returned as arrays of shape (p, n): row j is column j of X,
# i.e. the bytes are X in column-major order with leading dimension n.
# ---------------------------------------------------------------------------

def gaussian_f64(seed: int, n: int, p: int, j0: int = 0) -> np.ndarray:
    Xt = np.empty((p, n), dtype=np.float64)
    _load().dg_gaussian_f64(seed, n, p, j0, Xt.ctypes.data, n)
    return Xt


def maf(seed: int, p: int, lo: float = 0.05, hi: float = 0.5, j0: int = 0) -> np.ndarray:
    m = np.empty(p, dtype=np.float64)
    _load().dg_maf(seed, p, j0, lo, hi, m.ctypes.data)
    return m


def genotype_u8(seed: int, n: int, p: int, lo: float = 0.05, hi: float = 0.5, j0: int = 0) -> np.ndarray:
    m = maf(seed, p, lo, hi, j0)
    Xt = np.empty((p, n), dtype=np.uint8)
    _load().dg_genotype_u8(seed, n, p, j0, m.ctypes.data, Xt.ctypes.data, n)
    return Xt


def ar1_f32(seed: int, n: int, p: int, rho: float, block: int = 0) -> np.ndarray:
    Xt = np.empty((p, n), dtype=np.float32)
    _load().dg_ar1_f32(seed, n, p, rho, block, Xt.ctypes.data, n)
    return Xt


# ---------------------------------------------------------------------------
# workload recipes
# ---------------------------------------------------------------------------

@dataclass
class Recipe:
    name: str
    design: str            # "gaussian" | "genotype" | "ar1" | "block_ar1"
    n: int
    p: int
    seed: int
    nnz: int               # nonzeros of beta* per response
    coef: str              # "pm_unif" (+-U(0.5,1.5)) | "normal" (N(0,1))
    snr: float
    nlambda: int
    lambda_min_ratio: float
    storage: str           # dtype the GPU path stores X in
    rho: float = 0.0
    block: int = 0
    nresp: int = 1
    nsub: int = 1          # row subsets per response (batched form)
    extra: dict = field(default_factory=dict)

    def scaled(self, n: int | None = None, p: int | None = None, **kw) -> "Recipe":
        """Same recipe at a reduced shape (support sizes shrink with p if needed)."""
        d = dict(self.__dict__)
        d.update(kw)
        if n is not None:
            d["n"] = n
        if p is not None:
            d["p"] = p
            d["nnz"] = min(self.nnz, max(1, p // 10))
        return Recipe(**d)


RECIPES = {
    # plain path, i.i.d. Gaussian, the paper's simulated-design shape class
    "c1": Recipe("c1", "gaussian", 1000, 5000, 101, 20, "pm_unif", 3.0, 100, 0.1, "f64"),
    # plain path, genotype-valued design (GWAS-like), FP64 storage
    "c2": Recipe("c2", "genotype", 5000, 500_000, 102, 100, "normal", 1.0, 100, 0.05, "f64"),
    # precision form: genotype codes stored as 8-bit integers
    "c3": Recipe("c3", "genotype", 10_000, 2_000_000, 103, 200, "normal", 1.0, 100, 0.05, "i8"),
    # batched form: 32 responses x 2 CV row subsets over one AR(1) design
    "c4": Recipe("c4", "ar1", 20_000, 200_000, 104, 50, "normal", 2.0, 50, 0.1, "f32",
                 rho=0.5, nresp=32, nsub=2),
    # learned-screening form: block AR(1) design
    "c5": Recipe("c5", "block_ar1", 5000, 1_000_000, 105, 300, "pm_unif", 3.0, 100, 0.01, "f32",
                 rho=0.7, block=100),
}


def design(rec: Recipe) -> np.ndarray:
    """X of the recipe as a (p, n) array in its natural storage dtype."""
    if rec.design == "gaussian":
        return gaussian_f64(rec.seed, rec.n, rec.p)
    if rec.design == "genotype":
        return genotype_u8(rec.seed, rec.n, rec.p)
    if rec.design == "ar1":
        return ar1_f32(rec.seed, rec.n, rec.p, rec.rho, 0)
    if rec.design == "block_ar1":
        return ar1_f32(rec.seed, rec.n, rec.p, rec.rho, rec.block)
    raise ValueError(rec.design)


def coefficients(rec: Recipe, t: int = 0):
    """Support (sorted) and values of beta* for response t."""
    rng = np.random.default_rng([rec.seed, 7, t])
    if rec.design == "block_ar1" and rec.block > 0:
        nblk = rec.p // rec.block
        per = 10
        nb = max(1, rec.nnz // per)
        blocks = rng.choice(nblk, size=nb, replace=False)
        idx = []
        for b in blocks:
            pos = rng.choice(rec.block, size=min(per, rec.block), replace=False)
            idx.extend(int(b) * rec.block + pos)
        support = np.sort(np.asarray(idx, dtype=np.int64))
    else:
        support = np.sort(rng.choice(rec.p, size=rec.nnz, replace=False)).astype(np.int64)
    k = support.size
    if rec.coef == "pm_unif":
        vals = rng.uniform(0.5, 1.5, size=k) * rng.choice([-1.0, 1.0], size=k)
    elif rec.coef == "normal":
        vals = rng.standard_normal(k)
    else:
        raise ValueError(rec.coef)
    return support, vals


def response(rec: Recipe, Xt: np.ndarray, t: int = 0) -> np.ndarray:
    """y = X beta* + sigma * eps with sigma^2 = var(X beta*) / SNR (variance with divisor n)."""
    support, vals = coefficients(rec, t)
    signal = Xt[support].astype(np.float64).T @ vals
    sigma = np.sqrt(np.var(signal) / rec.snr)
    eps = np.random.default_rng([rec.seed, 11, t]).standard_normal(rec.n)
    return signal + sigma * eps


def cv_row_masks(rec: Recipe) -> np.ndarray:
    """Row masks (nresp*nsub, n) uint8 for the batched form.

    Rows are split into 10 folds by a seeded permutation.  Problem (t, s)
    leaves out fold f = (2t + s) mod 10 and, in addition, the first
    floor(|fold| * u) rows of fold f+1 with u ~ U(0,1) drawn per problem, so the
    training row counts are uneven.
    """
    rng = np.random.default_rng([rec.seed, 13])
    perm = rng.permutation(rec.n)
    folds = np.array_split(perm, 10)
    nprob = rec.nresp * rec.nsub
    masks = np.ones((nprob, rec.n), dtype=np.uint8)
    for t in range(rec.nresp):
        for s in range(rec.nsub):
            b = t * rec.nsub + s
            f = (2 * t + s) % 10
            masks[b, folds[f]] = 0
            u = rng.uniform()
            g = folds[(f + 1) % 10]
            masks[b, g[: int(np.floor(len(g) * u))]] = 0
    return masks


@dataclass
class Problem:
    recipe: Recipe
    Xt: np.ndarray          # (p, n) storage dtype
    y: np.ndarray           # (nresp, n) float64
    masks: np.ndarray | None = None   # (nprob, n) uint8 or None


def make(rec: Recipe | str, **scale) -> Problem:
    if isinstance(rec, str):
        rec = RECIPES[rec]
    if scale:
        rec = rec.scaled(**scale)
    Xt = design(rec)
    y = np.stack([response(rec, Xt, t) for t in range(rec.nresp)])
    masks = cv_row_masks(rec) if rec.nsub > 1 else None
    return Problem(rec, Xt, y, masks)


def cv_folds(n: int, nfolds: int, seed: int) -> np.ndarray:
    """Fold of each of n rows (int32 in 0..nfolds-1): a seeded permutation cut into nfolds nearly equal parts."""
    perm = np.random.default_rng([seed, 17]).permutation(n)
    fold = np.empty(n, dtype=np.int32)
    for f, part in enumerate(np.array_split(perm, nfolds)):
        fold[part] = f
    return fold
