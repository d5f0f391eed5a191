"""bl_kkt_check_noalloc, the check for callers that cannot allocate, against bl_kkt_check.

Two calls in a row, the second on a smaller problem (fewer columns and rows, a row mask), each compared
element by element with bl_kkt_check on the same inputs: z over the checked columns bit for bit (same
kernel, same order) and the same violator list.  Sizes beyond the array's limit are refused before any
device work.
"""
import ctypes

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


def one_case(ctx, n, p, seed, masked, dt):
    prob = datagen.make("c2", n=n, p=p)
    Xh = prob.Xt.astype(dt)
    X64 = Xh.astype(np.float64)
    rng = np.random.default_rng(seed)
    mask = (rng.uniform(size=n) < 0.8).astype(np.uint8) if masked else None
    c, s, keep, nn = oracle.standardize(X64, mask)
    r = rng.normal(size=n) + 0.1
    if mask is not None:
        r[mask == 0] = 0.0
    oz = oracle.zscan(X64, c, s, keep, r, mask)
    kept = np.flatnonzero(keep)
    check = kept[rng.uniform(size=kept.size) < 0.7].astype(np.int32)
    excl = np.zeros(p, dtype=np.uint8)
    excl[check[::7]] = 1
    lam = float(np.quantile(np.abs(oz[check]), 0.8))
    Xd, cd, sd, rd = to_dev(Xh), to_dev(c), to_dev(s), to_dev(r)
    md = to_dev(mask) if masked else None
    ck, ex = to_dev(check), to_dev(excl)
    z_ref, viol_ref = bl.kkt_check(ctx, Xd, cd, sd, rd, lam, ck, exclude=ex, row_mask=md)
    z = torch.full((p,), 7.0, dtype=torch.float64, device=DEV)
    z[ck.long()] = 0.0
    viol = torch.full((max(1, check.size),), -1, dtype=torch.int32, device=DEV)
    nv = bl.kkt_check_noalloc(ctx, Xd, cd, sd, rd, lam, ck, z, viol, exclude=ex, row_mask=md)
    assert nv == viol_ref.numel()
    assert torch.equal(viol[:nv], viol_ref)
    assert torch.equal(z[ck.long()], z_ref[ck.long()])
    # columns outside the checked set are left untouched
    outside = np.setdiff1d(np.arange(p), check)
    assert torch.all(z[to_dev(outside).long()] == 7.0)
    # and both agree with the oracle
    np.testing.assert_allclose(z.cpu().numpy()[check], oz[check], atol=1e-12 * np.abs(oz).max())
    print(f"n={n} p={p} masked={masked}: {nv} violators", flush=True)
    return nv


def test_noalloc_check_matches_check_twice_second_smaller(gpu_ctx):
    nv1 = one_case(gpu_ctx, 1500, 6000, 1, False, np.float64)
    nv2 = one_case(gpu_ctx, 900, 2500, 2, True, np.float32)
    assert nv1 > 0 and nv2 > 0


def test_noalloc_check_refuses_sizes_beyond_its_array(gpu_ctx):
    x = torch.zeros((4, 16), dtype=torch.float64, device=DEV)
    M = bl._Matrix(ctypes.c_void_p(x.data_ptr()), bl.X_F64, 16, bl.NOALLOC_MAX_P + 1, 16, None)
    v = torch.zeros(16, dtype=torch.float64, device=DEV)
    cols = torch.zeros(1, dtype=torch.int32, device=DEV)
    viol = torch.zeros(1, dtype=torch.int32, device=DEV)
    nv = ctypes.c_int64()
    L = bl.load_library()
    st = L.bl_kkt_check_noalloc(gpu_ctx.handle, ctypes.byref(M), ctypes.c_void_p(v.data_ptr()),
                                ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(v.data_ptr()), 1.0,
                                ctypes.c_void_p(cols.data_ptr()), 1, None, ctypes.c_void_p(v.data_ptr()),
                                ctypes.c_void_p(viol.data_ptr()), ctypes.byref(nv))
    assert st == bl.BL_ERR_UNSUPPORTED
    assert b"BL_NOALLOC_MAX_P" in L.bl_last_error(gpu_ctx.handle)
