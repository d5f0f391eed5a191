#!/usr/bin/env python3
"""Throughput of whole lasso paths on one GPU, plus the scan kernel against the HBM roofline.

One step = one full call of bl_fit_path: standardization, lambda_max, BEDPP
set-up, then 100 lambda values of screening, coordinate descent and
post-convergence checks, with X already resident in HBM.

Default workload: genotype design 5,000 x 500,000 (codes {0,1,2} from
Binomial(2, maf), maf ~ U(0.05, 0.5)) stored as FP64 (20 GB), 100 nonzero
coefficients ~ N(0,1), SNR 1, 100 lambda values down to 0.05 lambda_max,
hybrid BEDPP + strong-rule screening, CD tolerance 1e-8 (max |d beta| ~1e-8
against the FP64 oracle at tolerance 1e-13 on a reduced copy of this design).

Prints one JSON line (rank 0, N = 1).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "100-λ lasso paths/sec + XᵀR scan HBM GB/s vs plain GPU at stated error"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(Xt_u8, y, rec, cols, tol):
    """The FP64 oracle, as it is, on a column sample of the same design (bounded CPU work)."""
    import numpy as np

    import oracle

    p = Xt_u8.shape[0]
    stride = max(1, p // cols)
    sample = Xt_u8[::stride][:cols].astype(np.float64)
    t = time.perf_counter()
    path = oracle.fit_path(sample, y, K=rec.nlambda, ratio=rec.lambda_min_ratio, tol=tol)
    dt = time.perf_counter() - t
    return {
        "value": 1.0 / dt,
        "unit": "paths/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"full {rec.nlambda}-lambda path of the FP64 oracle (OpenMP column scans) on every "
                   f"{stride}th column ({sample.shape[0]} of {p} columns, all {sample.shape[1]} rows, same y, "
                   f"tol {tol:g}); {dt:.1f} s per path; a linear-in-p extrapolation to all columns would be "
                   f"{1.0 / (dt * p / sample.shape[0]):.3g} paths/s"),
        "k_done": int(path.k_done),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--cpu-cols", type=int, default=20000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the column-sharded design is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import datagen
    import paper_1701_05936_amd as bl

    rec = datagen.RECIPES[args.workload]
    t = time.perf_counter()
    Xt = datagen.design(rec)
    y = datagen.response(rec, Xt, 0)
    log(f"generated {rec.name} X {Xt.shape[1]}x{Xt.shape[0]} {Xt.dtype} in {time.perf_counter() - t:.1f} s")

    dev = torch.device("cuda", 0)
    storage = {"f64": torch.float64, "f32": torch.float32, "i8": torch.int8}[rec.storage]
    Xd = torch.from_numpy(Xt).to(dev)
    if Xd.dtype != storage:
        Xd = Xd.to(storage)
    yd = torch.from_numpy(y).to(dev)
    torch.cuda.synchronize()
    es = Xd.element_size()
    log(f"X resident on GPU: {Xd.numel() * es / 1e9:.1f} GB as {storage}")

    ctx = bl.Context(0)
    n_cu, name = ctx.device_info()
    kw = dict(nlambda=rec.nlambda, lambda_min_ratio=rec.lambda_min_ratio, rule=bl.SCREEN_SSR_BEDPP, tol=args.tol)
    for i in range(args.warmup):
        r = bl.fit_path(ctx, Xd, yd, **kw)
        log(f"warmup {i}: {r.time_ms:.0f} ms, active at the end {r.n_active[-1]}, sweeps {int(r.sweeps.sum())}")

    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(args.steps):
        results.append(bl.fit_path(ctx, Xd, yd, **kw))
        log(f"step {i}: {results[-1].time_ms:.0f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {k: ctx.profile_get(v) for k, v in (("scan", bl.PROF_SCAN), ("cd", bl.PROF_CD),
                                               ("colstats", bl.PROF_COLSTATS))}
    ctx.profile(False)

    kernels = {}
    for k, v in prof.items():
        if v["launches"]:
            kernels[k] = {"launches": v["launches"], "avg_ms": v["total_ms"] / v["launches"],
                          "share_of_step": v["total_ms"] / (elapsed * 1e3),
                          "GB_per_launch": v["bytes"] / v["launches"] / 1e9,
                          "GBs": v["bytes"] / (v["total_ms"] * 1e-3) / 1e9}
    sc = kernels["scan"]
    roofline = {"bound": "hbm", "achieved": sc["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": sc["GBs"] / HBM_PEAK_GBS, "traffic": None, "kernel": "k_scan (FP64 X)",
                "avg_launch_ms": sc["avg_ms"], "GB_per_launch": sc["GB_per_launch"]}
    last = results[-1]
    value = args.steps / elapsed
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{rec.name}: genotype X {rec.n}x{rec.p} stored {rec.storage}, "
                               f"{rec.nlambda} lambda to {rec.lambda_min_ratio} lambda_max, SSR-BEDPP, "
                               f"CD tol {args.tol:g}",
                   "n": rec.n, "p": rec.p, "nlambda": rec.nlambda, "device": name, "cu": n_cu},
        "roofline": roofline,
        "kernels": kernels,
        "path": {"n_active_last": int(last.n_active[-1]), "sweeps": int(last.sweeps.sum()),
                 "columns_scanned": int(last.n_scanned.sum()), "violations": int(last.n_viol.sum())},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a column sample) ...")
        out["cpu_baseline"] = cpu_baseline(Xt, y, rec, args.cpu_cols, args.tol)
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
