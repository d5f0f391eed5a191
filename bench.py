#!/usr/bin/env python3
"""Throughput of whole lasso paths on one GPU, plus the dominant kernel against its roofline.

One step = one full path call with X already resident in HBM: standardization,
lambda_max, BEDPP set-up, then every lambda value of screening, coordinate
descent and post-convergence checks.

Workloads (--workload):
  c2 (default)  plain path: genotype design 5,000 x 500,000 (codes {0,1,2} from
                Binomial(2, maf), maf ~ U(0.05, 0.5)) stored as FP64 (20 GB), 100
                nonzero coefficients ~ N(0,1), SNR 1, 100 lambda values down to
                0.05 lambda_max, hybrid BEDPP + strong-rule screening, CD tolerance 1e-8.
  c3            precision form: genotype 10,000 x 2,000,000 stored as int8 (20 GB),
                200 nonzeros, scans on BF16 matrix cores with FP64 decisions; the
                plain FP64-scan path on the same int8 storage is timed beside it.
  c4            batched form: AR(1) (rho 0.5) design 20,000 x 200,000 float32 (16 GB),
                64 problems = 32 responses x 2 cross-validation row subsets, 50 lambda
                values each; plain single-problem paths on a sample of the problems are
                timed beside it.

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
FP64_MFMA_PEAK_TFLOPS = 78.6
METRIC = "100-λ lasso paths/sec + XᵀR scan HBM GB/s vs plain GPU at stated error"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(Xt, y, rec, cols, tol, mask=None, what="path"):
    """The FP64 oracle, as it is, on a column sample of the same design (bounded CPU work)."""
    import numpy as np

    import oracle

    p = Xt.shape[0]
    stride = max(1, p // cols)
    sample = Xt[::stride][:cols].astype(np.float64)
    t = time.perf_counter()
    path = oracle.fit_path(sample, y, K=rec.nlambda, ratio=rec.lambda_min_ratio, tol=tol, mask=mask)
    dt = time.perf_counter() - t
    return {
        "value": 1.0 / dt,
        "unit": "paths/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"one full {rec.nlambda}-lambda {what} of the FP64 oracle (OpenMP column scans) on every "
                   f"{stride}th column ({sample.shape[0]} of {p} columns, all {sample.shape[1]} rows, same y, "
                   f"tol {tol:g}); {dt:.1f} s per path; a linear-in-p extrapolation to all columns would be "
                   f"{1.0 / (dt * p / sample.shape[0]):.3g} paths/s"),
        "k_done": int(path.k_done),
    }


def kernel_table(ctx, bl, elapsed):
    names = (("scan", bl.PROF_SCAN), ("bscan", bl.PROF_BSCAN), ("cd", bl.PROF_CD), ("colstats", bl.PROF_COLSTATS),
             ("gram", bl.PROF_GRAM), ("recheck", bl.PROF_RECHECK))
    kernels = {}
    for k, v in names:
        pr = ctx.profile_get(v)
        if pr["launches"]:
            kernels[k] = {"launches": pr["launches"], "avg_ms": pr["total_ms"] / pr["launches"],
                          "share_of_step": pr["total_ms"] / (elapsed * 1e3),
                          "GB_per_launch": pr["bytes"] / pr["launches"] / 1e9,
                          "GBs": pr["bytes"] / (pr["total_ms"] * 1e-3) / 1e9}
            if pr["flops"]:
                kernels[k]["TFLOP_per_launch"] = pr["flops"] / pr["launches"] / 1e12
                kernels[k]["TFLOPs"] = pr["flops"] / (pr["total_ms"] * 1e-3) / 1e12
    return kernels


def timed(fn, steps, warmup, ctx, label):
    import torch
    for i in range(warmup):
        r = fn()
        log(f"{label} warmup {i}: {r.time_ms:.0f} ms")
    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for i in range(steps):
        results.append(fn())
        log(f"{label} step {i}: {results[-1].time_ms:.0f} ms")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return results, elapsed


def hbm_roofline(kern, name):
    return {"bound": "hbm", "achieved": kern["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": kern["GBs"] / HBM_PEAK_GBS, "traffic": None, "kernel": name,
            "avg_launch_ms": kern["avg_ms"], "GB_per_launch": kern["GB_per_launch"]}


def run_plain(args, rec, ctx, bl, Xd, Xt, yd, y):
    kw = dict(nlambda=rec.nlambda, lambda_min_ratio=rec.lambda_min_ratio, rule=bl.SCREEN_SSR_BEDPP, tol=args.tol)
    results, elapsed = timed(lambda: bl.fit_path(ctx, Xd, yd, **kw), args.steps, args.warmup, ctx, "plain")
    kernels = kernel_table(ctx, bl, elapsed)
    ctx.profile(False)
    last = results[-1]
    out = {
        "value": args.steps / elapsed,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "dtype": "f64",
        "config": {"workload": f"{rec.name}: genotype X {rec.n}x{rec.p} stored {rec.storage}, "
                               f"{rec.nlambda} lambda to {rec.lambda_min_ratio} lambda_max, SSR-BEDPP, "
                               f"CD tol {args.tol:g}",
                   "n": rec.n, "p": rec.p, "nlambda": rec.nlambda},
        "roofline": hbm_roofline(kernels["scan"], "k_scan (FP64 X)"),
        "kernels": kernels,
        "path": {"n_active_last": int(last.n_active[-1]), "sweeps": int(last.sweeps.sum()),
                 "columns_scanned": int(last.n_scanned.sum()), "violations": int(last.n_viol.sum())},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a column sample) ...")
        out["cpu_baseline"] = cpu_baseline(Xt, y, rec, args.cpu_cols, args.tol)
    return out


def run_precision(args, rec, ctx, bl, Xd, Xt, yd, y):
    import torch
    kw = dict(nlambda=rec.nlambda, lambda_min_ratio=rec.lambda_min_ratio, rule=bl.SCREEN_SSR_BEDPP, tol=args.tol)
    results, elapsed = timed(lambda: bl.fit_path(ctx, Xd, yd, precision=bl.PREC_BF16X3, **kw), args.steps,
                             args.warmup, ctx, "bf16x3")
    kernels = kernel_table(ctx, bl, elapsed)
    ctx.profile(False)
    lp = results[-1]
    # the plain FP64-scan path on the same int8 storage, timed the same way
    plain, el_plain = timed(lambda: bl.fit_path(ctx, Xd, yd, precision=bl.PREC_FP64, **kw), 1, 0, ctx, "plain-i8")
    ctx.profile(False)
    hp = plain[-1]
    same = bool(torch.equal(lp.beta, hp.beta))
    dmax = float((lp.beta - hp.beta).abs().max())
    out = {
        "value": args.steps / elapsed,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "dtype": "i8 codes, bf16x3 matrix-core scan, f64 decisions",
        "config": {"workload": f"{rec.name}: genotype X {rec.n}x{rec.p} stored int8, precision form "
                               f"(BF16 x3 residual pieces, FP32 partial sums promoted to FP64), "
                               f"{rec.nlambda} lambda to {rec.lambda_min_ratio} lambda_max, SSR-BEDPP, "
                               f"CD tol {args.tol:g}",
                   "n": rec.n, "p": rec.p, "nlambda": rec.nlambda},
        "roofline": hbm_roofline(kernels["scan"], "k_scan_bf16 (int8 X, BF16 MFMA)"),
        "kernels": kernels,
        "forms": {"plain_gpu_same_storage_paths_per_s": 1.0 / el_plain,
                  "speedup_vs_plain_gpu": (args.steps / elapsed) * el_plain,
                  "max_abs_dbeta_vs_fp64_path": dmax, "beta_bitwise_equal_to_fp64_path": same,
                  "fp64_rechecks": int(lp.n_recheck.sum())},
        "path": {"n_active_last": int(lp.n_active[-1]), "sweeps": int(lp.sweeps.sum()),
                 "violations": int(lp.n_viol.sum())},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a column sample) ...")
        out["cpu_baseline"] = cpu_baseline(Xt, y, rec, args.cpu_cols, args.tol)
    return out


def run_batch(args, rec, ctx, bl, Xd, Xt, prob):
    import numpy as np
    import torch
    dev = Xd.device
    Y = np.repeat(prob.y, rec.nsub, axis=0)
    Yd = torch.from_numpy(Y).to(dev)
    Md = torch.from_numpy(prob.masks).to(dev)
    NB = Y.shape[0]
    kw = dict(nlambda=rec.nlambda, lambda_min_ratio=rec.lambda_min_ratio, rule=bl.SCREEN_SSR_BEDPP, tol=args.tol)
    results, elapsed = timed(lambda: bl.fit_path_batch(ctx, Xd, Yd, Md, **kw), args.steps, args.warmup, ctx,
                             "batch")
    kernels = kernel_table(ctx, bl, elapsed)
    ctx.profile(False)
    res = results[-1]
    # plain single-problem paths (row mask per problem) on a sample of the problems
    sample = [0, NB // 2 + 1, NB - 1][: max(1, args.plain_sample)]
    t_plain, dmax = [], 0.0
    for b in sample:
        pr, el = timed(lambda: bl.fit_path(ctx, Xd, Yd[b], row_mask=Md[b], **kw), 1, 0, ctx, f"plain[{b}]")
        ctx.profile(False)
        t_plain.append(el)
        dmax = max(dmax, float((pr[-1].beta - res.beta[b]).abs().max()))
    bs = kernels["bscan"]
    paths_per_s = NB * args.steps / elapsed
    plain_pps = len(t_plain) / sum(t_plain)
    out = {
        "value": paths_per_s,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "dtype": "f32 X, f64 MFMA scans, f64 CD",
        "config": {"workload": f"{rec.name}: AR(1) rho {rec.rho} X {rec.n}x{rec.p} float32, {NB} problems "
                               f"({rec.nresp} responses x {rec.nsub} CV row subsets, rows "
                               f"{int(prob.masks.sum(1).min())}..{int(prob.masks.sum(1).max())}), "
                               f"{rec.nlambda} lambda to {rec.lambda_min_ratio} lambda_max each, SSR-BEDPP, "
                               f"CD tol {args.tol:g}; value counts problem paths",
                   "n": rec.n, "p": rec.p, "nlambda": rec.nlambda, "nprob": NB},
        "roofline": {"bound": "mfma", "achieved": bs["TFLOPs"], "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": bs["TFLOPs"] / FP64_MFMA_PEAK_TFLOPS, "traffic": None,
                     "kernel": "k_bscan (X'R, 64 right-hand sides, FP64 MFMA)", "avg_launch_ms": bs["avg_ms"],
                     "TFLOP_per_launch": bs["TFLOP_per_launch"], "GBs": bs["GBs"]},
        "kernels": kernels,
        "forms": {"plain_gpu_paths_per_s": plain_pps, "plain_sample": sample,
                  "speedup_vs_plain_gpu": paths_per_s / plain_pps,
                  "max_abs_dbeta_vs_plain_path": dmax},
        "path": {"sweeps": int(res.sweeps.sum()), "violations": int(res.n_viol.sum()),
                 "n_active_last_mean": float(res.n_active[:, -1].mean())},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a column sample, one problem) ...")
        out["cpu_baseline"] = cpu_baseline(Xt, Y[0], rec, args.cpu_cols, args.tol, mask=prob.masks[0],
                                           what="path of one of the problems")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=("c2", "c3", "c4"))
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--cpu-cols", type=int, default=None)
    ap.add_argument("--plain-sample", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the column-sharded design is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.cpu_cols is None:
        args.cpu_cols = {"c2": 20000, "c3": 8000, "c4": 3000}[args.workload]

    import torch

    import datagen
    import paper_1701_05936_amd as bl

    rec = datagen.RECIPES[args.workload]
    t = time.perf_counter()
    prob = datagen.make(rec) if args.workload == "c4" else None
    Xt = prob.Xt if prob is not None else datagen.design(rec)
    log(f"generated {rec.name} X {Xt.shape[1]}x{Xt.shape[0]} {Xt.dtype} in {time.perf_counter() - t:.1f} s")

    dev = torch.device("cuda", 0)
    storage = {"f64": torch.float64, "f32": torch.float32, "i8": torch.int8}[rec.storage]
    if storage == torch.int8:
        Xd = torch.from_numpy(Xt.view("int8")).to(dev)
    else:
        Xd = torch.from_numpy(Xt).to(dev)
        if Xd.dtype != storage:
            Xd = Xd.to(storage)
    torch.cuda.synchronize()
    log(f"X resident on GPU: {Xd.numel() * Xd.element_size() / 1e9:.1f} GB as {storage}")

    ctx = bl.Context(0)
    n_cu, name = ctx.device_info()
    if args.workload == "c4":
        out = run_batch(args, rec, ctx, bl, Xd, Xt, prob)
    else:
        y = datagen.response(rec, Xt, 0)
        yd = torch.from_numpy(y).to(dev)
        fn = run_precision if args.workload == "c3" else run_plain
        out = fn(args, rec, ctx, bl, Xd, Xt, yd, y)
    ctx.close()
    line = {"metric": METRIC, "value": out.pop("value"), "unit": "paths/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": out.pop("ms_per_step"), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": out.pop("dtype"), "data": "synthetic"}
    line.update(out)
    line["config"]["device"] = name
    line["config"]["cu"] = n_cu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
