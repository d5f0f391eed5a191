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
                200 nonzeros, scans as int8 dot products (--precision-form i8x4, the
                default) or on BF16 matrix cores (bf16x3) with FP64 decisions; the plain
                FP64-scan path on the same int8 storage and the other form are timed
                beside it.
  c4            batched form: AR(1) (rho 0.5) design 20,000 x 200,000 float32 (16 GB),
                64 problems = 32 responses x 2 cross-validation row subsets, 50 lambda
                values each; check scans on BF16 matrix cores with x and r in two pieces
                (--batch-precision bf16x2, the default; bf16x3 three pieces, fp64 FP64
                matrix cores; the other two are timed once beside it, coefficients bit
                for bit); plain single-problem paths on a sample of the problems are
                timed beside it.
  c5            learned-screening form: block AR(1) (rho 0.7, blocks of 100) design
                5,000 x 1,000,000 float32 (20 GB), 300 nonzeros in 30 blocks, SNR 3, 100
                lambda values down to 0.01 lambda_max.  The screening network is first
                trained (on the GPU) on records of --train-paths strong-rule paths of the
                same recipe at --train-p columns (not timed in value); the hybrid-rule path
                on the full design is timed beside the learned one.

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


def _oracle_leg(Xt, y, rec, cols, tol, mask, what, threads):
    import numpy as np

    import oracle

    oracle.set_threads(threads)
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
        "sample": (f"one full {rec.nlambda}-lambda {what} of the FP64 oracle (OpenMP column scans, "
                   f"{oracle.num_threads()} threads) on every {stride}th column ({sample.shape[0]} of {p} columns, "
                   f"all {sample.shape[1]} rows, same y, tol {tol:g}); {dt:.1f} s per path; a linear-in-p "
                   f"extrapolation to all columns would be {1.0 / (dt * p / sample.shape[0]):.3g} paths/s"),
        "k_done": int(path.k_done),
    }


def cpu_baseline(Xt, y, rec, cols, tol, mask=None, what="path"):
    """The FP64 oracle, as it is, on a column sample of the same design (bounded CPU work): with every host
    thread, and with one thread on a tenth of the sample."""
    import oracle

    threads = oracle.num_threads()
    out = _oracle_leg(Xt, y, rec, cols, tol, mask, what, threads)
    out["one_thread"] = _oracle_leg(Xt, y, rec, max(100, cols // 10), tol, mask, what, 1)
    oracle.set_threads(threads)
    return out


ERR_CHUNK = 20_000


def path_error(Xt, y, beta_rows, lams, ks, mask=None):
    """Accuracy of GPU coefficients at lambda indices ks, certified by the FP64 oracle over every column of X
    (in chunks): the oracle's column statistics, the residual of the GPU coefficients, z = X~'r/n, then
      kkt_inactive = max over kept j with beta_j = 0 of |z_j| / lambda - 1   (<= 0 at the optimum),
      kkt_active   = max over beta_j != 0 of |z_j - lambda sign(beta_j)| / lambda,
      gap          = relative duality gap (P - D) / P with P = n Q(beta), theta = r / (n max(lambda, max|z|)),
                     D = ||y~||^2 / 2 - ||y~ - n lambda theta||^2 / 2: an upper bound on the relative
                     objective error of beta against the exact solution."""
    import numpy as np

    import oracle

    p = Xt.shape[0]
    m = None if mask is None else mask.astype(np.float64)
    c, s, keep = np.empty(p), np.empty(p), np.empty(p, dtype=bool)
    for j0 in range(0, p, ERR_CHUNK):
        blk = np.asarray(Xt[j0:j0 + ERR_CHUNK], dtype=np.float64)
        cc, ss, kk, n = oracle.standardize(blk, mask)
        c[j0:j0 + len(blk)], s[j0:j0 + len(blk)], keep[j0:j0 + len(blk)] = cc, ss, kk
    rows = y if mask is None else y[mask > 0]
    yt = y - rows.mean()
    if m is not None:
        yt = yt * m
    out = {}
    for k in ks:
        beta, lam = beta_rows[k], float(lams[k])
        act = np.flatnonzero(beta)
        r = yt.copy()
        for j in act:
            xj = (np.asarray(Xt[j], dtype=np.float64) - c[j]) / s[j]
            r -= beta[j] * (xj if m is None else xj * m)
        z = np.empty(p)
        for j0 in range(0, p, ERR_CHUNK):
            blk = np.asarray(Xt[j0:j0 + ERR_CHUNK], dtype=np.float64)
            z[j0:j0 + len(blk)] = oracle.zscan(blk, c[j0:j0 + len(blk)], s[j0:j0 + len(blk)], keep[j0:j0 + len(blk)],
                                               r, mask)
        inactive = keep & (beta == 0)
        zmax = float(np.max(np.abs(z[keep])))
        P = float(r @ r) / 2.0 + n * lam * float(np.abs(beta).sum())
        theta = r / (n * max(lam, zmax))
        D = float(yt @ yt) / 2.0 - float(np.sum((yt - n * lam * theta) ** 2)) / 2.0
        out[str(k)] = {"lambda": lam, "active": int(act.size),
                       "kkt_inactive": float(np.max(np.abs(z[inactive])) / lam - 1.0),
                       "kkt_active": float(np.max(np.abs(z[act] - lam * np.sign(beta[act]))) / lam) if act.size
                       else 0.0,
                       "rel_duality_gap": (P - D) / P}
    return out


def kernel_table(ctx, bl, elapsed):
    names = (("scan", bl.PROF_SCAN), ("bscan", bl.PROF_BSCAN), ("cd", bl.PROF_CD), ("colstats", bl.PROF_COLSTATS),
             ("gram", bl.PROF_GRAM), ("recheck", bl.PROF_RECHECK), ("setup_scan", bl.PROF_SETUP))
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
            if k == "cd" and pr["units"]:
                # coordinate descent is latency-bound: its figure of merit is time per coordinate update
                kernels[k]["updates"] = pr["units"]
                kernels[k]["updates_per_s"] = pr["units"] / (pr["total_ms"] * 1e-3)
                kernels[k]["ns_per_update"] = pr["total_ms"] * 1e6 / pr["units"]
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


def profiled_traffic(summary):
    """HBM bytes per launch from a committed rocprofv3 counter summary under profiles/, or None when the kernel
    source has changed since the counters were taken (the summary records the source's sha256)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", summary)
    if not os.path.exists(path):
        return None
    traffic, src, sha = None, None, None
    for line in open(path):
        if line.startswith("traffic_bytes_per_launch:"):
            traffic = float(line.split(":", 1)[1])
        elif line.startswith("source:"):
            parts = line.split()
            src, sha = parts[1], parts[-1]
    if traffic is None or src is None:
        return None
    cur = hashlib.sha256(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
    return traffic if cur == sha else None


def hbm_roofline(kern, name, traffic_summary=None):
    return {"bound": "hbm", "achieved": kern["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": kern["GBs"] / HBM_PEAK_GBS,
            "traffic": profiled_traffic(traffic_summary) if traffic_summary else None, "kernel": name,
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
        "roofline": hbm_roofline(kernels["scan"], "k_scan (FP64 X)", "k_scan_c2_genotype_5000x500000_f64.md"),
        "kernels": kernels,
        "path": {"n_active_last": int(last.n_active[-1]), "sweeps": int(last.sweeps.sum()),
                 "columns_scanned": int(last.n_scanned.sum()), "violations": int(last.n_viol.sum())},
    }
    if not args.no_error:
        log("error of the last timed path: oracle KKT certificates and duality gaps over every column ...")
        out["error"] = {"what": "oracle over every column, at the CD tolerance timed",
                        "per_lambda": path_error(Xt, y, last.beta.cpu().numpy(), last.lam, ERROR_KS)}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a column sample) ...")
        out["cpu_baseline"] = cpu_baseline(Xt, y, rec, args.cpu_cols, args.tol)
    return out


ERROR_KS = (20, 60, 99)


PRECISION_FORMS = {
    # form: (bl constant name, dtype, workload text, dominant kernel, counter summary under profiles/)
    "i8x4": ("PREC_I8X4", "i8 codes, int8 dot-product scan against 4 int8 residual pieces, f64 decisions",
             "int8 x4 power-of-two residual pieces, exact int32 sums", "k_scan_i8 (int8 X, int8 dot4)",
             "k_scan_i8_c3_genotype_10000x2000000_i8.md"),
    "bf16x3": ("PREC_BF16X3", "i8 codes, bf16x3 matrix-core scan, f64 decisions",
               "BF16 x3 residual pieces, FP32 partial sums promoted to FP64", "k_scan_bf16 (int8 X, BF16 MFMA)",
               "k_scan_bf16_c3_genotype_10000x2000000_i8.md"),
}


def run_precision(args, rec, ctx, bl, Xd, Xt, yd, y):
    import torch
    const, dtype, text, kname, summary = PRECISION_FORMS[args.precision_form]
    prec = getattr(bl, const)
    kw = dict(nlambda=rec.nlambda, lambda_min_ratio=rec.lambda_min_ratio, rule=bl.SCREEN_SSR_BEDPP, tol=args.tol)
    results, elapsed = timed(lambda: bl.fit_path(ctx, Xd, yd, precision=prec, **kw), args.steps,
                             args.warmup, ctx, args.precision_form)
    kernels = kernel_table(ctx, bl, elapsed)
    ctx.profile(False)
    lp = results[-1]
    # the plain FP64-scan path on the same int8 storage, timed the same way
    plain, el_plain = timed(lambda: bl.fit_path(ctx, Xd, yd, precision=bl.PREC_FP64, **kw), 1, 0, ctx, "plain-i8")
    ctx.profile(False)
    hp = plain[-1]
    same = bool(torch.equal(lp.beta, hp.beta))
    dmax = float((lp.beta - hp.beta).abs().max())
    forms = {"plain_gpu_same_storage_paths_per_s": 1.0 / el_plain,
             "speedup_vs_plain_gpu": (args.steps / elapsed) * el_plain,
             "max_abs_dbeta_vs_fp64_path": dmax, "beta_bitwise_equal_to_fp64_path": same,
             "fp64_rechecks": int(lp.n_recheck.sum())}
    for other in PRECISION_FORMS:
        if other == args.precision_form or args.no_other_forms:
            continue
        op = getattr(bl, PRECISION_FORMS[other][0])
        res_o, el_o = timed(lambda: bl.fit_path(ctx, Xd, yd, precision=op, **kw), 1, 0, ctx, other)
        ctx.profile(False)
        forms[f"{other}_paths_per_s"] = 1.0 / el_o
        forms[f"{other}_beta_bitwise_equal_to_fp64_path"] = bool(torch.equal(res_o[-1].beta, hp.beta))
        forms[f"{other}_fp64_rechecks"] = int(res_o[-1].n_recheck.sum())
    out = {
        "value": args.steps / elapsed,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "dtype": dtype,
        "config": {"workload": f"{rec.name}: genotype X {rec.n}x{rec.p} stored int8, precision form "
                               f"({text}), "
                               f"{rec.nlambda} lambda to {rec.lambda_min_ratio} lambda_max, SSR-BEDPP, "
                               f"CD tol {args.tol:g}",
                   "n": rec.n, "p": rec.p, "nlambda": rec.nlambda},
        "roofline": hbm_roofline(kernels["scan"], kname, summary),
        "kernels": kernels,
        "forms": forms,
        "path": {"n_active_last": int(lp.n_active[-1]), "sweeps": int(lp.sweeps.sum()),
                 "violations": int(lp.n_viol.sum())},
    }
    if not args.no_error:
        log("error of the last timed path: oracle KKT certificates and duality gaps over every column ...")
        out["error"] = {"what": "oracle over every column, at the CD tolerance timed",
                        "per_lambda": path_error(Xt, y, lp.beta.cpu().numpy(), lp.lam, ERROR_KS)}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a column sample) ...")
        out["cpu_baseline"] = cpu_baseline(Xt, y, rec, args.cpu_cols, args.tol)
    return out


BATCH_FORMS = {
    # name: (precision constant, dtype text, kernel text, counter summary under profiles/)
    "fp64": ("PREC_FP64", "f32 X, f64 MFMA check scans, f64 CD", "k_bscan (X'R, 64 right-hand sides, FP64 MFMA)",
             "k_bscan_c4_ar1_20000x200000_f32_64rhs.md"),
    "bf16x3": ("PREC_BF16X3", "f32 X, bf16 MFMA check scans (x, r in 3 pieces), f64 decisions in the band, f64 CD",
               "k_bscan_bf16<3> (X'R on BF16 MFMA, 3+3 pieces)", "k_bscan_bf16x3_c4_ar1_20000x200000_f32_64rhs.md"),
    "bf16x2": ("PREC_BF16X2", "f32 X, bf16 MFMA check scans (x, r in 2 pieces), f64 decisions in the band, f64 CD",
               "k_bscan_bf16<2> (X'R on BF16 MFMA, 2+2 pieces)", "k_bscan_bf16x2_c4_ar1_20000x200000_f32_64rhs.md"),
}


def run_batch(args, rec, ctx, bl, Xd, Xt, prob):
    import numpy as np
    import torch
    dev = Xd.device
    Y = np.repeat(prob.y, rec.nsub, axis=0)
    Yd = torch.from_numpy(Y).to(dev)
    Md = torch.from_numpy(prob.masks).to(dev)
    NB = Y.shape[0]
    kw = dict(nlambda=rec.nlambda, lambda_min_ratio=rec.lambda_min_ratio, rule=bl.SCREEN_SSR_BEDPP, tol=args.tol)
    form = args.batch_precision
    prec, dtype, kname, summary = BATCH_FORMS[form]
    results, elapsed = timed(lambda: bl.fit_path_batch(ctx, Xd, Yd, Md, precision=getattr(bl, prec), **kw),
                             args.steps, args.warmup, ctx, f"batch {form}")
    kernels = kernel_table(ctx, bl, elapsed)
    ctx.profile(False)
    res = results[-1]
    # the other check-scan forms, one step each after a warm-up: coefficients bit for bit
    others = {}
    for o in BATCH_FORMS:
        if o == form or args.no_other_forms:
            continue
        po = getattr(bl, BATCH_FORMS[o][0])
        ro, el = timed(lambda: bl.fit_path_batch(ctx, Xd, Yd, Md, precision=po, **kw), 1, 1, ctx, f"batch {o}")
        ko = kernel_table(ctx, bl, el)
        ctx.profile(False)
        others[o] = {"problem_paths_per_s": NB / el, "check_scan_avg_ms": ko["bscan"]["avg_ms"],
                     "beta_bit_identical": bool(torch.equal(ro[-1].beta, res.beta))}
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
    if form == "fp64":
        roof = {"bound": "mfma", "achieved": bs["TFLOPs"], "peak": FP64_MFMA_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": bs["TFLOPs"] / FP64_MFMA_PEAK_TFLOPS, "traffic": profiled_traffic(summary), "kernel": kname,
                "avg_launch_ms": bs["avg_ms"], "TFLOP_per_launch": bs["TFLOP_per_launch"], "GBs": bs["GBs"]}
    else:
        # the BF16 forms read X once per launch and take 3 (2 pieces) or 6 (3 pieces) BF16 products per FP64
        # product: far below the BF16 matrix-core peak, so HBM bounds them
        roof = hbm_roofline(bs, kname, summary)
    out = {
        "value": paths_per_s,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "dtype": dtype,
        "config": {"workload": f"{rec.name}: AR(1) rho {rec.rho} X {rec.n}x{rec.p} float32, {NB} problems "
                               f"({rec.nresp} responses x {rec.nsub} CV row subsets, rows "
                               f"{int(prob.masks.sum(1).min())}..{int(prob.masks.sum(1).max())}), "
                               f"{rec.nlambda} lambda to {rec.lambda_min_ratio} lambda_max each, SSR-BEDPP, "
                               f"CD tol {args.tol:g}, check scans {form}; value counts problem paths",
                   "n": rec.n, "p": rec.p, "nlambda": rec.nlambda, "nprob": NB, "check_scans": form},
        "roofline": roof,
        "kernels": kernels,
        "forms": {"check_scans": form, "other_check_scans": others,
                  "plain_gpu_paths_per_s": plain_pps, "plain_sample": sample, "scan_cols_autotuned": res.scan_cols,
                  "speedup_vs_plain_gpu": paths_per_s / plain_pps,
                  "max_abs_dbeta_vs_plain_path": dmax},
        "path": {"sweeps": int(res.sweeps.sum()), "violations": int(res.n_viol.sum()),
                 "n_active_last_mean": float(res.n_active[:, -1].mean())},
    }
    if not args.no_error:
        log("error of problem 0 of the last timed batch: oracle certificates over every column ...")
        out["error"] = {"what": "oracle over every column for problem 0 (its rows), at the CD tolerance timed",
                        "per_lambda": path_error(Xt, Y[0], res.beta[0].cpu().numpy(), res.lam[0], (10, 30, 49),
                                                 mask=prob.masks[0])}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a column sample, one problem) ...")
        out["cpu_baseline"] = cpu_baseline(Xt, Y[0], rec, args.cpu_cols, args.tol, mask=prob.masks[0],
                                           what="path of one of the problems")
    return out


def run_learned(args, rec, ctx, bl, Xd, Xt, yd, y):
    import numpy as np
    import torch

    import datagen
    dev = Xd.device
    kw = dict(nlambda=rec.nlambda, lambda_min_ratio=rec.lambda_min_ratio, tol=args.tol)
    # the hybrid-rule path on the full design first (also warms the context up)
    plain, el_plain = timed(lambda: bl.fit_path(ctx, Xd, yd, rule=bl.SCREEN_SSR_BEDPP, **kw), 1, 0, ctx, "hybrid")
    ctx.profile(False)
    hp = plain[-1]
    log(f"hybrid path: {int(hp.n_active[-1])} active at the end, working sets {int(hp.n_strong.sum())}, "
        f"sweeps {int(hp.sweeps.sum())}")
    # training records from strong-rule paths of the same recipe at a reduced column count
    t_train = time.perf_counter()
    cap = 40_000_000
    feat = torch.zeros((cap, 4), dtype=torch.float32, device=dev)
    lab = torch.zeros(cap, dtype=torch.float32, device=dev)
    n_rec, paths, per_x = 0, 0, 10
    # the same lambda grid (ratio per step) as the timed path, cut after --train-depth values: past that
    # depth a reduced design's fit approaches n active features and its paths only cost time
    step = rec.lambda_min_ratio ** (1.0 / (rec.nlambda - 1))
    gpu_ms = 0.0
    for xi in range((args.train_paths + per_x - 1) // per_x):
        trec = rec.scaled(p=args.train_p, seed=rec.seed + 1000 + xi, nresp=per_x)
        tp = datagen.make(trec)
        Xtr = torch.from_numpy(tp.Xt).to(dev)
        for t in range(per_x):
            if paths >= args.train_paths:
                break
            ytr = torch.from_numpy(tp.y[t]).to(dev)
            lmax = bl.fit_path(ctx, Xtr, ytr, nlambda=1, want_beta=False).lambda_max
            grid = lmax * step ** np.arange(args.train_depth)
            r = bl.fit_path(ctx, Xtr, ytr, nlambda=args.train_depth, lambdas=grid, rule=bl.SCREEN_SSR_BEDPP,
                            tol=args.tol, rec_feat=feat[n_rec:], rec_label=lab[n_rec:], want_beta=False)
            n_rec += r.n_recorded
            paths += 1
            gpu_ms += r.time_ms
            log(f"training path {paths}: {r.time_ms:.0f} ms, {r.n_recorded} records, "
                f"{int(r.n_active[-1])} active at the end")
        del Xtr
    P = torch.from_numpy(bl.mlp_init(1)).to(dev)
    info = bl.mlp_train(ctx, feat[:n_rec].contiguous(), lab[:n_rec].contiguous(), P, epochs=args.train_epochs,
                        batch=8192, lr=2e-3, seed=5, target_recall=args.target_recall)
    log(f"trained on {n_rec} records: {info}")
    positives = float(lab[:n_rec].sum())
    del feat, lab
    torch.cuda.empty_cache()
    train_s = time.perf_counter() - t_train

    results, elapsed = timed(lambda: bl.fit_path(ctx, Xd, yd, rule=bl.SCREEN_LEARNED, mlp=P, mlp_tau=info["tau"], **kw),
                             args.steps, args.warmup, ctx, "learned")
    kernels = kernel_table(ctx, bl, elapsed)
    ctx.profile(False)
    lr_ = results[-1]
    dmax = float((lr_.beta - hp.beta).abs().max())
    out = {
        "value": args.steps / elapsed,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "dtype": "f32 X, f64 scans and CD, f32 screening network",
        "config": {"workload": f"{rec.name}: block AR(1) rho {rec.rho} (blocks of {rec.block}) X {rec.n}x{rec.p} "
                               f"float32, {rec.nnz} nonzeros, SNR {rec.snr}, {rec.nlambda} lambda to "
                               f"{rec.lambda_min_ratio} lambda_max, learned screening (network-filtered strong rule "
                               f"+ BEDPP + exact check), CD tol {args.tol:g}",
                   "n": rec.n, "p": rec.p, "nlambda": rec.nlambda},
        "roofline": hbm_roofline(kernels["scan"], "k_scan (f32 X)", "k_scan_c5_blockar1_5000x1000000_f32.md"),
        "kernels": kernels,
        "forms": {"plain_gpu_paths_per_s": 1.0 / el_plain, "speedup_vs_plain_gpu": (args.steps / elapsed) * el_plain,
                  "max_abs_dbeta_vs_plain_path": dmax,
                  "working_set_sum_learned": int(lr_.n_strong.sum()), "working_set_sum_plain": int(hp.n_strong.sum()),
                  "violations_learned": int(lr_.n_viol.sum()), "violations_plain": int(hp.n_viol.sum()),
                  "sweeps_learned": int(lr_.sweeps.sum()), "sweeps_plain": int(hp.sweeps.sum()),
                  "training": {"paths": paths, "columns": args.train_p, "lambdas_per_path": args.train_depth,
                               "records": n_rec, "positives": positives,
                               "epochs": args.train_epochs, "tau": info["tau"], "recall": info["recall"],
                               "neg_pass": info["neg_pass"], "loss_first": info["loss_first"],
                               "loss_last": info["loss_last"], "train_ms": info["time_ms"],
                               "path_gpu_ms": gpu_ms, "wall_s": train_s}},
        "path": {"n_active_last": int(lr_.n_active[-1]), "sweeps": int(lr_.sweeps.sum()),
                 "violations": int(lr_.n_viol.sum())},
    }
    if not args.no_error:
        log("error of the last timed path: oracle KKT certificates and duality gaps over every column ...")
        out["error"] = {"what": "oracle over every column, at the CD tolerance timed",
                        "per_lambda": path_error(Xt, y, lr_.beta.cpu().numpy(), lr_.lam, ERROR_KS)}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on a column sample) ...")
        out["cpu_baseline"] = cpu_baseline(Xt, y, rec, args.cpu_cols, args.tol)
    return out


def _load_design(rec, dev):
    import torch

    import datagen
    t = time.perf_counter()
    prob = datagen.make(rec) if rec.name == "c4" else None
    Xt = prob.Xt if prob is not None else datagen.design(rec)
    log(f"generated {rec.name} X {Xt.shape[1]}x{Xt.shape[0]} {Xt.dtype} in {time.perf_counter() - t:.1f} s")
    storage = {"f64": torch.float64, "f32": torch.float32, "i8": torch.int8}[rec.storage]
    if storage == torch.int8:
        Xd = torch.from_numpy(Xt.view("int8")).to(dev)
    else:
        Xd = torch.from_numpy(Xt).to(dev)
        if Xd.dtype != storage:
            Xd = Xd.to(storage)
    torch.cuda.synchronize()
    log(f"X resident on GPU: {Xd.numel() * Xd.element_size() / 1e9:.1f} GB as {storage}")
    return prob, Xt, Xd


def run_forms(args, ctx, bl, dev):
    """The precision form (c3: int8 storage, int8 dot-product scans, against the FP64-scan path on the same
    storage) and the batched form (c4: 64 problems in lockstep, against single-problem paths), each timed
    over one step after one warm-up at the same CD tolerance, with the headline's context."""
    import copy

    import torch

    import datagen
    sub = copy.copy(args)
    sub.steps, sub.warmup, sub.no_cpu_baseline, sub.no_error = 1, 1, True, True
    forms = {}
    rec = datagen.RECIPES["c3"]
    _, Xt, Xd = _load_design(rec, dev)
    y = datagen.response(rec, Xt, 0)
    o = run_precision(sub, rec, ctx, bl, Xd, Xt, torch.from_numpy(y).to(dev), y)
    forms["c3_precision"] = {"workload": o["config"]["workload"], "paths_per_s": o["value"], "dtype": o["dtype"],
                             "roofline": o["roofline"], **o["forms"]}
    del Xd, Xt
    torch.cuda.empty_cache()
    rec = datagen.RECIPES["c4"]
    prob, Xt, Xd = _load_design(rec, dev)
    o = run_batch(sub, rec, ctx, bl, Xd, Xt, prob)
    forms["c4_batched"] = {"workload": o["config"]["workload"], "problem_paths_per_s": o["value"],
                           "dtype": o["dtype"], "roofline": o["roofline"], **o["forms"]}
    del Xd, Xt, prob
    torch.cuda.empty_cache()
    return forms


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=("c2", "c3", "c4", "c5"))
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--cpu-cols", type=int, default=None)
    ap.add_argument("--plain-sample", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision-form", default="i8x4", choices=tuple(PRECISION_FORMS),
                    help="matrix-core form of the c3 check scans (the other form is timed once beside it)")
    ap.add_argument("--no-other-forms", action="store_true",
                    help="c3, c4: skip the other precision forms' paths")
    ap.add_argument("--batch-precision", default="bf16x2", choices=tuple(BATCH_FORMS),
                    help="c4: arithmetic of the batched form's check scans (the others are timed once beside it)")
    ap.add_argument("--copy-calib", type=float, default=0.0,
                    help="only copy a buffer of this many GB once (device to device) and exit: the reference "
                         "kernel for scaling FETCH_SIZE / WRITE_SIZE counters")
    ap.add_argument("--train-paths", type=int, default=200)
    ap.add_argument("--train-p", type=int, default=10000)
    ap.add_argument("--train-depth", type=int, default=60)
    ap.add_argument("--train-epochs", type=int, default=20)
    ap.add_argument("--target-recall", type=float, default=0.995)
    ap.add_argument("--no-error", action="store_true", help="skip the oracle's error certificate of the timed path")
    ap.add_argument("--no-forms", action="store_true",
                    help="c2: skip timing the precision (c3) and batched (c4) forms beside the headline")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: there is no multi-GPU path (it would shard X by columns and "
              "exchange only screening candidates and violators per lambda); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.copy_calib > 0:
        import torch
        n = int(args.copy_calib * 1e9) // 8
        src = torch.arange(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8}), flush=True)
        return
    if args.cpu_cols is None:
        args.cpu_cols = {"c2": 20000, "c3": 1000, "c4": 3000, "c5": 500}[args.workload]

    import torch

    import datagen
    import paper_1701_05936_amd as bl

    rec = datagen.RECIPES[args.workload]
    dev = torch.device("cuda", 0)
    prob, Xt, Xd = _load_design(rec, dev)

    ctx = bl.Context(0)
    n_cu, name = ctx.device_info()
    if args.workload == "c4":
        out = run_batch(args, rec, ctx, bl, Xd, Xt, prob)
    else:
        y = datagen.response(rec, Xt, 0)
        yd = torch.from_numpy(y).to(dev)
        fn = {"c2": run_plain, "c3": run_precision, "c5": run_learned}[args.workload]
        out = fn(args, rec, ctx, bl, Xd, Xt, yd, y)
    if args.workload == "c2" and not args.no_forms:
        del Xd, Xt
        torch.cuda.empty_cache()
        out["forms"] = run_forms(args, ctx, bl, dev)
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
