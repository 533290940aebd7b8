#!/usr/bin/env python3
"""Benchmark of the Sinkhorn divergence hot path on one MI355X.

Default workload (--workload fibers1m): time-to-S_eps on n = m = 1,000,000 fibres
(20 points each flattened to 60-D and scaled by 1/sqrt(20), 200 Bezier bundles,
uniform weights), blur 1 mm, reach 20 mm, scaling 0.9, K-means coarse phase with
sqrt(n) clusters, cluster-block truncation (theta 20), converged mode (marginal
error <= 1e-4, checked every --check-every iterations).  A step is one whole
solve of the chosen path (BF16 hi/lo split + learned warm start: tokens, network
forward, broadcast, clustering, the averaged loop of four softmins per iteration
and the FP64 value of eq. (6)), inputs resident in HBM.  Beside it, each over the
same steps: the plain path (FP32, cold eps-scaling), the BF16 split cold, the
network's ablation (zero starting values on the chosen path's shortened schedule,
one solve), one dense 200k x 200k BF16 solve (the softmin kernel without
block-sparse ranges), and the FP64 oracle on sampled rows (one thread and all).

Other workloads: fibers200k (dense 200k x 200k solve, Gpair/s), grad200k (all four
gradients), labels200k / labels250k (label transfer with flips), pcost200k (cost
|x - y|, 3-D), barycenter10 (one barycenter descent step over 10 density maps).

Prints one JSON line:
  value       = fibers1m: mean time to S of the chosen path (s); otherwise the
                workload's own metric
  roofline    = the softmin kernel's algorithmic MFMA flops per launch over its
                average launch time (HIP events on the library's stream)
  cpu_baseline= the FP64 oracle's softmin on a bounded row sample of the same
                workload, on the host cores

    python bench.py [--steps K] [--warmup W] [--workload ...] [--legs ...]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp32": 157.3, "bf16x3": 2500.0}  # MI355X dense MFMA, FP32 and BF16
FLOP_PER_PAIR = {"fp32": 128, "bf16x3": 384}      # 64-wide contraction; x3 for the hi/lo split
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = {"fp32": os.path.join(ROOT, "paper_2107_02010_amd", "csrc", "softmin.hip"),
              "bf16x3": os.path.join(ROOT, "paper_2107_02010_amd", "csrc", "softmin_bf16.hip")}
# rocprofv3 FETCH_SIZE / WRITE_SIZE summaries, per workload (each taken on that workload)
TRAFFIC_FILES = {"fibers200k": os.path.join(ROOT, "profiles", "softmin_fiber200k_traffic.txt"),
                 "fibers1m": os.path.join(ROOT, "profiles", "softmin_bf16_fibers1m_traffic.txt")}


def kernel_hash(precision: str) -> str:
    return hashlib.sha256(open(KERNEL_SRC[precision], "rb").read()).hexdigest()[:16]


def read_traffic(precision: str, workload: str):
    """HBM bytes per softmin launch from the committed rocprofv3 PMC summary of this
    workload, or None when it is absent or was taken on another version of the kernel."""
    path = TRAFFIC_FILES.get(workload)
    if not path or not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(rf"kernel_sha256_16\[{precision}\]:\s*([0-9a-f]+)", txt)
    t = re.search(rf"^bytes_per_launch\[{precision}\]:\s*([0-9.eE+]+)", txt, flags=re.M)
    if not m or not t or m.group(1) != kernel_hash(precision):
        return None
    return float(t.group(1))


def cpu_baseline(x, y, b, target_s: float = 8.0):
    """FP64 oracle softmin of a row sample against all columns; doubles the sample
    until one measurement takes target_s seconds (or all rows are used)."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(0)
    h = np.zeros(len(y), np.float32)
    rows = 32
    while True:
        idx = rng.choice(len(x), size=min(rows, len(x)), replace=False)
        t0 = time.perf_counter()
        oracle.softmin(x[idx], y, b, h, 1.0, 1.0)
        dt = time.perf_counter() - t0
        if dt >= target_s or rows >= len(x):
            break
        rows *= 2
    pairs = len(idx) * len(y)
    return {"value": pairs / dt / 1e9, "unit": "Gpair/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"one FP64 softmin pass, {len(idx)} sampled rows x {len(y)} columns, "
                      f"60-D, eps=1 ({pairs:.3g} pairs, {dt:.1f} s)"}


def solve_steps(skh, X, A, Y, B, steps, warmup, label, **kw):
    import torch
    for k in range(warmup):
        skh.sinkhorn_divergence(X, A, Y, B, **kw)
        print(f"[bench] {label} warmup {k + 1}/{warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    agg = dict(pairs=0.0, ms_softmin=0.0, launches=0, dense_pairs=0.0)
    S, st = None, None
    for k in range(steps):
        S, _, st = skh.sinkhorn_divergence(X, A, Y, B, **kw)
        agg["pairs"] += st["pairs"]
        agg["dense_pairs"] += st["dense_pairs"]
        agg["ms_softmin"] += st["ms_softmin"]
        agg["launches"] += st["softmin_launches"]
        print(f"[bench] {label} step {k + 1}/{steps}: S={S:.10g} iters={st['iters']} "
              f"{st['ms_total']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    agg["dt"] = time.perf_counter() - t0
    agg["S"] = S
    agg["stats"] = st
    return agg


def roofline(agg, precision, workload):
    pairs_per_launch = agg["pairs"] / agg["launches"]
    avg_launch_s = agg["ms_softmin"] / agg["launches"] / 1e3
    achieved = FLOP_PER_PAIR[precision] * pairs_per_launch / avg_launch_s / 1e12
    peak = PEAK_TFLOPS[precision]
    return {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
            "frac": round(achieved / peak, 4), "traffic": read_traffic(precision, workload),
            "flop_per_pair": FLOP_PER_PAIR[precision],
            "avg_launch_ms": round(avg_launch_s * 1e3, 4),
            "kernel": "k_softmin_f32<64>" if precision == "fp32" else "k_softmin_bf16<64>"}, \
        pairs_per_launch / avg_launch_s / 1e9


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_1m(x, y, b, iters_dense: int, rows_all: int = 4096, rows_one: int = 256):
    """The FP64 oracle's softmin on sampled rows of the 1M x 1M fibre workload against all
    of its columns, on all host threads and on one thread; the time-to-S of a dense FP64
    oracle solve of the same iteration count is extrapolated from the all-threads rate
    (a full dense oracle solve, about 4e12 point pairs per iteration, is out of reach)."""
    import numpy as np

    import oracle
    rng = np.random.default_rng(0)
    h = np.zeros(len(y), np.float32)
    res = {}
    threads_all = oracle.num_threads()
    for tag, rows, threads in (("all_cores", rows_all, threads_all), ("one_core", rows_one, 1)):
        oracle.set_num_threads(threads)
        idx = rng.choice(len(x), size=min(rows, len(x)), replace=False)
        t0 = time.perf_counter()
        oracle.softmin(x[idx], y, b, h, 1.0, 1.0)
        dt = time.perf_counter() - t0
        res[tag] = {"gpair_s": len(idx) * len(y) / dt / 1e9, "threads": threads,
                    "sample": f"{len(idx)} sampled rows x {len(y)} columns ({dt:.1f} s)"}
        print(f"[bench] oracle softmin {tag}: {res[tag]['gpair_s']:.4f} Gpair/s",
              file=sys.stderr, flush=True)
    oracle.set_num_threads(threads_all)
    pairs = 4.0 * iters_dense * len(x) * len(y)
    return {"value": round(pairs / (res["all_cores"]["gpair_s"] * 1e9), 1), "unit": "s",
            "cores": threads_all, "kind": "oracle", "extrapolated": True,
            "cpu_model": cpu_model(),
            "sample": f"one FP64 oracle softmin pass over {res['all_cores']['sample']} on "
                      f"{threads_all} threads; value = time-to-S of a dense FP64 oracle solve "
                      f"of {iters_dense} iterations x 4 softmins x {len(x)} x {len(y)} pairs "
                      "at that rate (extrapolated, not run)",
            "gpair_s_all_cores": round(res["all_cores"]["gpair_s"], 5),
            "gpair_s_one_core": round(res["one_core"]["gpair_s"], 5),
            "sample_one_core": res["one_core"]["sample"]}


def _leg(label, fn, steps, warmup, precision):
    """Times `steps` calls of a solve after `warmup`; returns the leg's summary (mean time
    to S over the steps, iterations, S of the last step, the softmin roofline from the
    HIP-event times of every timed launch)."""
    import torch
    for k in range(warmup):
        fn()
        print(f"[bench] {label} warmup {k + 1}/{warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    agg = dict(pairs=0.0, ms_softmin=0.0, launches=0, dense_pairs=0.0)
    times, S, st = [], None, None
    for k in range(steps):
        t0 = time.perf_counter()
        S, _, st = fn()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        agg["pairs"] += st["pairs"]
        agg["dense_pairs"] += st["dense_pairs"]
        agg["ms_softmin"] += st["ms_softmin"]
        agg["launches"] += st["softmin_launches"]
        print(f"[bench] {label} step {k + 1}/{steps}: S={S:.10g} iters={st['iters']} "
              f"{times[-1] * 1e3:.1f} ms", file=sys.stderr, flush=True)
    rl, kern = roofline(agg, precision, "fibers1m")
    return {"time_to_S_s": round(sum(times) / len(times), 4),
            "time_to_S_min_s": round(min(times), 4), "S": S, "iters": st["iters"],
            "coarse_iters": st["coarse_iters"], "converged": st["converged"],
            "marginal_err": st["marginal_err"], "warm_fallback": st.get("warm_fallback", 0),
            "kept_fraction": round(agg["pairs"] / max(agg["dense_pairs"], 1.0), 5),
            "softmin_kernel_gpair_s": round(kern, 3), "roofline": rl,
            "_total_s": sum(times)}


def bench_fibers1m(args, skh, synth):
    """The metric's configuration: time-to-S_eps on 1M x 1M fibres, plain vs chosen."""
    import torch
    from paper_2107_02010_amd.warm_start import (DEFAULT_CHECKPOINT, WarmStartNet,
                                                 sinkhorn_divergence_warm)
    legs = set(args.legs.split(","))
    n = args.n if args.n != 200_000 else 1_000_000
    print(f"[bench] generating {n} x {n} fibre clouds (200 bundles)", file=sys.stderr, flush=True)
    x, a, y, b = synth.fiber_pair(n, 200, seed=0)
    dev = torch.device("cuda:0")
    X, A, Y, B = (torch.as_tensor(v).to(dev) for v in (x, a, y, b))
    blur, scaling = 1.0, 0.9
    kw = dict(reach=20.0, tol=1e-4, check_every=args.check_every, max_iters=20000,
              multiscale=True, timing=True)
    net = WarmStartNet.load(DEFAULT_CHECKPOINT, "cuda:0")
    K, W = args.steps, args.warmup
    res = {}
    # chosen: BF16 split + learned warm start; tokens, network forward, broadcast and the
    # solve are all inside the timed region
    if "chosen" in legs:
        res["chosen"] = _leg("chosen (bf16x3 + warm start)", lambda: sinkhorn_divergence_warm(
            net, X, A, Y, B, blur, scaling=scaling, precision="bf16x3", **kw), K, W, "bf16x3")
    if "plain" in legs:
        res["plain"] = _leg("plain (fp32, cold)", lambda: skh.sinkhorn_divergence(
            X, A, Y, B, blur=blur, scaling=scaling, precision="fp32", potentials=True, **kw),
            K, W, "fp32")
    if "bf16_cold" in legs:
        res["bf16_cold"] = _leg("bf16x3, cold", lambda: skh.sinkhorn_divergence(
            X, A, Y, B, blur=blur, scaling=scaling, precision="bf16x3", potentials=True, **kw),
            K, W, "bf16x3")
    if "zero_start" in legs:
        # ablation of the network: the chosen path's clustering, shortened schedule and
        # checked start, with zero starting values instead of the prediction
        zkw = dict(kw, max_iters=2000)
        res["zero_start"] = _leg("bf16x3, zero start at the warm schedule",
                                 lambda: sinkhorn_divergence_warm(
                                     net, X, A, Y, B, blur, scaling=scaling, precision="bf16x3",
                                     start="zero", **zkw), 1, 0, "bf16x3")
    dense = None
    if "dense200k" in legs:
        # the dense 200k x 200k BF16 softmin (C2 shape) beside it: the kernel's fraction of
        # the BF16 MFMA peak without block-sparse ranges
        del X, A, Y, B
        torch.cuda.empty_cache()
        xd, ad, yd, bd = synth.fiber_pair(200_000, 50, seed=0)
        Xd, Ad, Yd, Bd = (torch.as_tensor(v).to(dev) for v in (xd, ad, yd, bd))
        agg = solve_steps(skh, Xd, Ad, Yd, Bd, 1, 0, "dense 200k bf16x3", blur=1.0, reach=None,
                          scaling=0.9, potentials=True, timing=True, precision="bf16x3")
        rl, kern = roofline(agg, "bf16x3", "fibers200k")
        dense = {"workload": "fibre clouds n=m=200000, 50 bundles, blur 1 mm, balanced, dense, "
                             f"{agg['stats']['iters']} iterations",
                 "softmin_kernel_gpair_s": round(kern, 3), "solve_gpair_s":
                     round(agg["pairs"] / agg["dt"] / 1e9, 3), "S": agg["S"],
                 "frac": rl["frac"], "avg_launch_ms": rl["avg_launch_ms"],
                 "traffic": rl["traffic"]}
    out_legs = {k: {kk: vv for kk, vv in v.items() if not kk.startswith("_")}
                for k, v in res.items()}
    main = res.get("chosen") or next(iter(res.values()))
    out = {
        "metric": "Gpair/s of log-sum-exp softmin; time-to-S_eps 1M x 1M fibers, plain vs chosen",
        "value": main["time_to_S_s"], "unit": "s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(main["time_to_S_s"] * 1e3, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3",
        "data": "synthetic",
        "config": {"workload": f"time to S_eps, fibre clouds n=m={n}, 60-D (20 points x 3, "
                               "/sqrt(20)), 200 Bezier bundles, jitter 2 mm, blur 1 mm, reach "
                               "20 mm, scaling 0.9, K-means sqrt(n) clusters, truncation theta "
                               f"20, converged to a marginal error 1e-4 checked every "
                               f"{args.check_every} iteration(s); value = chosen path (BF16 split "
                               "+ learned warm start)"},
        "legs": out_legs,
        "roofline": main["roofline"],
        "softmin_kernel_gpair_s": main["softmin_kernel_gpair_s"],
    }
    if "chosen" in res and "plain" in res:
        out["speedup_chosen_vs_plain"] = round(res["plain"]["time_to_S_s"]
                                               / res["chosen"]["time_to_S_s"], 3)
        out["S_rel_diff_chosen_vs_plain"] = abs(res["chosen"]["S"] - res["plain"]["S"]) \
            / abs(res["plain"]["S"])
    if "chosen" in res and "zero_start" in res:
        out["network_gain"] = {
            "iters_zero_start": res["zero_start"]["iters"], "iters_network": res["chosen"]["iters"],
            "time_ratio": round(res["zero_start"]["time_to_S_s"] / res["chosen"]["time_to_S_s"], 3)}
    if dense:
        out["dense200k_bf16x3"] = dense
    if "cpu" in legs and not args.no_cpu_baseline:
        iters = res["plain"]["iters"] if "plain" in res else main["iters"]
        print("[bench] timing the FP64 oracle on sampled rows", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline_1m(x, y, b, iters)
    print(json.dumps(out), flush=True)
    return 0


def _timed(fn, steps, warmup):
    """Mean wall time of fn() over `steps` calls after `warmup`, bracketed by synchronisations."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        out = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, out


def bench_gradients(args, skh, synth):
    """All four gradients of S (dS/dx, dS/dy by the plan-weighted kernels, dS/da, dS/db
    elementwise) from the dual vectors of a converged 200k x 200k fibre solve."""
    import torch
    n = args.n
    print(f"[bench] generating {n} x {n} fibre clouds", file=sys.stderr, flush=True)
    x, a, y, b = synth.fiber_pair(n, args.bundles, seed=0)
    X, A, Y, B = (torch.as_tensor(v).cuda() for v in (x, a, y, b))
    S, pot, st = skh.sinkhorn_divergence(X, A, Y, B, blur=1.0, reach=20.0, scaling=0.9,
                                         tol=1e-4, max_iters=5000, precision="bf16x3",
                                         potentials=True)
    print("[bench] solve done; timing the gradients", file=sys.stderr, flush=True)
    dt, G = _timed(lambda: skh.gradients(X, A, Y, B, pot, 1.0, 20.0), args.steps, args.warmup)
    pairs = 2.0 * n * n + 2.0 * n * n  # grad_x: n x m and n x n plans; grad_y: m x n, m x m
    flop = 256  # per pair: 64-wide FP32 contraction + 64-wide weighted coordinate sum (MFMA)
    ach = flop * pairs / dt / 1e12
    out = {"metric": f"Gpair/s of the gradient plan kernels (dS/dx, dS/dy, dS/da, dS/db; "
                     f"{n} x {n} 60-D fibres)",
           "value": round(pairs / dt / 1e9, 3), "unit": "Gpair/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"gradients after a converged solve, fibre clouds n=m={n}, "
                                  f"{args.bundles} bundles, blur 1 mm, reach 20 mm"},
           "roofline": {"bound": "mfma", "achieved": round(ach, 3), "peak": 157.3,
                        "unit": "TFLOP/s", "frac": round(ach / 157.3, 4), "traffic": None,
                        "flop_per_pair": flop, "timed": "whole skh_gradients call"},
           "grad_norms": {k: float(torch.linalg.vector_norm(v.double())) for k, v in G.items()}}
    print(json.dumps(out), flush=True)
    return 0


def bench_labels(args, skh, synth):
    """Label transfer (eq. (7)) from a 200k-fibre atlas of 50 labelled bundles to a 200k-fibre
    subject stored in random directions plus 1 % aberrant fibres, with flip augmentation,
    multiscale BF16 solve over the Algorithm's schedule.  labels250k: the size of the
    paper's hemisphere experiment (250k-fibre subject, 200k-fibre atlas, blur 2 mm)."""
    import numpy as np
    import torch
    paper_size = args.workload == "labels250k"
    n = 250_000 if paper_size else args.n        # subject fibres
    n_at = 200_000 if paper_size else args.n     # atlas fibres
    blur = 2.0 if paper_size else 1.0
    nout = n // 100
    print(f"[bench] generating atlas ({n_at} fibres) and subject ({n} fibres, {nout} outliers)",
          file=sys.stderr, flush=True)
    y = synth.fibers(n_at, args.bundles, spine_seed=0, seed=1)
    ly = synth.fiber_labels(n_at, args.bundles)
    x = np.concatenate([synth.random_orientations(synth.fibers(n, args.bundles, spine_seed=0,
                                                               seed=2), 20, seed=3),
                        synth.outlier_fibers(nout, seed=4)])
    lx = np.concatenate([synth.fiber_labels(n, args.bundles), -np.ones(nout, np.int32)])
    a, b = synth.uniform_weights(len(x)), synth.uniform_weights(n_at)
    X, A, Y, B = (torch.as_tensor(v).cuda() for v in (x, a, y, b))
    LY = torch.as_tensor(ly, dtype=torch.int32).cuda()
    kw = dict(blur=blur, reach=20.0, flip_points=20, multiscale=True, tol=0.0,
              precision="bf16x3", stats=True)
    dt, (lab, score, st) = _timed(lambda: skh.label_transfer(X, A, Y, B, LY, args.bundles, **kw),
                                  args.steps, args.warmup)
    lab, score = lab.cpu().numpy(), score.cpu().numpy()
    inl = lx >= 0
    out = {"metric": f"time to soft labels, {n}-fibre subject (+1 % outliers, flips) from a "
                     f"{n_at}-fibre atlas",
           "value": round(dt, 4), "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(dt * 1e3, 3), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3", "data": "synthetic",
           "config": {"workload": f"label transfer, {args.bundles} labelled bundles, 60-D fibres "
                                  "stored in random directions, flip augmentation, "
                                  f"blur {blur:g} mm, "
                                  "reach 20 mm, scaling 0.9, multiscale, the Algorithm's "
                                  "schedule (one iteration per scale)"},
           "accuracy_inliers": float(np.mean(np.argmax(lab[inl], 1) == lx[inl])),
           "max_outlier_score": float(score[~inl].max()),
           "min_inlier_score": float(score[inl].min()),
           "iters": st["iters"], "converged": st["converged"],
           "kept_fraction": round(st["pairs"] / max(st["dense_pairs"], 1.0), 5)}
    print(json.dumps(out), flush=True)
    return 0


def bench_pcost(args, skh, synth):
    """Full solve with the cost |x - y| (p = 1) on 200k x 200k 3-D blob clouds: the VALU
    softmin (direct coordinate differences, a square root, one exponential per pair)."""
    import torch
    n = args.n
    print(f"[bench] generating {n} x {n} 3-D blob clouds", file=sys.stderr, flush=True)
    x, a, y, b = synth.blob_pair(n, seed=0)
    X, A, Y, B = (torch.as_tensor(v).cuda() for v in (x, a, y, b))
    kw = dict(blur=0.01, reach=None, scaling=0.9, potentials=True, timing=True, p=1.0)
    agg = solve_steps(skh, X, A, Y, B, args.steps, args.warmup, "p = 1", **kw)
    st = agg["stats"]
    kern_s = agg["ms_softmin"] / agg["launches"] / 1e3
    ppl = agg["pairs"] / agg["launches"]
    # algorithmic ALU work per pair: d subtractions and d multiply-adds for |x - y|^2, the
    # square root, the exponent FMA, the exponential and the sum (2 d + 2 lane operations
    # plus two transcendentals at TRANS_SLOTS each, d = 3); the running maximum and the
    # level subtraction are the kernel's own bookkeeping, not counted
    ops = 2 * 3 + 2 + 2 * TRANS_SLOTS
    peak = VALU_LANE_PEAK / 1e12
    ach = ops * ppl / kern_s / 1e12
    out = {"metric": "Gpair/s of the log-sum-exp softmin, cost |x - y| (full S_eps solve, "
                     f"{n} x {n} 3-D clouds)",
           "value": round(agg["pairs"] / agg["dt"] / 1e9, 3), "unit": "Gpair/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(agg["dt"] / args.steps * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"3-D Gaussian blob clouds n=m={n}, cost |x-y| (p = 1), "
                                  "blur 0.01, balanced, scaling 0.9, dense",
                      "iterations": st["iters"]},
           "S": agg["S"], "softmin_kernel_gpair_s": round(ppl / kern_s / 1e9, 3),
           "roofline": {"bound": "alu", "achieved": round(ach, 3), "peak": round(peak, 2),
                        "unit": "Tslot/s", "frac": round(ach / peak, 4), "traffic": None,
                        "slots_per_pair": ops, "avg_launch_ms": round(kern_s * 1e3, 4),
                        "kernel": "k_softmin_pcost<4, p = 1>"}}
    print(json.dumps(out), flush=True)
    return 0


# ALU ceiling of the VALU-bound kernels (3-D and p-cost softmins).  The issue-rate
# probe (paper_2107_02010_amd/valu_probe, `--workload valu_probe`) measures a wave64
# FP32 add at 2 clocks of a SIMD (32 lanes per clock: 256 CUs x 4 SIMDs x 32 lanes x
# 2.4 GHz = 78.6e12 lane operations per second, the FP32 vector peak counted one
# operation per lane) and v_exp_f32 at 4 such issue slots, not overlapping the adds.
VALU_LANE_PEAK = 256 * 4 * 32 * 2.4e9
TRANS_SLOTS = 4


def bench_blobs(args, skh, synth):
    """Full solve with the cost |x - y|^2 / 2 on 200k x 200k 3-D blob clouds (the 3-D
    path of the small-point workloads): k_softmin_f32<4>, the 4-wide contraction on the
    matrix cores, one exponential and one add per pair on the VALU."""
    import torch
    n = args.n
    print(f"[bench] generating {n} x {n} 3-D blob clouds", file=sys.stderr, flush=True)
    x, a, y, b = synth.blob_pair(n, seed=0)
    X, A, Y, B = (torch.as_tensor(v).cuda() for v in (x, a, y, b))
    kw = dict(blur=0.01, reach=None, scaling=0.9, potentials=True, timing=True,
              precision="fp32")
    agg = solve_steps(skh, X, A, Y, B, args.steps, args.warmup, "3-D p = 2", **kw)
    st = agg["stats"]
    kern_s = agg["ms_softmin"] / agg["launches"] / 1e3
    ppl = agg["pairs"] / agg["launches"]
    # algorithmic ALU work per pair: one exponential and one add (the 4-wide contraction
    # runs on the matrix cores: 8 flop per pair, 19.7e12 pairs/s at the FP32 MFMA peak,
    # above the ALU ceiling); issue slots of one lane operation each
    slots = TRANS_SLOTS + 1
    peak = VALU_LANE_PEAK / 1e12
    ach = slots * ppl / kern_s / 1e12
    out = {"metric": "Gpair/s of the log-sum-exp softmin (full S_eps solve, "
                     f"{n} x {n} 3-D clouds)",
           "value": round(agg["pairs"] / agg["dt"] / 1e9, 3), "unit": "Gpair/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(agg["dt"] / args.steps * 1e3, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"3-D Gaussian blob clouds n=m={n}, cost |x-y|^2/2, "
                                  "blur 0.01, balanced, scaling 0.9, dense",
                      "iterations": st["iters"]},
           "S": agg["S"], "softmin_kernel_gpair_s": round(ppl / kern_s / 1e9, 3),
           "roofline": {"bound": "alu", "achieved": round(ach, 3), "peak": round(peak, 2),
                        "unit": "Tslot/s", "frac": round(ach / peak, 4), "traffic": None,
                        "slots_per_pair": slots, "avg_launch_ms": round(kern_s * 1e3, 4),
                        "kernel": "k_softmin_f32<4>"}}
    print(json.dumps(out), flush=True)
    return 0


def bench_blobs2k(args, skh, synth):
    """The small 3-D case: 2000 x 2000 Gaussian blobs, blur 0.01, scaling 0.5, balanced,
    dense FP32, the Algorithm's schedule; latency-bound on the GPU (us per iteration),
    with the FP64 oracle's full solve timed on the host at one thread and all cores."""
    import torch

    import oracle
    x, a, y, b = synth.blob_pair(2000, seed=0)
    X, A, Y, B = (torch.as_tensor(v).cuda() for v in (x, a, y, b))
    kw = dict(blur=0.01, reach=None, scaling=0.5, potentials=True, timing=True,
              precision="fp32")
    agg = solve_steps(skh, X, A, Y, B, args.steps, args.warmup, "2k blobs", **kw)
    st = agg["stats"]
    t_gpu = agg["dt"] / args.steps
    cpu = {}
    threads_all = oracle.num_threads()
    for label, k in (("one_core", 1), ("all_cores", threads_all)):
        oracle.set_num_threads(k)
        t0 = time.perf_counter()
        Sr, r = oracle.sinkhorn_divergence(x, a, y, b, 0.01, None, scaling=0.5)
        cpu[label] = {"s": round(time.perf_counter() - t0, 4), "threads": k, "S": Sr,
                      "iters": r["iters"]}
        print(f"[bench] oracle full solve ({label}, {k} threads): {cpu[label]['s']:.3f} s",
              file=sys.stderr, flush=True)
    oracle.set_num_threads(threads_all)
    out = {"metric": "time to S_eps, 2000 x 2000 3-D blobs (the Algorithm's schedule)",
           "value": round(t_gpu, 6), "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(t_gpu * 1e3, 4),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": "3 Gaussian blobs per cloud, n=m=2000, blur 0.01, scaling "
                                  "0.5, balanced, dense FP32", "iterations": st["iters"]},
           "S": agg["S"], "us_per_iteration": round(t_gpu / st["iters"] * 1e6, 2),
           "solve_gpair_s": round(agg["pairs"] / agg["dt"] / 1e9, 3),
           "S_rel_diff_vs_oracle": abs(agg["S"] - cpu["one_core"]["S"]) / abs(cpu["one_core"]["S"]),
           "cpu_baseline": {"value": cpu["all_cores"]["s"], "unit": "s",
                            "cores": threads_all, "kind": "oracle", "cpu_model": cpu_model(),
                            "sample": "the whole FP64 oracle solve (same inputs and schedule)",
                            "one_core_s": cpu["one_core"]["s"]}}
    print(json.dumps(out), flush=True)
    return 0


def bench_warmstart_eval(args, skh, synth):
    """What the learned warm start gains on fresh pairs (seeds disjoint from training):
    per pair the cold BF16 multiscale solve, the zero-start ablation at the network's
    schedule (same clustering, start scale and checks, starting values 0) and the
    network's start, all converged to the same marginal error; five 1M x 1M pairs
    (200 bundles) and eight 100k x 100k pairs (50-200 bundles)."""
    import numpy as np
    import torch
    from paper_2107_02010_amd.warm_start import (DEFAULT_CHECKPOINT, WarmStartNet,
                                                 sinkhorn_divergence_warm)
    net = WarmStartNet.load(DEFAULT_CHECKPOINT, "cuda:0")
    kw = dict(reach=20.0, tol=1e-4, check_every=1, max_iters=20000, multiscale=True,
              timing=True)
    rng = np.random.default_rng(900)
    plan = [(1_000_000, 200, 900001 + k) for k in range(5)]
    plan += [(100_000, int(rng.integers(50, 201)), 900101 + k) for k in range(8)]
    rows = []
    for n, nb, seed in plan:
        print(f"[bench] pair n={n} bundles={nb} seed={seed}: generating", file=sys.stderr,
              flush=True)
        x, a, y, b = synth.fiber_pair(n, nb, seed=seed)
        X, A, Y, B = (torch.as_tensor(v).cuda() for v in (x, a, y, b))
        legs = {"cold": lambda: skh.sinkhorn_divergence(X, A, Y, B, blur=1.0, scaling=0.9,
                                                        precision="bf16x3", potentials=True,
                                                        **kw),
                "zero_start": lambda: sinkhorn_divergence_warm(
                    net, X, A, Y, B, 1.0, scaling=0.9, precision="bf16x3", start="zero", **kw),
                "network": lambda: sinkhorn_divergence_warm(
                    net, X, A, Y, B, 1.0, scaling=0.9, precision="bf16x3", **kw)}
        row = {"n": n, "bundles": nb, "seed": seed}
        for name, fn in legs.items():
            fn()  # warm-up (workspace, clustering caches)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S, _, st = fn()
            torch.cuda.synchronize()
            row[name] = {"s": round(time.perf_counter() - t0, 4), "iters": st["iters"],
                         "S": S, "fallback": st.get("warm_fallback", 0)}
        print(f"[bench]   cold {row['cold']['iters']} it {row['cold']['s']:.3f} s | zero start "
              f"{row['zero_start']['iters']} it {row['zero_start']['s']:.3f} s | network "
              f"{row['network']['iters']} it {row['network']['s']:.3f} s", file=sys.stderr,
              flush=True)
        rows.append(row)
        del X, A, Y, B
        torch.cuda.empty_cache()

    def summary(sel):
        r = [q for q in rows if sel(q)]
        return {"pairs": len(r),
                "iters_cold": sum(q["cold"]["iters"] for q in r),
                "iters_zero_start": sum(q["zero_start"]["iters"] for q in r),
                "iters_network": sum(q["network"]["iters"] for q in r),
                "s_cold": round(sum(q["cold"]["s"] for q in r), 4),
                "s_zero_start": round(sum(q["zero_start"]["s"] for q in r), 4),
                "s_network": round(sum(q["network"]["s"] for q in r), 4),
                "max_S_rel_diff_network_vs_cold": max(
                    abs(q["network"]["S"] - q["cold"]["S"]) / abs(q["cold"]["S"]) for q in r)}
    out = {"metric": "learned warm start on fresh fibre pairs: iterations and time to S "
                     "(cold, zero start at the network's schedule, network)",
           "value": summary(lambda q: q["n"] == 1_000_000)["s_network"], "unit": "s",
           "n_gpus": 1, "steps": 1, "warmup": 1, "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3", "data": "synthetic",
           "config": {"workload": "fresh fibre pairs (seeds 900001-900005 at 1M x 1M, 200 "
                                  "bundles; 900101-900108 at 100k x 100k, 50-200 bundles), "
                                  "reach 20 mm, blur 1 mm, multiscale BF16, marginal error "
                                  "1e-4 checked every iteration"},
           "at_1m": summary(lambda q: q["n"] == 1_000_000),
           "at_100k": summary(lambda q: q["n"] == 100_000), "pairs": rows}
    print(json.dumps(out), flush=True)
    return 0


def bench_barycenter(args, skh, synth):
    """One Wasserstein-barycenter descent step (Section 3, track density atlas): 10 density
    maps on a 128^3 grid (~200k-270k voxels each), a 200k-point support, blur 1 voxel,
    balanced; the maps' cross loops as one batched solve against one solve per map."""
    import torch
    from paper_2107_02010_amd.barycenter import Barycenter
    print("[bench] generating 10 density maps (128^3)", file=sys.stderr, flush=True)
    maps = synth.density_maps(10, seed=11)
    x0, a = synth.barycenter_support(maps, 200_000, seed=12)
    ym = [(torch.as_tensor(c).cuda(), torch.as_tensor(w).cuda()) for c, w in maps]
    X, A = torch.as_tensor(x0).cuda(), torch.as_tensor(a).cuda()
    res = {}
    for leg, batched, ms in (("batched", True, False), ("per_map", False, False),
                             ("per_map_multiscale", False, True)):
        B = Barycenter(A, ym, blur=1.0, scaling=0.9, x0=X, batched=batched, multiscale=ms)
        B._setup(X)  # the maps' self vectors: once for the whole descent, outside the step
        dt, (x1, S, _) = _timed(lambda: B.step(X), args.steps, args.warmup)
        res[leg] = {"s_per_step": round(dt, 4), "mean_S": S}
        print(f"[bench] barycenter step ({leg}): {dt:.3f} s", file=sys.stderr, flush=True)
    # a 10-step descent, every step after the first started from the previous step's
    # vectors with the scale list [3, 3 q, ..., blur] (batched cross loops)
    B = Barycenter(A, ym, blur=1.0, scaling=0.9, x0=X, batched=True, start_scale=3.0)
    B._setup(X)
    x, hist, times = X, [], []
    for k in range(10):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, S, _ = B.step(x)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        hist.append(S)
        print(f"[bench] warm-started descent step {k + 1}/10: S={S:.8g} {times[-1]:.3f} s",
              file=sys.stderr, flush=True)
    res["descent_warm"] = {"start_scale": 3.0, "s_first_step": round(times[0], 4),
                           "s_per_warm_step": round(sum(times[1:]) / 9, 4),
                           "s_total_10_steps": round(sum(times), 4), "S_history": hist}
    m_total = sum(len(c) for c, _ in maps)
    out = {"metric": "time per barycenter step, 10 density maps (128^3), 200k support points",
           "value": res["batched"]["s_per_step"], "unit": "s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": round(res["batched"]["s_per_step"] * 1e3, 3),
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic",
           "config": {"workload": f"Wasserstein barycenter step, 10 maps ({m_total} voxels in "
                                  "total), 200000 support points, blur 1 voxel, reach none, "
                                  "scaling 0.9; self loop of the support per step, cross loops "
                                  "of all maps, 10 gradients"},
           "batched": res["batched"], "per_map": res["per_map"],
           "per_map_multiscale": res["per_map_multiscale"],
           "descent_warm": res["descent_warm"],
           "speedup_batched": round(res["per_map"]["s_per_step"] / res["batched"]["s_per_step"], 3),
           "S_rel_diff_multiscale": abs(res["per_map_multiscale"]["mean_S"] - res["batched"]["mean_S"])
                                    / abs(res["batched"]["mean_S"])}
    print(json.dumps(out), flush=True)
    return 0


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="bf16x3", choices=["fp32", "bf16x3"])
    ap.add_argument("--workload", default="fibers1m",
                    choices=["fibers1m", "multiscale1m", "fibers200k", "grad200k", "labels200k",
                             "labels250k", "pcost200k", "blobs200k", "barycenter10",
                             "warmstart_eval", "valu_probe", "blobs2k"])
    ap.add_argument("--legs", default="chosen,plain,bf16_cold,zero_start,dense200k,cpu",
                    help="fibers1m: comma-separated legs to run (chosen, plain, bf16_cold, "
                         "zero_start, dense200k, cpu)")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain FP32 comparison solve")
    ap.add_argument("--n", type=int, default=200_000)
    ap.add_argument("--bundles", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--check-every", type=int, default=1,
                    help="multiscale1m: iterations between marginal-error checks at blur")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES bytes (5 times), "
                         "to scale the HBM byte counters of a profiler")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the solver is a "
              "single-device library; sharding across GPUs is described in the design notes, "
              "not built.", file=sys.stderr)
        return 2

    import torch

    if args.copy_calibration:
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n * 4, "copies": 5}), flush=True)
        return 0

    import paper_2107_02010_amd as skh
    import synth

    if args.workload in ("fibers1m", "multiscale1m"):
        return bench_fibers1m(args, skh, synth)
    if args.workload == "grad200k":
        return bench_gradients(args, skh, synth)
    if args.workload in ("labels200k", "labels250k"):
        return bench_labels(args, skh, synth)
    if args.workload == "blobs2k":
        return bench_blobs2k(args, skh, synth)
    if args.workload == "valu_probe":
        import subprocess
        exe = os.path.join(ROOT, "paper_2107_02010_amd", "valu_probe")
        if not os.path.exists(exe):
            print("valu_probe is missing: build it with python -m paper_2107_02010_amd.build",
                  file=sys.stderr)
            return 1
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        sys.stdout.write(r.stdout)
        return r.returncode
    if args.workload == "warmstart_eval":
        return bench_warmstart_eval(args, skh, synth)
    if args.workload == "blobs200k":
        return bench_blobs(args, skh, synth)
    if args.workload == "pcost200k":
        return bench_pcost(args, skh, synth)
    if args.workload == "barycenter10":
        return bench_barycenter(args, skh, synth)
    print(f"[bench] generating {args.n} x {args.n} fibre clouds", file=sys.stderr, flush=True)
    x, a, y, b = synth.fiber_pair(args.n, args.bundles, seed=0)
    dev = torch.device("cuda:0")
    X, A, Y, B = (torch.as_tensor(v).to(dev) for v in (x, a, y, b))
    kw = dict(blur=1.0, reach=None, scaling=0.9, potentials=True, timing=True)
    agg = solve_steps(skh, X, A, Y, B, args.steps, args.warmup, args.precision,
                      precision=args.precision, **kw)
    rl, kern = roofline(agg, args.precision, "fibers200k")
    st = agg["stats"]
    out = {
        "metric": "Gpair/s of log-sum-exp softmin (full S_eps solve, 200k x 200k 60-D fibres)",
        "value": round(agg["pairs"] / agg["dt"] / 1e9, 3),
        "unit": "Gpair/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(agg["dt"] / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "bf16x3",
        "data": "synthetic",
        "config": {"workload": f"fibre clouds n=m={args.n}, 60-D (20 points x 3, /sqrt(20)), "
                               f"{args.bundles} Bezier bundles, jitter 2 mm, blur 1 mm, "
                               "reach none, scaling 0.9, dense (no multiscale)",
                   "precision": args.precision, "iterations": st["iters"],
                   "softmins_per_iteration": 4},
        "S": agg["S"],
        "softmin_kernel_gpair_s": round(kern, 3),
        "roofline": rl,
    }
    if args.precision != "fp32" and not args.no_plain:
        plain = solve_steps(skh, X, A, Y, B, 1, 0, "plain fp32", precision="fp32", **kw)
        prl, pk = roofline(plain, "fp32", "fibers200k")
        out["plain_fp32"] = {"value": round(plain["pairs"] / plain["dt"] / 1e9, 3),
                             "ms_per_step": round(plain["dt"] * 1e3, 3), "S": plain["S"],
                             "softmin_kernel_gpair_s": round(pk, 3), "roofline": prl}
        out["S_rel_diff_vs_fp32"] = abs(agg["S"] - plain["S"]) / abs(plain["S"])
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a row sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(x, y, b)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
