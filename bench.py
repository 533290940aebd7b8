#!/usr/bin/env python3
"""Benchmark of the Sinkhorn divergence hot path on one MI355X.

A step is one full S_eps solve (every row of the hot path: bounding box and
scale list, packing, the averaged symmetric loop of four softmins per
iteration, the merge/averaging kernel, and the FP64 value of eq. (6)) on a
synthetic fibre workload: n = m = 200,000 fibres, 20 points each flattened to
60-D and scaled by 1/sqrt(20), 50 bundles, uniform weights, blur = 1 mm,
reach = none (balanced), scaling 0.9.  Inputs are resident in HBM before the
timed region.

Prints one JSON line:
  value       = softmin point pairs evaluated / wall time of the timed steps (Gpair/s)
  roofline    = the softmin kernel's algorithmic MFMA flops per launch over its
                average launch time (HIP events on the library's stream)
  cpu_baseline= the FP64 oracle's softmin on a bounded row sample of the same
                workload, on the host cores

    python bench.py [--steps K] [--warmup W] [--precision fp32|bf16x3] [--n N]
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
KERNEL_SRC = os.path.join(ROOT, "paper_2107_02010_amd", "csrc", "softmin.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "softmin_fiber200k_traffic.txt")


def kernel_hash() -> str:
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


def read_traffic(precision: str):
    """HBM bytes per softmin launch from the committed rocprofv3 PMC summary, or
    None when it is absent or was taken on another version of the kernel."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    m = re.search(r"kernel_sha256_16:\s*([0-9a-f]+)", txt)
    t = re.search(rf"bytes_per_launch\[{precision}\]:\s*([0-9.eE+]+)", txt)
    if not m or not t or m.group(1) != kernel_hash():
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


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawTextHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16x3"])
    ap.add_argument("--n", type=int, default=200_000)
    ap.add_argument("--bundles", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the solver is a "
              "single-device library; sharding across GPUs is described in the design notes, "
              "not built.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2107_02010_amd as skh
    import synth

    print(f"[bench] generating {args.n} x {args.n} fibre clouds", file=sys.stderr, flush=True)
    x, a, y, b = synth.fiber_pair(args.n, args.bundles, seed=0)
    dev = torch.device("cuda:0")
    X, A, Y, B = (torch.as_tensor(v).to(dev) for v in (x, a, y, b))
    kw = dict(blur=1.0, reach=None, scaling=0.9, precision=args.precision, potentials=True,
              timing=True)
    for k in range(args.warmup):
        skh.sinkhorn_divergence(X, A, Y, B, **kw)
        print(f"[bench] warmup {k + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pairs = 0.0
    ms_softmin = 0.0
    launches = 0
    S = None
    for k in range(args.steps):
        S, _, st = skh.sinkhorn_divergence(X, A, Y, B, **kw)
        pairs += st["pairs"]
        ms_softmin += st["ms_softmin"]
        launches += st["softmin_launches"]
        print(f"[bench] step {k + 1}/{args.steps}: S={S:.8g} iters={st['iters']} "
              f"{st['ms_total']:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = pairs / dt / 1e9
    pairs_per_launch = pairs / launches
    avg_launch_s = ms_softmin / launches / 1e3
    achieved = FLOP_PER_PAIR[args.precision] * pairs_per_launch / avg_launch_s / 1e12
    peak = PEAK_TFLOPS[args.precision]
    traffic = read_traffic(args.precision)
    out = {
        "metric": "Gpair/s of log-sum-exp softmin (full S_eps solve, 200k x 200k 60-D fibres)",
        "value": round(value, 3),
        "unit": "Gpair/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt / args.steps * 1e3, 3),
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
        "S": S,
        "softmin_kernel_gpair_s": round(pairs_per_launch / avg_launch_s / 1e9, 3),
        "roofline": {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak,
                     "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                     "traffic": traffic,
                     "flop_per_pair": FLOP_PER_PAIR[args.precision],
                     "avg_launch_ms": round(avg_launch_s * 1e3, 4),
                     "kernel": "k_softmin_f32<64>" if args.precision == "fp32" else "k_softmin_bf16<64>"},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the FP64 oracle on a row sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(x, y, b)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
