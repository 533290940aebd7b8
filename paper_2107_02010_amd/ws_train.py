"""Data generation, training and start-scale selection of the learned warm start.

    python -m paper_2107_02010_amd.ws_train --pairs 256 --val 16 --out ws_fibers.safetensors

1. Data: random fibre-cloud pairs (N log-uniform in [n_min, n_max], bundles
   uniform in [b_min, b_max], fresh spine seeds per pair), each solved cold in
   converged mode by the library; the example is the pair's cluster tokens and
   the cluster means of the converged duals divided by blur^2.
2. Training: Adam on the weighted MSE, batches of whole pairs, FP32 kernels.
3. Start scale: on the validation pairs, the number of schedule steps s above
   blur (start_scale = blur / q^s) with the least solve time.

Every solve, token, forward and backward step runs in libskh; this script
only draws the random pair parameters and loops.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

from . import sinkhorn_divergence  # noqa: E402
from .warm_start import TokenBatch, WarmStartNet, make_example, sinkhorn_divergence_warm  # noqa: E402


def solve_kw(args):
    return dict(reach=args.reach, scaling=args.scaling, tol=args.tol, check_every=5,
                max_iters=args.max_iters, multiscale=True, precision=args.precision)


def pair_plan(args, count, seed0):
    """(n, bundles, seed) of each pair: N log-uniform, bundles uniform, fresh seeds."""
    rng = np.random.default_rng(seed0)
    plan = []
    for i in range(count):
        n = int(round(math.exp(rng.uniform(math.log(args.n_min), math.log(args.n_max)))))
        bundles = int(rng.integers(args.b_min, args.b_max + 1))
        plan.append((n, bundles, seed0 * 1000 + 7 * i))
    return plan


def _make_pair(spec):
    """Host-side generation of one pair (runs in a worker process, no GPU)."""
    n, bundles, seed = spec
    x, a, y, b = synth.fiber_pair(n, bundles, seed)
    return spec, x, a, y, b


def generate(args, pool, count, seed0, label):
    out = []
    dev = torch.device("cuda")
    t = lambda v: torch.as_tensor(v, dtype=torch.float32, device=dev)
    plan = pair_plan(args, count, seed0)
    pairs = pool.imap(_make_pair, plan) if pool is not None else map(_make_pair, plan)
    for i, ((n, nb, seed), x, a, y, b) in enumerate(pairs):
        x, a, y, b = t(x), t(a), t(y), t(b)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ex, S, st = make_example(x, a, y, b, blur=args.blur, **solve_kw(args))
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ex = {k: (v.cpu() if torch.is_tensor(v) else v) for k, v in ex.items()}
        ex.update(n=n, bundles=nb, S=S, iters=st["iters"], coarse=st["coarse_iters"],
                  converged=st["converged"], seconds=dt, seed=seed)
        out.append(ex)
        print(f"[{label} {i + 1}/{count}] n={n} bundles={nb} S={S:.6g} iters={st['iters']} "
              f"coarse={st['coarse_iters']} conv={st['converged']} {dt:.2f}s", flush=True)
    return out


def to_dev(examples, idx):
    ex = [examples[i] for i in idx]
    dev = torch.device("cuda")
    b = TokenBatch.concat([{k: (v.to(dev) if torch.is_tensor(v) else v) for k, v in e.items()}
                           for e in ex])
    return b


def train(net, data, val, args):
    rng = np.random.default_rng(args.seed + 1)
    vb = to_dev(val, range(len(val))) if val else None
    for step in range(1, args.steps + 1):
        idx = rng.choice(len(data), size=min(args.batch, len(data)), replace=False)
        lr = args.lr * 0.5 * (1 + math.cos(math.pi * (step - 1) / args.steps))
        loss = net.train_step(to_dev(data, idx), lr)
        if step % args.log_every == 0 or step == 1 or step == args.steps:
            msg = f"[train {step}/{args.steps}] loss={loss:.5g} lr={lr:.3g}"
            if vb is not None:
                msg += f" val={net.loss_grad(vb)[0]:.5g}"
            print(msg, flush=True)


def pick_start_steps(net, val, args):
    """Times warm solves of the validation pairs for each candidate s (same stopping
    rule as the cold solves that made the examples); reports the S difference."""
    best = None
    table = {}
    dev = torch.device("cuda")
    t = lambda v: torch.as_tensor(v, dtype=torch.float32, device=dev)
    clouds = [tuple(t(v) for v in synth.fiber_pair(e["n"], e["bundles"], e["seed"])) for e in val]
    for s in args.start_candidates:
        tot_t, tot_it, dS = 0.0, 0, 0.0
        for e, (x, a, y, b) in zip(val, clouds):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            S, _, st = sinkhorn_divergence_warm(net, x, a, y, b, args.blur, start_steps=s,
                                                **solve_kw(args))
            torch.cuda.synchronize()
            tot_t += time.perf_counter() - t0
            tot_it += st["iters"]
            dS = max(dS, abs(S - e["S"]) / abs(e["S"]))
        cold_t = sum(e["seconds"] for e in val)
        table[s] = dict(seconds=tot_t, iters=tot_it, max_rel_dS=dS)
        print(f"[start] s={s} warm {tot_t:.2f}s {tot_it} iters (cold {cold_t:.2f}s "
              f"{sum(e['iters'] for e in val)} iters), max |dS|/S = {dS:.2e}", flush=True)
        if best is None or tot_t < table[best]["seconds"]:
            best = s
    return best, table


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=256)
    ap.add_argument("--val", type=int, default=16)
    ap.add_argument("--n-min", type=int, default=20000)
    ap.add_argument("--n-max", type=int, default=200000)
    ap.add_argument("--b-min", type=int, default=50)
    ap.add_argument("--b-max", type=int, default=200)
    ap.add_argument("--blur", type=float, default=1.0)
    ap.add_argument("--reach", type=float, default=20.0)
    ap.add_argument("--scaling", type=float, default=0.9)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--max-iters", type=int, default=5000)
    ap.add_argument("--precision", default="bf16x3")
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--log-every", type=int, default=250)
    ap.add_argument("--start-candidates", type=int, nargs="+", default=[0, 2, 4, 8, 12])
    ap.add_argument("--data", default=None, help="cache of generated examples (.pt, tensors only)")
    ap.add_argument("--workers", type=int, default=8, help="host processes generating pairs")
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)
    # the generator pool starts before this process touches the GPU
    import multiprocessing as mp
    pool = mp.get_context("spawn").Pool(args.workers) if args.workers > 1 else None

    if args.data and os.path.exists(args.data):
        blob = torch.load(args.data, weights_only=True)
        data, val = blob["train"], blob["val"]
        print(f"[data] loaded {len(data)} + {len(val)} examples from {args.data}", flush=True)
    else:
        data = generate(args, pool, args.pairs, args.seed + 100, "gen")
        val = generate(args, pool, args.val, args.seed + 200, "val")
        if args.data:
            torch.save({"train": data, "val": val}, args.data)
    if pool is not None:
        pool.close()
        pool.join()
    net = WarmStartNet("cuda", seed=args.seed)
    train(net, data, val, args)
    best, table = pick_start_steps(net, val, args)
    net.meta.update(start_steps=best, blur=args.blur, reach=args.reach, scaling=args.scaling,
                    tol=args.tol, pairs=len(data), n_range=[args.n_min, args.n_max],
                    start_table={str(k): v for k, v in table.items()})
    net.save(args.out)
    print(json.dumps({"out": args.out, "start_steps": best, "table": table}), flush=True)


if __name__ == "__main__":
    main()
