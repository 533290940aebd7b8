"""Learned warm start of the symmetric Sinkhorn loop.

Not part of the paper's method: the Algorithm (eps-scaling from the largest
scale) stays the cold start, the fallback and what decides the fixed point.  A
set encoder reads one token per K-means cluster of each cloud (the coarse scale
of Section 2's coarse-to-fine strategy) and predicts the cluster's mean cross
dual and self dual, divided by blur^2.  Broadcast to the points, these are the
starting values of a solve whose schedule begins at ``start_scale`` instead of
the diameter; only the number of iterations changes, the stopping rule and the
fixed point are those of the cold solve.

Every arithmetic step (tokens, network forward and backward, Adam, targets,
broadcast) runs in libskh's kernels; this module batches tensors and calls them.
"""
from __future__ import annotations

import ctypes
import json
import math
import os

import torch

from . import _lib
from . import _Ctx, _as_points, _as_vec, _ptr, sinkhorn_divergence

N_PARAMS = _lib.SKH_WS_N_PARAMS
# network trained by ws_train on fibre pairs (blur 1 mm, reach 20 mm, scaling 0.9)
DEFAULT_CHECKPOINT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                                  "ws_fibers.safetensors")
WIDTH = _lib.SKH_WS_WIDTH
IN = _lib.SKH_WS_IN
_SHAPES = [(WIDTH, IN), (WIDTH,), (WIDTH, WIDTH), (WIDTH,), (WIDTH, WIDTH), (WIDTH,),
           (WIDTH, 3 * WIDTH), (WIDTH,), (2, WIDTH), (2,)]


def init_theta(seed: int) -> torch.Tensor:
    """He initialisation (N(0, 2 / fan_in) weights, zero biases), flat FP32 on the CPU."""
    gen = torch.Generator().manual_seed(int(seed))
    parts = []
    for shape in _SHAPES:
        if len(shape) == 2:
            parts.append(torch.randn(shape, generator=gen, dtype=torch.float64).mul_(
                math.sqrt(2.0 / shape[1])).reshape(-1))
        else:
            parts.append(torch.zeros(shape, dtype=torch.float64))
    return torch.cat(parts).to(torch.float32)


class TokenBatch:
    """Tokens of several cloud pairs, in order pair 0 alpha, pair 0 beta, pair 1 alpha, ..."""

    def __init__(self, tokens, w, seg, target=None):
        self.tokens = tokens.contiguous()
        self.w = w.contiguous()
        self.seg = [int(s) for s in seg]
        self.target = None if target is None else target.contiguous()

    @property
    def n_pairs(self) -> int:
        return (len(self.seg) - 1) // 2

    @staticmethod
    def concat(examples):
        """examples: dicts with tokens, w, kx, ky (and target); one pair each."""
        seg = [0]
        for e in examples:
            seg += [seg[-1] + e["kx"], seg[-1] + e["kx"] + e["ky"]]
        tok = torch.cat([e["tokens"] for e in examples])
        w = torch.cat([e["w"] for e in examples])
        tgt = None
        if all("target" in e for e in examples):
            tgt = torch.cat([e["target"] for e in examples])
        return TokenBatch(tok, w, seg, tgt)

    def _seg_arg(self):
        return (ctypes.c_int32 * len(self.seg))(*self.seg)


class WarmStartNet:
    """Network parameters and Adam state on one device."""

    def __init__(self, device="cuda", seed: int = 0, theta=None, meta=None):
        device = torch.device(device)
        self.theta = (init_theta(seed) if theta is None else theta.to(torch.float32)).to(device)
        if self.theta.numel() != N_PARAMS:
            raise ValueError(f"theta must have {N_PARAMS} values")
        self.theta = self.theta.contiguous()
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.step = 0
        self.meta = dict(seed=int(seed), start_steps=5, blur=1.0)
        if meta:
            self.meta.update(meta)

    @property
    def device(self):
        return self.theta.device

    def forward(self, batch: TokenBatch, precision: str = "bf16x3") -> torch.Tensor:
        """Predictions (T, 2): per cluster (cross dual, self dual) / blur^2."""
        prec = {"fp32": _lib.SKH_FP32, "bf16x3": _lib.SKH_BF16_SPLIT, "bf16": _lib.SKH_BF16_SPLIT}
        T = batch.seg[-1]
        out = torch.empty(T, 2, dtype=torch.float32, device=self.device)
        ctx = _Ctx.get(self.device)
        rc = _lib.load().skh_ws_forward(ctx, _ptr(self.theta), batch.n_pairs, batch._seg_arg(),
                                        _ptr(batch.tokens), _ptr(batch.w), prec[precision], _ptr(out))
        _lib.check(rc, ctx)
        return out

    def loss_grad(self, batch: TokenBatch, theta=None):
        """(loss, gradient) of the weighted MSE on a batch with targets (FP32)."""
        if batch.target is None:
            raise ValueError("batch has no targets")
        th = self.theta if theta is None else theta.contiguous()
        grad = torch.empty(N_PARAMS, dtype=torch.float32, device=self.device)
        loss = ctypes.c_double()
        ctx = _Ctx.get(self.device)
        rc = _lib.load().skh_ws_loss_grad(ctx, _ptr(th), batch.n_pairs, batch._seg_arg(),
                                          _ptr(batch.tokens), _ptr(batch.w), _ptr(batch.target),
                                          ctypes.byref(loss), _ptr(grad))
        _lib.check(rc, ctx)
        return loss.value, grad

    def adam(self, grad, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8):
        self.step += 1
        ctx = _Ctx.get(self.device)
        rc = _lib.load().skh_ws_adam(ctx, N_PARAMS, _ptr(self.theta), _ptr(grad), _ptr(self.m),
                                     _ptr(self.v), self.step, float(lr), float(beta1), float(beta2),
                                     float(eps))
        _lib.check(rc, ctx)

    def train_step(self, batch: TokenBatch, lr: float) -> float:
        loss, grad = self.loss_grad(batch)
        self.adam(grad, lr)
        return loss

    # checkpoint: parameters, Adam moments, step and metadata (safetensors, no pickle)
    def save(self, path: str):
        from safetensors.torch import save_file
        meta = dict(self.meta, step=self.step)
        save_file({"theta": self.theta.cpu(), "m": self.m.cpu(), "v": self.v.cpu()}, path,
                  metadata={"skh_ws": json.dumps(meta)})

    @staticmethod
    def load(path: str, device="cuda") -> "WarmStartNet":
        from safetensors import safe_open
        with safe_open(path, framework="pt") as fh:
            meta = json.loads(fh.metadata()["skh_ws"])
            theta, m, v = fh.get_tensor("theta"), fh.get_tensor("m"), fh.get_tensor("v")
        net = WarmStartNet(device, seed=meta.get("seed", 0), theta=theta, meta=meta)
        net.m.copy_(m)
        net.v.copy_(v)
        net.step = int(meta.get("step", 0))
        return net


def cluster_tokens(x, a, y, b, n_clusters: int = 0, kmeans_iters: int = 10) -> dict:
    """Tokens of the pair (alpha, beta) and the cluster label of every point."""
    x, y = _as_points(x, "x"), _as_points(y, "y")
    n, m, d = x.shape[0], y.shape[0], x.shape[1]
    a = _as_vec(a, n, "a", x.device)
    b = _as_vec(b, m, "b", x.device)
    dev = x.device
    kcap = lambda k_, N: min(k_, 4096, N) if k_ > 0 else min(math.ceil(math.sqrt(N)), 4096)
    cap = kcap(n_clusters, n) + kcap(n_clusters, m) + 2
    tokens = torch.empty(cap, IN, dtype=torch.float32, device=dev)
    w = torch.empty(cap, dtype=torch.float32, device=dev)
    lx = torch.empty(n, dtype=torch.int32, device=dev)
    ly = torch.empty(m, dtype=torch.int32, device=dev)
    k = (ctypes.c_int32 * 2)()
    ctx = _Ctx.get(dev)
    rc = _lib.load().skh_ws_tokens(ctx, _ptr(x), _ptr(a), n, _ptr(y), _ptr(b), m, d,
                                   int(n_clusters), int(kmeans_iters), cap, _ptr(tokens), _ptr(w),
                                   _ptr(lx), _ptr(ly), k)
    _lib.check(rc, ctx)
    kx, ky = int(k[0]), int(k[1])
    return dict(tokens=tokens[:kx + ky], w=w[:kx + ky], labels_x=lx, labels_y=ly, kx=kx, ky=ky)


def cluster_targets(labels, k: int, w, pot_cross, pot_self, scale: float) -> torch.Tensor:
    """(k, 2): scale x the w-weighted mean of (pot_cross, pot_self) over each cluster."""
    n = labels.numel()
    out = torch.empty(k, 2, dtype=torch.float32, device=labels.device)
    ctx = _Ctx.get(labels.device)
    rc = _lib.load().skh_ws_targets(ctx, _ptr(labels), n, int(k), _ptr(w), _ptr(pot_cross),
                                    _ptr(pot_self), float(scale), _ptr(out))
    _lib.check(rc, ctx)
    return out


def expand(labels, k: int, pred, scale: float):
    """Starting values of one cloud: scale x pred[label] (cross, self)."""
    n = labels.numel()
    pc = torch.empty(n, dtype=torch.float32, device=labels.device)
    ps = torch.empty(n, dtype=torch.float32, device=labels.device)
    ctx = _Ctx.get(labels.device)
    rc = _lib.load().skh_ws_expand(ctx, _ptr(labels), n, int(k), _ptr(pred.contiguous()),
                                   float(scale), _ptr(pc), _ptr(ps))
    _lib.check(rc, ctx)
    return pc, ps


def make_example(x, a, y, b, blur: float, n_clusters: int = 0, kmeans_iters: int = 10, **solve_kw):
    """One training pair: a cold converged solve, its cluster tokens and the
    cluster-mean dual targets (divided by blur^2).  Returns (example, S, stats)."""
    S, pot, st = sinkhorn_divergence(x, a, y, b, blur=blur, potentials=True, **solve_kw)
    tk = cluster_tokens(x, a, y, b, n_clusters, kmeans_iters)
    inv = 1.0 / (blur * blur)
    ta = cluster_targets(tk["labels_x"], tk["kx"], _as_vec(a, x.shape[0], "a", x.device),
                         pot["f"], pot["p"], inv)
    tb = cluster_targets(tk["labels_y"], tk["ky"], _as_vec(b, y.shape[0], "b", y.device),
                         pot["g"], pot["q"], inv)
    ex = dict(tokens=tk["tokens"], w=tk["w"], kx=tk["kx"], ky=tk["ky"],
              target=torch.cat([ta, tb]))
    return ex, S, st


def predict_potentials(net: WarmStartNet, x, a, y, b, blur: float, precision: str = "bf16x3",
                       n_clusters: int = 0, kmeans_iters: int = 10, return_labels: bool = False):
    """Starting (f, g, p, q) for the pair from the network's cluster predictions (and the
    cluster labels of the two clouds when return_labels)."""
    tk = cluster_tokens(x, a, y, b, n_clusters, kmeans_iters)
    batch = TokenBatch(tk["tokens"], tk["w"], [0, tk["kx"], tk["kx"] + tk["ky"]])
    pred = net.forward(batch, precision)
    s2 = blur * blur
    f, p = expand(tk["labels_x"], tk["kx"], pred[:tk["kx"]], s2)
    g, q = expand(tk["labels_y"], tk["ky"], pred[tk["kx"]:], s2)
    if return_labels:
        return (f, g, p, q), (tk["labels_x"], tk["labels_y"])
    return f, g, p, q


def sinkhorn_divergence_warm(net: WarmStartNet, x, a, y, b, blur: float, scaling: float = 0.9,
                             start_steps=None, net_precision: str = "bf16x3",
                             n_clusters: int = 0, kmeans_iters: int = 10, start: str = "network",
                             **kw):
    """S_eps(alpha, beta) with the learned warm start: predicted starting values and a
    schedule from start_scale = blur / scaling^start_steps down to blur.  Non-finite
    predictions make the solver run cold (stats["warm_fallback"] = 1).  Returns
    (S, potentials, stats) like sinkhorn_divergence(..., potentials=True).

    start="zero" is the ablation of the network: the same clustering, the same shortened
    schedule and the same checked start, but every starting value 0 instead of the
    prediction (net may be None)."""
    if start not in ("network", "zero"):
        raise ValueError("start must be 'network' or 'zero'")
    if start == "network":
        s = net.meta.get("start_steps", 5) if start_steps is None else start_steps
        init, labels = predict_potentials(net, x, a, y, b, blur, net_precision, n_clusters,
                                          kmeans_iters, return_labels=True)
    else:
        if start_steps is None:
            s = net.meta.get("start_steps", 5) if net is not None else 5
        else:
            s = start_steps
        tk = cluster_tokens(x, a, y, b, n_clusters, kmeans_iters)
        labels = (tk["labels_x"], tk["labels_y"])
        zx = torch.zeros(x.shape[0], dtype=torch.float32, device=x.device)
        zy = torch.zeros(y.shape[0], dtype=torch.float32, device=y.device)
        init = (zx, zy, zx.clone(), zy.clone())
    kw.pop("potentials", None)
    # the solver's clustered layout reuses the token clustering (same K-means on the
    # same packed points) instead of running the K-means again
    return sinkhorn_divergence(x, a, y, b, blur=blur, scaling=scaling, init=init,
                               start_scale=blur / scaling ** s, checked_init=True,
                               potentials=True, n_clusters=n_clusters, kmeans_iters=kmeans_iters,
                               labels=labels, **kw)
