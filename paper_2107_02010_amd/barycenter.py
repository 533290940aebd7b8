"""Wasserstein barycenter of track-density maps by gradient descent on the
support points (Section 3, "Track density atlas").

The loss is (1/K) sum_k S_{eps,rho}(alpha, beta_k) over the positions x_i of
alpha = sum_i a_i delta_{x_i}; each step moves every point by
x_i <- x_i - lr * mean_k grad_x S(alpha, beta_k) / a_i.

The Algorithm's four updates form three independent loops (alpha<->alpha reads
only p, beta<->beta only q, the cross pair only f and g), so with one scale
list for all maps a step needs:
  * the self vector p of alpha once (it does not depend on the map),
  * the self vectors q_k of the maps once for the whole descent (the maps do
    not move),
  * per map only the cross loop (two softmins per iteration), with p and q_k
    fixed,
and gives the same S_k, f_k, g_k as K full solves with that scale list.  The
common largest scale is the largest joint bounding-box diagonal over the maps
at the start (any upper bound of the distances is a valid first scale).  In
FP32 the K cross loops run as one batched solve: every iteration is one launch
over all maps (row tiles of each map's copy of the support against that map's
columns only).  With multiscale=True each map's cross loop runs the coarse-to-fine
scheme of Section 2 instead (K-means coarse loop, jump, cluster-block truncation at
e^{-trunc_theta}), from a cold start with p and q_k fixed; the self vectors stay dense.

Warm start (start_scale > 0): the first step runs the whole scale list from the
common largest scale; every later step starts the self loop of alpha and the K
cross loops from the previous step's vectors (p, f_k, g_k) with a scale list that
begins at start_scale (start_scale, start_scale * scaling, ..., blur), while the
q_k stay those of the first step.  The support moves a little per step, so the
previous vectors are close to the new ones and the long descent of sigma from the
diameter is not repeated.
"""
from __future__ import annotations

import torch

from . import (SKH_FIX_P, SKH_FIX_Q, diameter, grad_x, self_potential, sinkhorn_divergence,
               sinkhorn_divergence_batched)


class Barycenter:
    """Gradient descent on the support of alpha against K fixed maps."""

    def __init__(self, a, maps, blur: float = 1.0, reach=None, scaling: float = 0.9,
                 lr: float = 1.0, precision: str = "fp32", extra_iters: int = 0, x0=None,
                 batched: bool = True, multiscale: bool = False, trunc_theta: float = 20.0,
                 n_clusters: int = 0, tol: float = 0.0, max_iters: int = 1000,
                 start_scale: float = 0.0):
        self.a = a
        self.maps = maps
        self.multiscale = multiscale
        self.batched = batched and precision == "fp32" and not multiscale
        # tol > 0: every loop iterates at blur until its marginal error is <= tol
        self.kw = dict(blur=blur, reach=reach, scaling=scaling, precision=precision,
                       extra_iters=extra_iters, tol=tol, max_iters=max_iters)
        self.ms_kw = dict(multiscale=True, trunc_theta=trunc_theta, n_clusters=n_clusters)
        self.lr = lr
        self.d = None if x0 is None else max(diameter(x0, y) for y, _ in maps)
        self.q = None
        # warm start: largest scale of every step after the first (0: each step cold)
        self.start_scale = float(start_scale)
        if self.start_scale > 0.0 and multiscale:
            raise ValueError("the warm-started descent runs the dense cross loops")
        self.prev = None  # (p, [f_k], [g_k]) of the last step

    def _setup(self, x):
        if self.d is None:
            self.d = max(diameter(x, y) for y, _ in self.maps)
        if self.q is None:
            self.q = [self_potential(y, b, diameter=self.d, **self.kw)[0] for y, b in self.maps]

    def step(self, x):
        """One descent step; returns (new x, mean S, per-map potential dicts)."""
        self._setup(x)
        warm = self.start_scale > 0.0 and self.prev is not None
        if warm:
            p, _ = self_potential(x, self.a, init=self.prev[0], start_scale=self.start_scale,
                                  **self.kw)
        else:
            p, _ = self_potential(x, self.a, diameter=self.d, **self.kw)
        top = self.start_scale if warm else self.d
        grad = torch.zeros_like(x)
        total = 0.0
        pots = []
        if self.batched:
            K, n = len(self.maps), x.shape[0]
            m = sum(y.shape[0] for y, _ in self.maps)
            if warm:
                f0, g0 = torch.cat(self.prev[1]), torch.cat(self.prev[2])
            else:
                f0 = torch.zeros(K * n, dtype=torch.float32, device=x.device)
                g0 = torch.zeros(m, dtype=torch.float32, device=x.device)
            init = (f0, g0, p.repeat(K), torch.cat(self.q))
            kw = {k: v for k, v in self.kw.items() if k != "precision"}
            S, pot, _ = sinkhorn_divergence_batched(
                [x] * K, [self.a] * K, [y for y, _ in self.maps], [b for _, b in self.maps],
                diameter=top, init=init, fixed=SKH_FIX_P | SKH_FIX_Q, potentials=True, **kw)
            for k, (y, b) in enumerate(self.maps):
                pk = dict(f=pot["f"][k], g=pot["g"][k], p=pot["p"][k], q=pot["q"][k])
                grad += grad_x(x, self.a, y, b, pk["f"], pk["g"], pk["p"], self.kw["blur"])
                pots.append(pk)
            grad /= K
            self.prev = (p, [u["f"] for u in pots], [u["g"] for u in pots])
            return x - self.lr * grad / self.a[:, None], sum(S) / K, pots
        for k, ((y, b), q) in enumerate(zip(self.maps, self.q)):
            if self.multiscale:  # cold cross loop (coarse phase first), p and q fixed
                S, pot, _ = sinkhorn_divergence(x, self.a, y, b, diameter=self.d,
                                                init=(None, None, p, q),
                                                fixed=SKH_FIX_P | SKH_FIX_Q, potentials=True,
                                                **self.kw, **self.ms_kw)
            else:
                if warm:
                    zf, zg = self.prev[1][k], self.prev[2][k]
                else:
                    zf = torch.zeros(x.shape[0], dtype=torch.float32, device=x.device)
                    zg = torch.zeros(y.shape[0], dtype=torch.float32, device=x.device)
                S, pot, _ = sinkhorn_divergence(x, self.a, y, b, diameter=top,
                                                init=(zf, zg, p, q),
                                                fixed=SKH_FIX_P | SKH_FIX_Q, potentials=True,
                                                **self.kw)
            grad += grad_x(x, self.a, y, b, pot["f"], pot["g"], pot["p"], self.kw["blur"])
            total += S
            pots.append(pot)
        grad /= len(self.maps)
        self.prev = (p, [u["f"] for u in pots], [u["g"] for u in pots])
        return x - self.lr * grad / self.a[:, None], total / len(self.maps), pots


def barycenter_step(x, a, maps, blur: float = 1.0, reach=None, scaling: float = 0.9,
                    lr: float = 1.0, precision: str = "fp32", extra_iters: int = 0,
                    diameter_=None, batched: bool = True, multiscale: bool = False,
                    trunc_theta: float = 20.0, n_clusters: int = 0, tol: float = 0.0,
                    max_iters: int = 1000):
    """One gradient step with the scale list from diameter_ (None: the largest joint
    bounding-box diagonal of x with each map).  maps: list of (y_k, b_k) CUDA tensors.

    Returns (new x, mean S, list of per-map potentials dicts)."""
    B = Barycenter(a, maps, blur, reach, scaling, lr, precision, extra_iters, batched=batched,
                   multiscale=multiscale, trunc_theta=trunc_theta, n_clusters=n_clusters,
                   tol=tol, max_iters=max_iters)
    B.d = diameter_
    return B.step(x)


def wasserstein_barycenter(x0, a, maps, steps: int = 10, **kw):
    """Runs `steps` gradient steps from x0; returns (x, list of mean S per step).
    start_scale > 0 warm-starts every step after the first (see Barycenter)."""
    B = Barycenter(a, maps, x0=x0, **kw)
    x = x0.clone()
    history = []
    for _ in range(steps):
        x, S, _ = B.step(x)
        history.append(S)
    return x, history
