"""Wasserstein barycenter of track-density maps by gradient descent on the
support points (Section 3, "Track density atlas").

The loss is (1/K) sum_k S_{eps,rho}(alpha, beta_k) over the positions x_i of
alpha = sum_i a_i delta_{x_i}; each step solves the K divergences on the GPU,
takes the x-gradient of each from its dual vectors (hand-written kernel), and
moves every point by x_i <- x_i - lr * grad_i / a_i.  With p = 2, reach = inf
and blur = one voxel this is the paper's probabilistic atlas.
"""
from __future__ import annotations

import torch

from . import grad_x, sinkhorn_divergence


def barycenter_step(x, a, maps, blur: float = 1.0, reach=None, scaling: float = 0.9,
                    lr: float = 1.0, precision: str = "fp32", extra_iters: int = 0,
                    init=None):
    """One gradient step.  maps: list of (y_k, b_k) CUDA tensors.

    Returns (new x, mean S, list of per-map potentials dicts).
    """
    K = len(maps)
    grad = torch.zeros_like(x)
    total = 0.0
    pots = []
    for k, (y, b) in enumerate(maps):
        kw = dict(blur=blur, reach=reach, scaling=scaling, precision=precision,
                  extra_iters=extra_iters, potentials=True)
        S, pot, _ = sinkhorn_divergence(x, a, y, b, **kw)
        grad += grad_x(x, a, y, b, pot["f"], pot["g"], pot["p"], blur)
        total += S
        pots.append(pot)
    grad /= K
    x_new = x - lr * grad / a[:, None]
    return x_new, total / K, pots


def wasserstein_barycenter(x0, a, maps, steps: int = 10, **kw):
    """Runs `steps` gradient steps from x0; returns (x, list of mean S per step)."""
    x = x0.clone()
    history = []
    for _ in range(steps):
        x, S, _ = barycenter_step(x, a, maps, **kw)
        history.append(S)
    return x, history
