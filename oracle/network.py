"""FP64 reference of the warm-start set encoder (TEST INFRASTRUCTURE ONLY).

The network is the learned warm start of the solver: a permutation-equivariant
set encoder over coarse-cluster tokens that predicts, for every cluster of the
two clouds, its (cross, self) dual values divided by blur^2.  It is not in the
paper; the paper's Algorithm is the cold start it accelerates and what decides
its fixed point.  This module writes the same computation as the HIP kernels
in plain numpy FP64 (library matrix products as steps), with a hand-derived
backward pass, so that the kernels can be checked against it and it can be
checked against finite differences.

Layout of the flat parameter vector (row-major weights, out x in):
    W1 (256 x 64), b1, W2 (256 x 256), b2, W3 (256 x 256), b3,
    W4 (256 x 768), b4, W5 (2 x 256), b5
Forward for tokens X (T x 64), masses w (T), alpha tokens first (na of them):
    h = relu(relu(relu(X W1^T + b1) W2^T + b2) W3^T + b3)          (T x 256)
    P_a = sum_{t < na} w_t h_t / sum w_t,  P_b likewise over t >= na
    z_t = [h_t, P_a, P_b]                                          (T x 768)
    y = relu(z W4^T + b4) W5^T + b5                                 (T x 2)
Loss: sum_t wn_t |y_t - target_t|^2 with wn = w / sum(w) over all tokens.
"""
from __future__ import annotations

import numpy as np

WIDTH = 256
IN = 64
OUT = 2
SHAPES = [("W1", (WIDTH, IN)), ("b1", (WIDTH,)), ("W2", (WIDTH, WIDTH)), ("b2", (WIDTH,)),
          ("W3", (WIDTH, WIDTH)), ("b3", (WIDTH,)), ("W4", (WIDTH, 3 * WIDTH)), ("b4", (WIDTH,)),
          ("W5", (OUT, WIDTH)), ("b5", (OUT,))]


def n_params() -> int:
    return int(sum(np.prod(s) for _, s in SHAPES))


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        k = int(np.prod(shape))
        out[name] = theta[o:o + k].reshape(shape)
        o += k
    return out


def pack(params) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], np.float64).ravel() for name, _ in SHAPES])


def init_params(seed: int) -> np.ndarray:
    """He-style initialisation: N(0, 2/fan_in) weights, zero biases."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SHAPES:
        if name.startswith("W"):
            p[name] = rng.standard_normal(shape) * np.sqrt(2.0 / shape[1])
        else:
            p[name] = np.zeros(shape)
    return pack(p)


def _relu(v):
    return np.maximum(v, 0.0)


def forward(theta, X, w, na, keep=False):
    P = unpack(theta)
    X = np.asarray(X, np.float64)
    w = np.asarray(w, np.float64)
    a1 = _relu(X @ P["W1"].T + P["b1"])
    a2 = _relu(a1 @ P["W2"].T + P["b2"])
    h = _relu(a2 @ P["W3"].T + P["b3"])
    wa, wb = w[:na], w[na:]
    Pa = (wa[:, None] * h[:na]).sum(0) / wa.sum() if na > 0 else np.zeros(WIDTH)
    Pb = (wb[:, None] * h[na:]).sum(0) / wb.sum() if len(wb) > 0 else np.zeros(WIDTH)
    T = X.shape[0]
    z = np.concatenate([h, np.broadcast_to(Pa, (T, WIDTH)), np.broadcast_to(Pb, (T, WIDTH))], 1)
    a4 = _relu(z @ P["W4"].T + P["b4"])
    y = a4 @ P["W5"].T + P["b5"]
    if keep:
        return y, dict(X=X, w=w, na=na, a1=a1, a2=a2, h=h, z=z, a4=a4, P=P)
    return y


def loss_and_grad(theta, X, w, na, target):
    """Weighted MSE and its gradient with respect to theta (hand-derived backward)."""
    y, c = forward(theta, X, w, na, keep=True)
    P = c["P"]
    w = c["w"]
    wn = w / w.sum()
    r = y - np.asarray(target, np.float64)
    loss = float((wn[:, None] * r * r).sum())
    dy = 2.0 * wn[:, None] * r                          # T x 2
    g = {}
    g["W5"] = dy.T @ c["a4"]
    g["b5"] = dy.sum(0)
    da4 = (dy @ P["W5"]) * (c["a4"] > 0)                # T x 256
    g["W4"] = da4.T @ c["z"]
    g["b4"] = da4.sum(0)
    dz = da4 @ P["W4"]                                  # T x 768
    dh = dz[:, :WIDTH].copy()
    dPa = dz[:, WIDTH:2 * WIDTH].sum(0)
    dPb = dz[:, 2 * WIDTH:].sum(0)
    na = c["na"]
    if na > 0:
        dh[:na] += (w[:na] / w[:na].sum())[:, None] * dPa
    if len(w) > na:
        dh[na:] += (w[na:] / w[na:].sum())[:, None] * dPb
    dh3 = dh * (c["h"] > 0)
    g["W3"] = dh3.T @ c["a2"]
    g["b3"] = dh3.sum(0)
    da2 = (dh3 @ P["W3"]) * (c["a2"] > 0)
    g["W2"] = da2.T @ c["a1"]
    g["b2"] = da2.sum(0)
    da1 = (da2 @ P["W2"]) * (c["a1"] > 0)
    g["W1"] = da1.T @ c["X"]
    g["b1"] = da1.sum(0)
    return loss, pack(g)


def adam_step(theta, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam (Kingma & Ba) with bias correction; returns new (theta, m, v)."""
    m = beta1 * m + (1 - beta1) * grad
    v = beta2 * v + (1 - beta2) * grad * grad
    mh = m / (1 - beta1 ** step)
    vh = v / (1 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
