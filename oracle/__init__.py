"""FP64 CPU oracle for the Sinkhorn divergence (Feydy et al., arXiv 2107.02010).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the product package.  It shares no
code with the HIP library.  The arithmetic lives in ``oracle.c`` (plain C,
double precision); this module compiles it with gcc on first use and marshals
numpy arrays to it.  FP32 inputs are widened to FP64 exactly.

Notation follows Section 2 and the Algorithm of the paper:
``f = b^{beta->alpha}``, ``g = a^{alpha->beta}``, ``p = a^{alpha<->alpha}``,
``q = b^{beta<->beta}``; ``eps = sigma**2``, ``rho = reach**2``; ``reach=None``
(or inf, or <= 0) is the balanced problem.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

_D = ctypes.c_double
_I64 = ctypes.c_int64
_I = ctypes.c_int
_P = ctypes.POINTER(ctypes.c_double)


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (gcc, -O2, OpenMP, IEEE semantics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            lib = ctypes.CDLL(_LIB)
            lib.oracle_num_threads.argtypes = []
            lib.oracle_num_threads.restype = _I
            lib.oracle_set_num_threads.argtypes = [_I]
            lib.oracle_set_num_threads.restype = None
            lib.oracle_softmin.argtypes = [_I64, _I64, _I, _P, _P, _P, _P, _D, _D, _P]
            lib.oracle_softmin.restype = None
            lib.oracle_diameter.argtypes = [_I64, _I64, _I, _P, _P]
            lib.oracle_diameter.restype = _D
            lib.oracle_schedule.argtypes = [_D, _D, _D, _P, _I]
            lib.oracle_schedule.restype = _I
            lib.oracle_sinkhorn.argtypes = [_I64, _I64, _I, _P, _P, _P, _P, _D, _D, _D, _D,
                                            _I, _D, _I, _I, _I, _P, _P, _P, _P, _P]
            lib.oracle_sinkhorn.restype = _I
            lib.oracle_divergence.argtypes = [_I64, _I64, _P, _P, _P, _P, _P, _P, _D, _D]
            lib.oracle_divergence.restype = _D
            lib.oracle_ot_dual.argtypes = [_I64, _I64, _I, _P, _P, _P, _P, _P, _P, _D, _D]
            lib.oracle_ot_dual.restype = _D
            lib.oracle_ot_primal.argtypes = [_I64, _I64, _I, _P, _P, _P, _P, _P, _P, _D, _D]
            lib.oracle_ot_primal.restype = _D
            lib.oracle_marginals.argtypes = [_I64, _I64, _I, _P, _P, _P, _P, _P, _P, _D, _P, _P]
            lib.oracle_marginals.restype = None
            lib.oracle_plan_apply.argtypes = [_I64, _I64, _I, _P, _P, _P, _P, _P, _P, _D, _P,
                                              _I, _I, _P]
            lib.oracle_plan_apply.restype = None
            lib.oracle_grad_x.argtypes = [_I64, _I64, _I, _P, _P, _P, _P, _P, _P, _P, _D, _P]
            lib.oracle_grad_x.restype = None
            lib.oracle_grad_weights.argtypes = [_I64, _P, _P, _D, _D, _P]
            lib.oracle_grad_weights.restype = None
            lib.oracle_softmin_p.argtypes = [_I64, _I64, _I, _P, _P, _P, _P, _D, _D, _D, _P]
            lib.oracle_softmin_p.restype = None
            lib.oracle_sinkhorn_p.argtypes = [_I64, _I64, _I, _P, _P, _P, _P, _D, _D, _D, _D,
                                              _I, _D, _I, _I, _I, _D, _P, _P, _P, _P, _P]
            lib.oracle_sinkhorn_p.restype = _I
            lib.oracle_divergence_p.argtypes = [_I64, _I64, _P, _P, _P, _P, _P, _P, _D, _D, _D]
            lib.oracle_divergence_p.restype = _D
            lib.oracle_ot_dual_p.argtypes = [_I64, _I64, _I, _P, _P, _P, _P, _P, _P, _D, _D, _D]
            lib.oracle_ot_dual_p.restype = _D
            lib.oracle_ot_primal_p.argtypes = [_I64, _I64, _I, _P, _P, _P, _P, _P, _P, _D, _D, _D]
            lib.oracle_ot_primal_p.restype = _D
            _lib = lib
    return _lib


def _f64(a, shape=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


def _ptr(a):
    return a.ctypes.data_as(_P)


def _pts(x):
    x = _f64(x)
    if x.ndim == 1:
        x = x.reshape(-1, 1)
    return x


def _reach(reach):
    if reach is None or not (reach > 0) or math.isinf(reach):
        return 0.0
    return float(reach)


def num_threads() -> int:
    """Threads the oracle's OpenMP loops run on."""
    return int(_load().oracle_num_threads())


def set_num_threads(k: int) -> None:
    """Threads for the oracle's OpenMP loops from now on (timing only)."""
    _load().oracle_set_num_threads(int(k))


def softmin(rows, cols, w, h, eps, lam=1.0, p=2.0):
    """out_i = -lam*eps*log sum_j w_j exp((h_j - C(rows_i, cols_j))/eps)  (Algorithm, tilde updates),
    C = |x - y|^p / p."""
    r, c = _pts(rows), _pts(cols)
    w, h = _f64(w), _f64(h)
    out = np.empty(r.shape[0])
    _load().oracle_softmin_p(r.shape[0], c.shape[0], r.shape[1], _ptr(r), _ptr(c), _ptr(w),
                             _ptr(h), float(eps), float(lam), float(p), _ptr(out))
    return out


def diameter(x, y):
    """Joint bounding-box diagonal, the reading of the Algorithm's diameter heuristic."""
    x, y = _pts(x), _pts(y)
    return _load().oracle_diameter(x.shape[0], y.shape[0], x.shape[1], _ptr(x), _ptr(y))


def schedule(diam, blur, scaling):
    """The list [d, d q, ..., blur] of the Algorithm's loop header."""
    lib = _load()
    n = lib.oracle_schedule(float(diam), float(blur), float(scaling), None, 0)
    out = np.empty(n)
    lib.oracle_schedule(float(diam), float(blur), float(scaling), _ptr(out), n)
    return out


def sinkhorn(x, a, y, b, blur, reach=None, scaling=0.9, diam=None, extra_iters=0, tol=0.0,
             max_iters=0, check_every=1, init=None, p=2.0):
    """Symmetric averaged Sinkhorn loop with eps-scaling (Algorithm); cost |x - y|^p / p,
    eps = sigma^p, rho = reach^p.

    Returns dict(f, g, p, q, iters, n_scales, marginal_err, diameter, eps, converged).
    """
    pexp = float(p)
    x, y = _pts(x), _pts(y)
    a, b = _f64(a), _f64(b)
    n, m, d = x.shape[0], y.shape[0], x.shape[1]
    if init is None:
        f, g, p, q = np.zeros(n), np.zeros(m), np.zeros(n), np.zeros(m)
        flag = 0
    else:
        f, g, p, q = (_f64(v).copy() for v in init)
        flag = 1
    info = np.zeros(6)
    _load().oracle_sinkhorn_p(n, m, d, _ptr(x), _ptr(a), _ptr(y), _ptr(b), float(blur),
                              _reach(reach), float(scaling), float(diam or 0.0), int(extra_iters),
                              float(tol), int(max_iters), int(check_every), flag, pexp, _ptr(f),
                              _ptr(g), _ptr(p), _ptr(q), _ptr(info))
    return dict(f=f, g=g, p=p, q=q, iters=int(info[0]), n_scales=int(info[1]),
                marginal_err=float(info[2]), diameter=float(info[3]), eps=float(info[4]),
                converged=bool(info[5]))


def divergence(a, b, f, g, p, q, blur, reach=None, pexp=2.0):
    """S_{eps,rho} in the dual form of eq. (6) at eps = blur**pexp."""
    a, b, f, g, p, q = (_f64(v) for v in (a, b, f, g, p, q))
    return _load().oracle_divergence_p(a.size, b.size, _ptr(a), _ptr(b), _ptr(f), _ptr(g),
                                       _ptr(p), _ptr(q), float(blur), _reach(reach), float(pexp))


def ot_dual(x, a, y, b, f, g, eps, reach=None, p=2.0):
    """Dual objective of eq. (3) at (f, g) (cost |x - y|^p / p, rho = reach^p)."""
    x, y = _pts(x), _pts(y)
    a, b, f, g = (_f64(v) for v in (a, b, f, g))
    return _load().oracle_ot_dual_p(x.shape[0], y.shape[0], x.shape[1], _ptr(x), _ptr(a),
                                    _ptr(y), _ptr(b), _ptr(f), _ptr(g), float(eps), _reach(reach),
                                    float(p))


def ot_primal(x, a, y, b, f, g, eps, reach=None, p=2.0):
    """Primal objective of eq. (2) at the plan of eq. (4) built from (f, g)."""
    x, y = _pts(x), _pts(y)
    a, b, f, g = (_f64(v) for v in (a, b, f, g))
    return _load().oracle_ot_primal_p(x.shape[0], y.shape[0], x.shape[1], _ptr(x), _ptr(a),
                                      _ptr(y), _ptr(b), _ptr(f), _ptr(g), float(eps),
                                      _reach(reach), float(p))


def divergence_eq5(x, a, y, b, f, g, p, q, blur, reach=None, pexp=2.0):
    """S by eq. (5), each OT term by its dual objective eq. (3) at the given potentials."""
    eps = float(blur) ** 2 if pexp == 2.0 else float(blur) ** float(pexp)
    ab = ot_dual(x, a, y, b, f, g, eps, reach, p=pexp)
    aa = ot_dual(x, a, x, a, p, p, eps, reach, p=pexp)
    bb = ot_dual(y, b, y, b, q, q, eps, reach, p=pexp)
    ma, mb = float(np.sum(_f64(a))), float(np.sum(_f64(b)))
    return ab - 0.5 * aa - 0.5 * bb + 0.5 * eps * (ma - mb) ** 2


def marginals(x, a, y, b, f, g, eps):
    """Row and column sums of the plan of eq. (4)."""
    x, y = _pts(x), _pts(y)
    a, b, f, g = (_f64(v) for v in (a, b, f, g))
    row, col = np.empty(x.shape[0]), np.empty(y.shape[0])
    _load().oracle_marginals(x.shape[0], y.shape[0], x.shape[1], _ptr(x), _ptr(a), _ptr(y),
                             _ptr(b), _ptr(f), _ptr(g), float(eps), _ptr(row), _ptr(col))
    return row, col


def plan_apply(x, a, y, b, f, g, eps, V, divide_by_a=False):
    """(pi V)_i of eq. (4); with divide_by_a the soft labels of eq. (7)."""
    x, y = _pts(x), _pts(y)
    a, b, f, g = (_f64(v) for v in (a, b, f, g))
    V = _f64(V)
    if V.ndim == 1:
        V = V.reshape(-1, 1)
    out = np.empty((x.shape[0], V.shape[1]))
    _load().oracle_plan_apply(x.shape[0], y.shape[0], x.shape[1], _ptr(x), _ptr(a), _ptr(y),
                              _ptr(b), _ptr(f), _ptr(g), float(eps), _ptr(V), V.shape[1],
                              int(bool(divide_by_a)), _ptr(out))
    return out


def grad_x(x, a, y, b, f, g, p, eps):
    """Gradient of S with respect to x from the dual vectors (envelope theorem on eq. (3))."""
    x, y = _pts(x), _pts(y)
    a, b, f, g, p = (_f64(v) for v in (a, b, f, g, p))
    out = np.empty_like(x)
    _load().oracle_grad_x(x.shape[0], y.shape[0], x.shape[1], _ptr(x), _ptr(a), _ptr(y), _ptr(b),
                          _ptr(f), _ptr(g), _ptr(p), float(eps), _ptr(out))
    return out


def grad_x_p(x, a, y, b, f, g, p, blur, cost_p=2.0):
    """Gradient of S with respect to x for the cost |x - y|^P / P (Section 2), from the
    dual vectors at eps = blur^P: the envelope theorem on eq. (3) for the two OT terms of
    eq. (5) that depend on x,

      grad_i = sum_j pi_ij |x_i - y_j|^{P-2} (x_i - y_j) - sum_k pi^aa_ik |x_i - x_k|^{P-2} (x_i - x_k),

    pi from eq. (4) with that cost (the self term carries the factor 2 of a plan whose
    two marginals both move with x, times the 1/2 of eq. (5)).  A pair at distance 0
    contributes 0 (its difference vanishes; for P = 1 this is the zero subgradient).
    Dense numpy in FP64."""
    P = float(cost_p)
    eps = float(blur) ** P
    x, y = _pts(x), _pts(y)
    a, b, f, g, p = (_f64(v) for v in (a, b, f, g, p))

    def term(X, A, Y, B, F, G):
        diff = X[:, None, :] - Y[None, :, :]
        D = np.sqrt((diff ** 2).sum(-1))
        C = D ** P / P
        pi = A[:, None] * B[None, :] * np.exp((F[:, None] + G[None, :] - C) / eps)
        with np.errstate(divide="ignore"):
            w = np.where(D > 0.0, D ** (P - 2.0), 0.0)
        return ((pi * w)[:, :, None] * diff).sum(1)

    return term(x, a, y, b, f, g) - term(x, a, x, a, p, p)


def grad_y(x, a, y, b, f, g, q, eps):
    """Gradient of S with respect to y: the x formula with the roles of the two
    measures exchanged (S is symmetric in (alpha, beta))."""
    return grad_x(y, b, x, a, g, f, q, eps)


def grad_weights(f, p, blur, reach=None, cost_p=2.0):
    """dS/d alpha_i from (f, p) (dS/d beta_j from (g, q)): (rho + eps)(e^{-p/rho} - e^{-f/rho}),
    f - p when balanced (envelope theorem on the dual of eq. (3), Section 2); for the cost
    |x - y|^P / P the same expression at eps = blur^P, rho = reach^P."""
    f, p = _f64(f), _f64(p)
    out = np.empty_like(f)
    P = float(cost_p)
    if P == 2.0:
        _load().oracle_grad_weights(f.size, _ptr(f), _ptr(p), float(blur), _reach(reach),
                                    _ptr(out))
        return out
    eps = float(blur) ** P
    if reach is None or not np.isfinite(reach):
        return f - p
    rho = float(reach) ** P
    return -(rho + eps) * np.exp(-p / rho) * np.expm1(-(f - p) / rho)


def flip_fibers(x, points):
    """Mirror flips of fibres stored point-major (p0, p1, ..., p_{P-1}), each point d/P
    coordinates: the same curve traversed backwards (Section 2: the tractograms are
    augmented with the flips of all fibres, the simplest encoding of unoriented curves)."""
    x = _pts(x)
    n, d = x.shape
    return x.reshape(n, points, d // points)[:, ::-1, :].reshape(n, d).copy()


def label_transfer(x, a, y, b, labels, n_labels, blur, reach=None, flip_points=0, scaling=0.9,
                   tol=0.0, max_iters=0, check_every=1, extra_iters=0):
    """Soft labels of eq. (7) for the subject alpha from an atlas beta with integer labels
    (Section 3, label transfer): the cross dual vectors (f, g) of OT(alpha, beta), then
    Lab_i = sum_j beta_j onehot(l_j) exp((f_i + g_j - C_ij)/eps).  With flip_points = P
    the subject is augmented with the flips of its fibres at the same weights and the two
    versions of fibre i add up (the plan keeps the better-oriented one).  Returns
    (Lab (n x L), score = sum_l Lab_il, the augmented loop's result dict)."""
    x, y = _pts(x), _pts(y)
    a, b = _f64(a), _f64(b)
    n = x.shape[0]
    if flip_points:
        xs = np.concatenate([x, flip_fibers(x, flip_points)])
        as_ = np.concatenate([a, a])
    else:
        xs, as_ = x, a
    r = sinkhorn(xs, as_, y, b, blur, reach, scaling=scaling, tol=tol, max_iters=max_iters,
                 check_every=check_every, extra_iters=extra_iters)
    V = np.eye(int(n_labels))[np.asarray(labels, dtype=np.int64)]
    lab = plan_apply(xs, as_, y, b, r["f"], r["g"], float(blur) ** 2, V, divide_by_a=True)
    if flip_points:
        lab = lab[:n] + lab[n:]
    return lab, lab.sum(1), r


def sinkhorn_divergence(x, a, y, b, blur, reach=None, scaling=0.9, diam=None, extra_iters=0,
                        tol=0.0, max_iters=0, check_every=1, p=2.0):
    """Run the loop and return (S by eq. (6), the loop's result dict); cost |x - y|^p / p."""
    r = sinkhorn(x, a, y, b, blur, reach, scaling, diam, extra_iters, tol, max_iters, check_every,
                 p=p)
    S = divergence(a, b, r["f"], r["g"], r["p"], r["q"], blur, reach, pexp=p)
    return S, r


def barycenter_steps(x, a, maps, steps, blur, reach=None, scaling=0.9, lr=1.0, extra_iters=0,
                     diam=None, start_scale=0.0):
    """Gradient descent on the support of alpha for (1/K) sum_k S(alpha, beta_k)
    (Section 3, track density atlas): x <- x - lr * mean_k grad_x S(alpha, beta_k) / a,
    each S and gradient from the loop's dual vectors (full solve per map; diam: the
    largest scale of every solve, None: each pair's own).  Returns (x, mean S per step).

    start_scale > 0: every step after the first starts from the previous step's dual
    vectors with the scale list [start_scale, start_scale * scaling, ..., blur]: the self
    vector p of alpha from the alpha<->alpha loop alone (a run of the loop on the pair
    (alpha, alpha) started from (p, p, p, p), whose p is that loop), the cross vectors
    f_k, g_k from a run on (alpha, beta_k) started from (f_k, g_k, p, q_k) (the cross loop
    reads neither p nor q_k), and q_k held at its value from the first step (beta_k does
    not move)."""
    x = _pts(x).copy()
    a = _f64(a)
    eps = float(blur) ** 2
    hist = []
    prev = None
    for _ in range(steps):
        grad = np.zeros_like(x)
        tot = 0.0
        warm = start_scale > 0.0 and prev is not None
        if warm:
            p_prev, fs, gs, qs = prev
            p = sinkhorn(x, a, x, a, blur, reach, scaling, diam=start_scale,
                         extra_iters=extra_iters, init=(p_prev, p_prev, p_prev, p_prev))["p"]
        cur_f, cur_g, cur_q = [], [], []
        for k, (y, b) in enumerate(maps):
            if warm:
                r = sinkhorn(x, a, y, b, blur, reach, scaling, diam=start_scale,
                             extra_iters=extra_iters, init=(fs[k], gs[k], p, qs[k]))
                r["p"], r["q"] = p, qs[k]
                S = divergence(a, b, r["f"], r["g"], p, qs[k], blur, reach)
            else:
                S, r = sinkhorn_divergence(x, a, y, b, blur, reach, scaling=scaling, diam=diam,
                                           extra_iters=extra_iters)
            grad += grad_x(x, a, y, b, r["f"], r["g"], r["p"], eps)
            tot += S
            cur_f.append(r["f"])
            cur_g.append(r["g"])
            cur_q.append(r["q"])
        prev = (r["p"], cur_f, cur_g, cur_q)
        x = x - lr * (grad / len(maps)) / a[:, None]
        hist.append(tot / len(maps))
    return x, hist
