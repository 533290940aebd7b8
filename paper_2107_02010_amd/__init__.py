"""MI355X-native symmetric, debiased, multiscale Sinkhorn divergence (Feydy et al., arXiv 2107.02010).

Python face of libskh (HIP kernels for gfx950 behind the C ABI of
``include/skh.h``).  PyTorch is used for device memory and streams only:
every arithmetic step runs in the library.

    import paper_2107_02010_amd as skh
    S = skh.sinkhorn_divergence(x, a, y, b, blur=1.0, reach=None, scaling=0.9)
"""
from __future__ import annotations

import ctypes
import itertools
import math
import threading

import torch

from . import _lib
from ._lib import SkhError, SKH_FP32, SKH_BF16_SPLIT, SKH_FIX_P, SKH_FIX_Q, SKH_FIX_CROSS  # noqa: F401

__all__ = ["softmin", "sinkhorn_divergence", "kmeans", "plan_apply", "grad_x", "gradients",
           "label_transfer", "sinkhorn_divergence_batched",
           "diameter",
           "self_potential", "set_workspace_limit", "workspace_bytes",
           "SinkhornDivergence", "sinkhorn_loss", "SkhError", "library_path"]

library_path = _lib.LIB_PATH
_PREC = {"fp32": _lib.SKH_FP32, "bf16x3": _lib.SKH_BF16_SPLIT, "bf16_split": _lib.SKH_BF16_SPLIT}


class _Ctx:
    """One library context per device; rebound to torch's current stream on each call."""

    _ctxs: dict = {}
    _lock = threading.Lock()

    @classmethod
    def get(cls, device: torch.device):
        idx = device.index if device.index is not None else torch.cuda.current_device()
        with cls._lock:
            h = cls._ctxs.get(idx)
            if h is None:
                lib = _lib.load()
                h = ctypes.c_void_p()
                _lib.check(lib.skh_create(ctypes.byref(h), idx, None))
                cls._ctxs[idx] = h
        stream = torch.cuda.current_stream(idx).cuda_stream
        _lib.check(_lib.load().skh_set_stream(h, ctypes.c_void_p(stream)), h)
        return h


def _as_points(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dim() == 1:
        t = t.unsqueeze(1)
    if t.dim() != 2:
        raise ValueError(f"{name} must be (n, d)")
    return t.to(torch.float32).contiguous()


def _as_vec(t: torch.Tensor, n: int, name: str, device) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    t = t.to(torch.float32).reshape(-1).contiguous()
    if t.numel() != n:
        raise ValueError(f"{name} must have {n} entries")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    return t


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def softmin(x, y, w, h, eps: float, lam: float = 1.0, precision: str = "fp32") -> torch.Tensor:
    """out_i = -lam*eps*log sum_j w_j exp((h_j - |x_i - y_j|^2/2)/eps), on the GPU.

    The reduction behind the four updates of the Algorithm; x (n, d), y (m, d), w, h (m,).
    """
    x, y = _as_points(x, "x"), _as_points(y, "y")
    if x.shape[1] != y.shape[1]:
        raise ValueError("x and y must have the same dimension")
    w = _as_vec(w, y.shape[0], "w", y.device)
    h = _as_vec(h, y.shape[0], "h", y.device)
    out = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
    ctx = _Ctx.get(x.device)
    rc = _lib.load().skh_softmin(ctx, _ptr(x), x.shape[0], _ptr(y), y.shape[0], x.shape[1], _ptr(w),
                                 _ptr(h), float(eps), float(lam), _PREC[precision], _ptr(out))
    _lib.check(rc, ctx)
    return out


def _solver_params(blur, reach, scaling, diameter, extra_iters, tol, max_iters, check_every,
                   precision, timing, multiscale, jump_scale, trunc_theta, n_clusters,
                   kmeans_iters):
    P = _lib.default_params()
    P.blur = float(blur)
    P.reach = math.inf if reach is None else float(reach)
    P.scaling = float(scaling)
    P.diameter = 0.0 if diameter is None else float(diameter)
    P.tol = float(tol)
    P.extra_iters = int(extra_iters)
    P.max_iters = int(max_iters)
    P.check_every = int(check_every)
    P.precision = _PREC[precision]
    P.timing = 1 if timing else 0
    P.multiscale = 1 if multiscale else 0
    P.jump_scale = float(jump_scale)
    P.trunc_theta = float(trunc_theta)
    P.n_clusters = int(n_clusters)
    P.kmeans_iters = int(kmeans_iters)
    return P


def sinkhorn_divergence(x, a, y, b, blur: float = 0.05, reach=None, scaling: float = 0.9,
                        diameter=None, extra_iters: int = 0, tol: float = 0.0,
                        max_iters: int = 1000, check_every: int = 5, precision: str = "fp32",
                        init=None, potentials: bool = False, timing: bool = False,
                        multiscale: bool = False, jump_scale: float = 0.0,
                        trunc_theta: float = 20.0, n_clusters: int = 0, kmeans_iters: int = 10,
                        start_scale: float = 0.0, checked_init: bool = False, fixed: int = 0,
                        labels=None, p: float = 2.0):
    """S_{eps,rho}(alpha, beta) of eq. (5), through eq. (6) after the averaged symmetric loop.

    x (n, d), a (n,), y (m, d), b (m,): CUDA tensors.  reach=None is balanced.
    tol > 0 selects converged mode (iterate at blur until the marginal error <= tol).
    init: optional (f, g, p, q) starting potentials; the schedule then starts at start_scale
    (<= 0: the diameter rule).  Entries left None start cold (the schedule and multiscale
    phases as without init); every vector of a fixed loop must then be given.  checked_init=True: non-finite starting values are discarded
    and the call runs cold (stats["warm_fallback"] = 1).  fixed: SKH_FIX_* bits of the loops
    whose vectors are inputs (taken from init) and stay as given.  labels: optional (labels_x,
    labels_y) int32 cluster labels that replace the K-means on the clustered paths.
    With potentials=True returns
    (S, dict(f=..., g=..., p=..., q=...), stats dict), else S (a Python float).
    timing=True records HIP events around every softmin launch (stats["ms_softmin"]).
    multiscale=True: K-means coarse phase while sigma > jump_scale (0: RMS cluster radius,
    < 0: none), then cluster-block truncation at weight e^{-trunc_theta} (<= 0: none).
    p: exponent of the cost |x - y|^p / p in [1, 2] (eps = blur^p, rho = reach^p); p != 2
    runs the dense FP32 path.
    """
    x, y = _as_points(x, "x"), _as_points(y, "y")
    if x.shape[1] != y.shape[1]:
        raise ValueError("x and y must have the same dimension")
    n, m, d = x.shape[0], y.shape[0], x.shape[1]
    a = _as_vec(a, n, "a", x.device)
    b = _as_vec(b, m, "b", x.device)
    P = _solver_params(blur, reach, scaling, diameter, extra_iters, tol, max_iters, check_every,
                       precision, timing, multiscale, jump_scale, trunc_theta, n_clusters,
                       kmeans_iters)
    P.fixed = int(fixed)
    P.cost_p = float(p)
    if labels is not None:
        lx, ly = labels
        for t, k, nm in ((lx, n, "labels_x"), (ly, m, "labels_y")):
            if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32
                    and t.is_contiguous() and t.numel() == k):
                raise ValueError(f"{nm} must be a contiguous int32 CUDA tensor of {k} values")
        P.labels_x = lx.data_ptr()
        P.labels_y = ly.data_ptr()
    if fixed and init is None:
        raise ValueError("fixed dual vectors are passed through init=(f, g, p, q)")
    dev = x.device
    if init is not None and any(v is None for v in init):
        # cold start for the vectors left out; the fixed ones are read as given
        need = (fixed & _lib.SKH_FIX_CROSS, fixed & _lib.SKH_FIX_CROSS, fixed & _lib.SKH_FIX_P,
                fixed & _lib.SKH_FIX_Q)
        vecs = []
        for v, k, nm, nd in zip(init, (n, m, n, m), ("f", "g", "p", "q"), need):
            if v is None and nd:
                raise ValueError(f"the fixed vector {nm} must be given")
            vecs.append(torch.empty(k, dtype=torch.float32, device=dev) if v is None
                        else _as_vec(v, k, nm, dev).clone())
        f, g, p, q = vecs
    elif init is not None:
        f, g, p, q = (_as_vec(v, k, nm, dev).clone() for v, k, nm in
                      zip(init, (n, m, n, m), ("f", "g", "p", "q")))
        P.init = _lib.SKH_INIT_WARM if checked_init else _lib.SKH_INIT_GIVEN
        P.start_scale = float(start_scale)
    else:
        f = torch.empty(n, dtype=torch.float32, device=dev)
        g = torch.empty(m, dtype=torch.float32, device=dev)
        p = torch.empty(n, dtype=torch.float32, device=dev)
        q = torch.empty(m, dtype=torch.float32, device=dev)
    S = ctypes.c_double()
    st = _lib.SkhStats()
    ctx = _Ctx.get(dev)
    rc = _lib.load().skh_sinkhorn_divergence(ctx, _ptr(x), _ptr(a), n, _ptr(y), _ptr(b), m, d,
                                             ctypes.byref(P), ctypes.byref(S), _ptr(f), _ptr(g),
                                             _ptr(p), _ptr(q), ctypes.byref(st))
    _lib.check(rc, ctx, allow_not_converged=True)
    if potentials:
        return S.value, dict(f=f, g=g, p=p, q=q), st.as_dict()
    return S.value


def label_transfer(x, a, y, b, labels, n_labels: int, blur: float = 1.0, reach=20.0,
                   flip_points: int = 0, scaling: float = 0.9, diameter=None,
                   extra_iters: int = 0, tol: float = 0.0, max_iters: int = 1000,
                   check_every: int = 5, precision: str = "fp32", multiscale: bool = False,
                   jump_scale: float = 0.0, trunc_theta: float = 20.0, n_clusters: int = 0,
                   kmeans_iters: int = 10, stats: bool = False):
    """Soft labels of eq. (7) for the subject (x, a) from an atlas (y, b) with int32 labels in
    [0, n_labels) (Section 3, label transfer).  flip_points = P augments the subject with the
    mirror flips of its P-point fibres (the two versions add up).  Returns (Lab (n, L),
    score (n)); score ~ 1 for a matched fibre, ~ 0 for an outlier (unbalanced).  The
    default runs the Algorithm's schedule (one iteration per scale, tol = 0); with flips
    the subject carries twice the atlas mass, and the unbalanced loop removes the excess
    only at the rate rho / (rho + eps) per iteration, so tight tolerances take thousands
    of iterations without changing the decided labels."""
    x, y = _as_points(x, "x"), _as_points(y, "y")
    if x.shape[1] != y.shape[1]:
        raise ValueError("x and y must have the same dimension")
    n, m, d = x.shape[0], y.shape[0], x.shape[1]
    a, b = _as_vec(a, n, "a", x.device), _as_vec(b, m, "b", x.device)
    if not (isinstance(labels, torch.Tensor) and labels.is_cuda and labels.dtype == torch.int32
            and labels.is_contiguous() and labels.numel() == m):
        raise ValueError(f"labels must be a contiguous int32 CUDA tensor of {m} values")
    P = _solver_params(blur, reach, scaling, diameter, extra_iters, tol, max_iters, check_every,
                       precision, False, multiscale, jump_scale, trunc_theta, n_clusters,
                       kmeans_iters)
    L = int(n_labels)
    lab = torch.empty((n, L), dtype=torch.float32, device=x.device)
    score = torch.empty(n, dtype=torch.float32, device=x.device)
    st = _lib.SkhStats()
    ctx = _Ctx.get(x.device)
    rc = _lib.load().skh_label_transfer(ctx, _ptr(x), _ptr(a), n, _ptr(y), _ptr(b), m, d,
                                        _ptr(labels), L, int(flip_points), ctypes.byref(P),
                                        _ptr(lab), _ptr(score), ctypes.byref(st))
    _lib.check(rc, ctx, allow_not_converged=True)
    return (lab, score, st.as_dict()) if stats else (lab, score)


def sinkhorn_divergence_batched(xs, as_, ys, bs, blur: float = 0.05, reach=None,
                                scaling: float = 0.9, diameter=None, extra_iters: int = 0,
                                tol: float = 0.0, max_iters: int = 1000, check_every: int = 5,
                                init=None, fixed: int = 0, potentials: bool = False,
                                timing: bool = False):
    """S_eps(alpha_k, beta_k) for K independent pairs in one solve (four softmin launches per
    iteration for all pairs; dense FP32, p = 2).  xs, as_, ys, bs: lists of K CUDA tensors.
    The scale list is shared (largest scale: diameter, else the bounding-box diagonal of all
    points).  init: optional (f, g, p, q) over the concatenated points; fixed as for
    sinkhorn_divergence.  Returns the list of K values, with potentials=True also the
    per-pair dual vectors (lists) and the stats."""
    K = len(xs)
    if not (K >= 1 and len(as_) == K and len(ys) == K and len(bs) == K):
        raise ValueError("xs, as_, ys, bs must be lists of the same length >= 1")
    xs = [_as_points(t, "x") for t in xs]
    ys = [_as_points(t, "y") for t in ys]
    d = xs[0].shape[1]
    if any(t.shape[1] != d for t in xs + ys):
        raise ValueError("every cloud must have the same dimension")
    dev = xs[0].device
    xn = [t.shape[0] for t in xs]
    yn = [t.shape[0] for t in ys]
    x = torch.cat(xs).contiguous()
    y = torch.cat(ys).contiguous()
    a = torch.cat([_as_vec(w, k, "a", dev) for w, k in zip(as_, xn)]).contiguous()
    b = torch.cat([_as_vec(w, k, "b", dev) for w, k in zip(bs, yn)]).contiguous()
    n, m = x.shape[0], y.shape[0]
    xo = (ctypes.c_int64 * (K + 1))(*([0] + list(itertools.accumulate(xn))))
    yo = (ctypes.c_int64 * (K + 1))(*([0] + list(itertools.accumulate(yn))))
    P = _solver_params(blur, reach, scaling, diameter, extra_iters, tol, max_iters, check_every,
                       "fp32", timing, False, 0.0, 20.0, 0, 10)
    P.fixed = int(fixed)
    if fixed and init is None:
        raise ValueError("fixed dual vectors are passed through init=(f, g, p, q)")
    if init is not None:
        f, g, p, q = (_as_vec(v, k, nm, dev).clone() for v, k, nm in
                      zip(init, (n, m, n, m), ("f", "g", "p", "q")))
        P.init = _lib.SKH_INIT_GIVEN
    else:
        f, g, p, q = (torch.empty(k, dtype=torch.float32, device=dev) for k in (n, m, n, m))
    S = (ctypes.c_double * K)()
    st = _lib.SkhStats()
    ctx = _Ctx.get(dev)
    rc = _lib.load().skh_sinkhorn_divergence_batched(ctx, _ptr(x), _ptr(a), xo, _ptr(y), _ptr(b),
                                                     yo, K, d, ctypes.byref(P), S, _ptr(f),
                                                     _ptr(g), _ptr(p), _ptr(q), ctypes.byref(st))
    _lib.check(rc, ctx, allow_not_converged=True)
    vals = list(S)
    if not potentials:
        return vals
    pot = dict(f=list(torch.split(f, xn)), g=list(torch.split(g, yn)),
               p=list(torch.split(p, xn)), q=list(torch.split(q, yn)))
    return vals, pot, st.as_dict()


def _device(device):
    if device is None:
        return torch.device("cuda", torch.cuda.current_device())
    device = torch.device(device)
    if device.type != "cuda":
        raise ValueError("device must be a CUDA (HIP) device")
    return device


def set_workspace_limit(nbytes: int, device=None) -> None:
    """Caps the device workspace of the library's context on `device` (0: no cap).  A call
    that would need more raises SkhError (SKH_ENOMEM); a cap below the current holding
    frees the workspace."""
    if int(nbytes) < 0:
        raise ValueError("nbytes must be >= 0")
    ctx = _Ctx.get(_device(device))
    _lib.check(_lib.load().skh_set_workspace_limit(ctx, int(nbytes)), ctx)


def workspace_bytes(device=None) -> int:
    """Device workspace bytes the library's context on `device` holds now."""
    ctx = _Ctx.get(_device(device))
    out = ctypes.c_size_t()
    _lib.check(_lib.load().skh_workspace_bytes(ctx, ctypes.byref(out)), ctx)
    return int(out.value)


def diameter(x, y) -> float:
    """Largest scale of the Algorithm's list for (x, y): the joint bounding-box diagonal."""
    x, y = _as_points(x, "x"), _as_points(y, "y")
    out = ctypes.c_double()
    ctx = _Ctx.get(x.device)
    rc = _lib.load().skh_diameter(ctx, _ptr(x), x.shape[0], _ptr(y), y.shape[0], x.shape[1],
                                  ctypes.byref(out))
    _lib.check(rc, ctx)
    return out.value


def self_potential(x, a, blur: float = 0.05, reach=None, scaling: float = 0.9, diameter=None,
                   extra_iters: int = 0, tol: float = 0.0, max_iters: int = 1000,
                   check_every: int = 5, precision: str = "fp32", init=None,
                   start_scale: float = 0.0):
    """The self dual vector p = a^{alpha<->alpha} of the Algorithm's alpha<->alpha loop alone.

    With the diameter of a full problem (alpha, beta) it equals that solve's p.
    Returns (p, stats dict)."""
    x = _as_points(x, "x")
    n, d = x.shape
    a = _as_vec(a, n, "a", x.device)
    P = _lib.default_params()
    P.blur = float(blur)
    P.reach = math.inf if reach is None else float(reach)
    P.scaling = float(scaling)
    P.diameter = 0.0 if diameter is None else float(diameter)
    P.tol = float(tol)
    P.extra_iters = int(extra_iters)
    P.max_iters = int(max_iters)
    P.check_every = int(check_every)
    P.precision = _PREC[precision]
    if init is not None:
        p = _as_vec(init, n, "init", x.device).clone()
        P.init = _lib.SKH_INIT_GIVEN
        P.start_scale = float(start_scale)
    else:
        p = torch.empty(n, dtype=torch.float32, device=x.device)
    st = _lib.SkhStats()
    ctx = _Ctx.get(x.device)
    rc = _lib.load().skh_self_potential(ctx, _ptr(x), _ptr(a), n, d, ctypes.byref(P), _ptr(p),
                                        ctypes.byref(st))
    _lib.check(rc, ctx, allow_not_converged=True)
    return p, st.as_dict()


def kmeans(x, w=None, k: int = None, iters: int = 10) -> dict:
    """K-means coarse scale of a cloud (Section 2, coarse-to-fine strategy), on the GPU.

    Returns dict(centres (k, d), masses (k,), labels (n,), perm (n,), offsets (k+1,)).
    k defaults to ceil(sqrt(n)).
    """
    x = _as_points(x, "x")
    n, d = x.shape
    if k is None:
        k = max(1, math.ceil(math.sqrt(n)))
    wt = _as_vec(w, n, "w", x.device) if w is not None else None
    dev = x.device
    out = dict(centres=torch.empty((k, d), dtype=torch.float32, device=dev),
               masses=torch.empty(k, dtype=torch.float32, device=dev),
               labels=torch.empty(n, dtype=torch.int32, device=dev),
               perm=torch.empty(n, dtype=torch.int32, device=dev),
               offsets=torch.empty(k + 1, dtype=torch.int32, device=dev))
    ctx = _Ctx.get(dev)
    rc = _lib.load().skh_kmeans(ctx, _ptr(x), _ptr(wt), n, d, int(k), int(iters),
                                _ptr(out["centres"]), _ptr(out["masses"]), _ptr(out["labels"]),
                                _ptr(out["perm"]), _ptr(out["offsets"]))
    _lib.check(rc, ctx)
    return out


def plan_apply(x, a, y, b, f, g, eps: float, V, divide_by_a: bool = False,
               return_mass: bool = False):
    """(pi V)_i = a_i sum_j b_j exp((f_i + g_j - C(x_i, y_j))/eps) V_j  (eq. (4)); with
    divide_by_a the a_i factor is dropped (eq. (7) soft labels for one-hot V)."""
    x, y = _as_points(x, "x"), _as_points(y, "y")
    n, m, d = x.shape[0], y.shape[0], x.shape[1]
    dev = x.device
    a, b = _as_vec(a, n, "a", dev), _as_vec(b, m, "b", dev)
    f, g = _as_vec(f, n, "f", dev), _as_vec(g, m, "g", dev)
    V = V.to(torch.float32)
    V = (V.unsqueeze(1) if V.dim() == 1 else V).contiguous()
    if V.shape[0] != m:
        raise ValueError("V must have one row per column point")
    L = V.shape[1]
    out = torch.empty((n, L), dtype=torch.float32, device=dev)
    mass = torch.empty(n, dtype=torch.float32, device=dev) if return_mass else None
    ctx = _Ctx.get(dev)
    rc = _lib.load().skh_plan_apply(ctx, _ptr(x), _ptr(a), n, _ptr(y), _ptr(b), m, d, _ptr(f),
                                    _ptr(g), float(eps), _ptr(V), L, int(bool(divide_by_a)),
                                    _ptr(out), _ptr(mass))
    _lib.check(rc, ctx)
    return (out, mass) if return_mass else out


def grad_x(x, a, y, b, f, g, p, blur: float) -> torch.Tensor:
    """Gradient of S with respect to x from the dual vectors (f, g, p) of a solve:
    sum_j pi_ij (x_i - y_j) - sum_k pi^aa_ik (x_i - x_k) at eps = blur**2."""
    x, y = _as_points(x, "x"), _as_points(y, "y")
    n, m, d = x.shape[0], y.shape[0], x.shape[1]
    dev = x.device
    a, b = _as_vec(a, n, "a", dev), _as_vec(b, m, "b", dev)
    f, g, p = _as_vec(f, n, "f", dev), _as_vec(g, m, "g", dev), _as_vec(p, n, "p", dev)
    out = torch.empty((n, d), dtype=torch.float32, device=dev)
    ctx = _Ctx.get(dev)
    rc = _lib.load().skh_grad_x(ctx, _ptr(x), _ptr(a), n, _ptr(y), _ptr(b), m, d, _ptr(f),
                                _ptr(g), _ptr(p), float(blur), _ptr(out))
    _lib.check(rc, ctx)
    return out


def gradients(x, a, y, b, pot, blur: float, reach=None, wrt=("a", "b", "x", "y"),
              p: float = 2.0) -> dict:
    """Gradients of S with respect to the weights and positions of both measures from
    the dual vectors pot = {f, g, p, q} of a solve (Section 2: expressions of the four
    dual vectors).  dS/da_i = (rho + eps)(e^{-p_i/rho} - e^{-f_i/rho}) (f_i - p_i when
    balanced: then dS/da and dS/db share a free additive constant), dS/db likewise from
    (g, q); dS/dx as grad_x, dS/dy with the roles exchanged.  wrt: which to compute.
    p: exponent of the cost |x - y|^p / p the potentials were solved with (eps = blur^p,
    rho = reach^p; dS/dx then weights each pair by |x_i - y_j|^{p-2})."""
    x, y = _as_points(x, "x"), _as_points(y, "y")
    n, m, d = x.shape[0], y.shape[0], x.shape[1]
    dev = x.device
    a, b = _as_vec(a, n, "a", dev), _as_vec(b, m, "b", dev)
    f, g = _as_vec(pot["f"], n, "f", dev), _as_vec(pot["g"], m, "g", dev)
    p_, q = _as_vec(pot["p"], n, "p", dev), _as_vec(pot["q"], m, "q", dev)
    shapes = {"a": (n,), "b": (m,), "x": (n, d), "y": (m, d)}
    out = {k: torch.empty(shapes[k], dtype=torch.float32, device=dev) for k in wrt}
    rr = 0.0 if reach is None else float(reach)
    ctx = _Ctx.get(dev)
    rc = _lib.load().skh_gradients_p(ctx, _ptr(x), _ptr(a), n, _ptr(y), _ptr(b), m, d, _ptr(f),
                                     _ptr(g), _ptr(p_), _ptr(q), float(blur), rr, float(p),
                                     *(_ptr(out[k]) if k in out else None for k in "abxy"))
    _lib.check(rc, ctx)
    return out


class SinkhornDivergence(torch.autograd.Function):
    """S_eps(alpha, beta) as a differentiable function of x, a, y and b.

    forward runs the solver (eq. (6) after the symmetric loop); backward calls the
    hand-written gradient kernels with the saved dual vectors, without
    differentiating through the iterations (envelope theorem at the fixed point).
    Balanced problems: the weight gradients carry the free constant of (f, g)."""

    @staticmethod
    def forward(ctx, x, a, y, b, kw):
        S, pot, st = sinkhorn_divergence(x, a, y, b, potentials=True, **kw)
        ctx.save_for_backward(x, a, y, b, pot["f"], pot["g"], pot["p"], pot["q"])
        ctx.blur = kw.get("blur", 0.05)
        ctx.reach = kw.get("reach", None)
        ctx.cost_p = float(kw.get("p", 2.0))  # the backward uses the solve's cost
        return torch.tensor(S, dtype=torch.float64, device=x.device)

    @staticmethod
    def backward(ctx, gS):
        x, a, y, b, f, g, p, q = ctx.saved_tensors
        want = [k for k, need in zip("xayb", ctx.needs_input_grad[:4]) if need]
        res = {}
        if want:
            res = gradients(x.detach(), a.detach(), y.detach(), b.detach(),
                            dict(f=f, g=g, p=p, q=q), ctx.blur, ctx.reach, wrt=tuple(want),
                            p=ctx.cost_p)
        src = {"x": x, "a": a, "y": y, "b": b}
        grads = [(res[k].to(torch.float64) * gS).to(src[k].dtype) if k in res else None
                 for k in "xayb"]
        return (*grads, None)


def sinkhorn_loss(x, a, y, b, **kw):
    """Differentiable S_eps (see SinkhornDivergence); kw as for sinkhorn_divergence."""
    kw.pop("potentials", None)
    return SinkhornDivergence.apply(x, a, y, b, kw)
