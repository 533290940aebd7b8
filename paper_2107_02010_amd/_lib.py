"""ctypes binding of libskh.so (include/skh.h): argument marshalling only.

Every step of the computation runs in the HIP library; this module converts
torch tensors to device pointers and the current torch stream to a hipStream_t.
It raises when the library is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libskh.so")

SKH_OK = 0
SKH_NOT_CONVERGED = 1
SKH_EINVAL = -1
SKH_EHIP = -2
SKH_ENOMEM = -3
SKH_ENONFINITE = -4
SKH_FP32 = 0
SKH_BF16_SPLIT = 1
SKH_MAX_DIM = 63
SKH_FIX_P = 1
SKH_FIX_Q = 2
SKH_FIX_CROSS = 4
SKH_INIT_COLD = 0
SKH_INIT_GIVEN = 1
SKH_INIT_WARM = 2
SKH_WS_IN = 64
SKH_WS_WIDTH = 256
SKH_WS_OUT = 2
SKH_WS_N_PARAMS = 345602
SKH_WS_MAX_PAIRS = 256

_c_i32, _c_i64, _c_d, _c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class SkhParams(ctypes.Structure):
    _fields_ = [
        ("blur", _c_d), ("reach", _c_d), ("scaling", _c_d), ("diameter", _c_d), ("tol", _c_d),
        ("jump_scale", _c_d), ("trunc_theta", _c_d), ("start_scale", _c_d), ("cost_p", _c_d),
        ("labels_x", _c_vp), ("labels_y", _c_vp),
        ("extra_iters", _c_i32), ("max_iters", _c_i32), ("check_every", _c_i32),
        ("precision", _c_i32), ("init", _c_i32), ("timing", _c_i32), ("multiscale", _c_i32),
        ("n_clusters", _c_i32), ("kmeans_iters", _c_i32), ("fixed", _c_i32),
        ("reserved", _c_i32 * 4),
    ]


class SkhStats(ctypes.Structure):
    _fields_ = [
        ("iters", _c_i32), ("n_scales", _c_i32), ("converged", _c_i32), ("checks", _c_i32),
        ("softmin_launches", _c_i32), ("coarse_iters", _c_i32), ("warm_fallback", _c_i32),
        ("reserved_i", _c_i32 * 1),
        ("diameter", _c_d), ("eps", _c_d), ("marginal_err", _c_d), ("pairs", _c_d),
        ("ms_total", _c_d), ("ms_softmin", _c_d), ("dense_pairs", _c_d), ("reserved", _c_d * 1),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if not k.startswith("reserved")}


class SkhError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"skh error {code}: {msg}")
        self.code = code


# name -> (restype, argtypes); every entry point declared in include/skh.h
SIGNATURES = {
    "skh_params_default": (None, [ctypes.POINTER(SkhParams)]),
    "skh_create": (_c_i32, [ctypes.POINTER(_c_vp), _c_i32, _c_vp]),
    "skh_destroy": (None, [_c_vp]),
    "skh_set_stream": (_c_i32, [_c_vp, _c_vp]),
    "skh_last_error": (ctypes.c_char_p, [_c_vp]),
    "skh_set_workspace_limit": (_c_i32, [_c_vp, ctypes.c_size_t]),
    "skh_workspace_bytes": (_c_i32, [_c_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "skh_softmin": (_c_i32, [_c_vp, _c_vp, _c_i64, _c_vp, _c_i64, _c_i32, _c_vp, _c_vp, _c_d, _c_d,
                             _c_i32, _c_vp]),
    "skh_softmin_noalloc": (_c_i32, [_c_vp, _c_vp, _c_i64, _c_vp, _c_i64, _c_i32, _c_vp, _c_vp,
                                     _c_d, _c_d, _c_i32, _c_vp]),
    "skh_sinkhorn_divergence": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_i64, _c_vp, _c_vp, _c_i64, _c_i32,
                                         ctypes.POINTER(SkhParams), ctypes.POINTER(_c_d), _c_vp,
                                         _c_vp, _c_vp, _c_vp, ctypes.POINTER(SkhStats)]),
    "skh_sinkhorn_divergence_batched": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp, _c_vp,
                                                 _c_i32, _c_i32, ctypes.POINTER(SkhParams),
                                                 _c_vp, _c_vp, _c_vp, _c_vp, _c_vp,
                                                 ctypes.POINTER(SkhStats)]),
    "skh_plan_apply": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_i64, _c_vp, _c_vp, _c_i64, _c_i32, _c_vp,
                                _c_vp, _c_d, _c_vp, _c_i32, _c_i32, _c_vp, _c_vp]),
    "skh_grad_x": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_i64, _c_vp, _c_vp, _c_i64, _c_i32, _c_vp, _c_vp,
                            _c_vp, _c_d, _c_vp]),
    "skh_gradients": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_i64, _c_vp, _c_vp, _c_i64, _c_i32, _c_vp,
                               _c_vp, _c_vp, _c_vp, _c_d, _c_d, _c_vp, _c_vp, _c_vp, _c_vp]),
    "skh_gradients_p": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_i64, _c_vp, _c_vp, _c_i64, _c_i32, _c_vp,
                                 _c_vp, _c_vp, _c_vp, _c_d, _c_d, _c_d, _c_vp, _c_vp, _c_vp,
                                 _c_vp]),
    "skh_label_transfer": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_i64, _c_vp, _c_vp, _c_i64, _c_i32,
                                    _c_vp, _c_i32, _c_i32, ctypes.POINTER(SkhParams), _c_vp,
                                    _c_vp, ctypes.POINTER(SkhStats)]),
    "skh_kmeans": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_i64, _c_i32, _c_i32, _c_i32, _c_vp, _c_vp,
                            _c_vp, _c_vp, _c_vp]),
    "skh_diameter": (_c_i32, [_c_vp, _c_vp, _c_i64, _c_vp, _c_i64, _c_i32, ctypes.POINTER(_c_d)]),
    "skh_self_potential": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_i64, _c_i32, ctypes.POINTER(SkhParams),
                                    _c_vp, ctypes.POINTER(SkhStats)]),
    "skh_ws_tokens": (_c_i32, [_c_vp, _c_vp, _c_vp, _c_i64, _c_vp, _c_vp, _c_i64, _c_i32, _c_i32,
                               _c_i32, _c_i32, _c_vp, _c_vp, _c_vp, _c_vp,
                               ctypes.POINTER(_c_i32)]),
    "skh_ws_forward": (_c_i32, [_c_vp, _c_vp, _c_i32, ctypes.POINTER(_c_i32), _c_vp, _c_vp, _c_i32,
                                _c_vp]),
    "skh_ws_loss_grad": (_c_i32, [_c_vp, _c_vp, _c_i32, ctypes.POINTER(_c_i32), _c_vp, _c_vp,
                                  _c_vp, ctypes.POINTER(_c_d), _c_vp]),
    "skh_ws_adam": (_c_i32, [_c_vp, _c_i64, _c_vp, _c_vp, _c_vp, _c_vp, _c_i32, _c_d, _c_d, _c_d,
                             _c_d]),
    "skh_ws_targets": (_c_i32, [_c_vp, _c_vp, _c_i64, _c_i32, _c_vp, _c_vp, _c_vp, _c_d, _c_vp]),
    "skh_ws_expand": (_c_i32, [_c_vp, _c_vp, _c_i64, _c_i32, _c_vp, _c_d, _c_vp, _c_vp]),
}

_lib = None
_lock = threading.Lock()


def load() -> ctypes.CDLL:
    """Loads libskh.so from the package directory (built by ``paper_2107_02010_amd.build``)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(
                    f"{LIB_PATH} is missing: build it with `python -m paper_2107_02010_amd.build` "
                    "(or __graft_entry__.build()); there is no non-HIP fallback")
            lib = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def check(rc: int, ctx=None, allow_not_converged: bool = False) -> int:
    if rc == SKH_OK or (allow_not_converged and rc == SKH_NOT_CONVERGED):
        return rc
    msg = load().skh_last_error(ctx)
    raise SkhError(rc, msg.decode() if msg else "")


def default_params() -> SkhParams:
    p = SkhParams()
    load().skh_params_default(ctypes.byref(p))
    return p
