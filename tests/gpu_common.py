"""Helpers shared by the GPU parity tests (no arithmetic of the method here)."""
import math
import sys

import numpy as np

U32 = 2.0 ** -24  # FP32 unit roundoff


def note(msg: str) -> None:
    """Names the case before a GPU step, flushed, so a crash log says what ran."""
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def cuda(a):
    import torch
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float32).cuda()


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def centred(x, y):
    """Coordinates minus the midpoint of the joint bounding box (what the library packs)."""
    lo = np.minimum(x.min(0), y.min(0)).astype(np.float64)
    hi = np.maximum(x.max(0), y.max(0)).astype(np.float64)
    c = (0.5 * (lo + hi)).astype(np.float32).astype(np.float64)
    return x.astype(np.float64) - c, y.astype(np.float64) - c


def softmin_fp32_bound(x, y, w, h, eps, lam, out_ref):
    """Per-row error bound of an FP32 softmin evaluated as the library does.

    The kernel forms s_ij = <x_i, y_j> log2(e)/eps + u_j in FP32 from centred
    coordinates (D+1 products), u_j = log2(e)(log w_j + (h_j - |y_j|^2/2)/eps).
    log-sum-exp is 1-Lipschitz in the max norm, so the row error is bounded by
    the largest error of one s_ij plus the FP32 rounding of the running sum and
    of |x_i|^2/2 and of the output.  Random-walk (sqrt) growth is used for the
    sums, with a factor 8 of headroom.
    """
    xc, yc = centred(x, y)
    d = x.shape[1]
    nx = np.linalg.norm(xc, axis=1)
    ny = np.linalg.norm(yc, axis=1)
    hn_y = 0.5 * ny ** 2
    with np.errstate(divide="ignore"):
        lw = np.where(w > 0, np.log(np.maximum(w, 1e-300)), 0.0)
    ucost = np.abs(eps * lw + h - hn_y)  # eps*ln2*|u_j| in cost units
    A = nx * ny.max() + ucost.max()
    m = y.shape[0]
    return 8 * U32 * lam * (math.sqrt(d + 2) * A + 0.5 * nx ** 2 + eps * math.sqrt(m)) \
        + 2 * U32 * np.abs(out_ref)
