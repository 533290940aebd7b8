"""Seeded synthetic inputs shared by the oracle checks, the GPU tests and the benchmark.

This module only draws point clouds and weights (numpy PCG64 generators); it
holds none of the optimal-transport arithmetic.  Every generator is a pure
function of its arguments, returns FP32 arrays, and stands in for data the
paper uses but that is not available here (HCP tractograms, the fibre atlas and
the IFOF track-density maps).

* ``blobs``       isotropic Gaussian blobs in the unit cube (3-D clouds).
* ``fibers``      tractogram-like clouds: fibres along random cubic Bezier
                  spines with per-fibre control-point jitter, resampled to P
                  points at equal arc length and flattened to P*3 features
                  scaled by 1/sqrt(P) (the paper's fibre encoding, Section 2).
* ``density_maps``  track-density-like volumes: sums of Gaussian tubes along
                  jittered Bezier spines on a voxel grid, kept to the densest
                  voxels, returned as weighted voxel centres.
* ``fiber_labels``, ``random_orientations``, ``outlier_fibers``  atlas labels
                  (bundle ids), fibres stored in random directions, aberrant fibres
                  far from every bundle (label-transfer inputs).
* ``uniform_weights``  1/N weights.
"""
from __future__ import annotations

import numpy as np


def uniform_weights(n: int) -> np.ndarray:
    return np.full(n, 1.0 / n, dtype=np.float32) if n > 0 else np.zeros(0, np.float32)


def blobs(n: int, seed: int, n_blobs: int = 3, sigma: float = 0.1, d: int = 3,
          lo: float = 0.2, hi: float = 0.8) -> np.ndarray:
    """n points, split as evenly as possible over ``n_blobs`` isotropic Gaussians.

    Centres ~ U[lo, hi]^d and offsets ~ N(0, sigma^2) both come from ``seed``;
    the first ``n % n_blobs`` blobs take one extra point.  No clipping.
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(lo, hi, size=(n_blobs, d))
    sizes = [n // n_blobs + (1 if k < n % n_blobs else 0) for k in range(n_blobs)]
    parts = [centres[k] + sigma * rng.standard_normal((sizes[k], d)) for k in range(n_blobs)]
    out = np.concatenate(parts, axis=0) if n > 0 else np.zeros((0, d))
    return out.astype(np.float32)


def _bezier(ctrl: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Cubic Bezier curves. ctrl: (F, 4, 3); t: (T,) -> (F, T, 3)."""
    s = 1.0 - t
    basis = np.stack([s ** 3, 3 * s * s * t, 3 * s * t * t, t ** 3], axis=1)  # (T, 4)
    F = ctrl.shape[0]
    flat = np.ascontiguousarray(ctrl.transpose(0, 2, 1)).reshape(F * 3, 4) @ basis.T  # (3F, T)
    return flat.reshape(F, 3, -1).transpose(0, 2, 1)


def _resample_equal_arclength(poly: np.ndarray, P: int) -> np.ndarray:
    """Resample polylines (F, T, 3) to P points equally spaced in arc length (both ends kept).

    Target k of a fibre lies on the segment [idx, idx + 1] with idx the last
    sample whose cumulative length is <= the target (clipped to the last
    segment), and is interpolated linearly on that segment."""
    F, T, _ = poly.shape
    dif = np.diff(poly, axis=1)
    seg = np.sqrt(np.sum(dif * dif, axis=2))
    cum = np.concatenate([np.zeros((F, 1)), np.cumsum(seg, axis=1)], axis=1)  # (F, T)
    targets = cum[:, -1:] * np.linspace(0.0, 1.0, P)[None, :]  # (F, P)
    # one sorted search over all fibres (row offsets keep rows apart), then an
    # exact fix-up against the unshifted lengths
    span = 2.0 * cum[:, -1].max() + 1.0
    shift = np.arange(F, dtype=np.float64)[:, None] * span
    pos = np.searchsorted((cum + shift).ravel(), (targets + shift).ravel(), side="right")
    idx = np.clip(pos.reshape(F, P) - 1 - np.arange(F)[:, None] * T, 0, T - 2)
    rows = np.arange(F)[:, None]
    for _ in range(3):
        idx = idx + ((idx < T - 2) & (cum[rows, np.minimum(idx + 1, T - 1)] <= targets))
        idx = idx - ((idx > 0) & (cum[rows, idx] > targets))
    c0, c1 = cum[rows, idx], cum[rows, idx + 1]
    den = np.where(c1 > c0, c1 - c0, 1.0)
    w = np.where(c1 > c0, (targets - c0) / den, 0.0)
    p0, p1 = poly[rows, idx], poly[rows, idx + 1]
    return p0 + w[..., None] * (p1 - p0)


def fibers(n: int, n_bundles: int, spine_seed: int, seed: int, points: int = 20,
           box: float = 150.0, jitter: float = 2.0, samples: int = 256,
           chunk: int = 8192) -> np.ndarray:
    """Tractogram-like cloud of n fibres, returned as (n, 3*points) FP32.

    * ``n_bundles`` spines, each a cubic Bezier curve with 4 control points
      ~ U[0, box]^3 drawn from ``spine_seed`` (shared by the two clouds of a pair).
    * Fibre k of a bundle jitters every control point by N(0, jitter^2) per
      coordinate, drawn from ``seed``.
    * Bundle sizes are n // n_bundles, the first n % n_bundles bundles taking one
      more fibre; fibres are stored bundle after bundle.
    * Each fibre is sampled at ``samples`` uniform curve parameters, then
      resampled to ``points`` points at equal arc length, flattened point-major
      (p0x, p0y, p0z, p1x, ...) and scaled by 1/sqrt(points), so that the
      Euclidean distance of two feature vectors is the RMS point distance.
    """
    srng = np.random.default_rng(spine_seed)
    spines = srng.uniform(0.0, box, size=(n_bundles, 4, 3))
    rng = np.random.default_rng(seed)
    sizes = np.array([n // n_bundles + (1 if k < n % n_bundles else 0) for k in range(n_bundles)])
    bundle_of = np.repeat(np.arange(n_bundles), sizes)
    t = np.linspace(0.0, 1.0, samples)
    out = np.empty((n, 3 * points), dtype=np.float32)
    scale = 1.0 / np.sqrt(points)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        ctrl = spines[bundle_of[s:e]] + jitter * rng.standard_normal((e - s, 4, 3))
        poly = _bezier(ctrl, t)
        res = _resample_equal_arclength(poly, points)
        out[s:e] = (res.reshape(e - s, 3 * points) * scale).astype(np.float32)
    return out


def fiber_labels(n: int, n_bundles: int) -> np.ndarray:
    """Bundle index of each fibre of ``fibers(n, n_bundles, ...)`` (stored bundle after bundle)."""
    sizes = [n // n_bundles + (1 if k < n % n_bundles else 0) for k in range(n_bundles)]
    return np.repeat(np.arange(n_bundles, dtype=np.int32), sizes)


def random_orientations(x: np.ndarray, points: int, seed: int, frac: float = 0.5) -> np.ndarray:
    """Tractograms store each fibre in an arbitrary direction: a random fraction ``frac``
    of the fibres (drawn from ``seed``) is stored with its points in reverse order."""
    rng = np.random.default_rng(seed)
    n, d = x.shape
    rev = rng.uniform(size=n) < frac
    out = x.copy()
    out[rev] = x[rev].reshape(-1, points, d // points)[:, ::-1, :].reshape(-1, d)
    return out


def outlier_fibers(n: int, seed: int, points: int = 20, offset: float = 300.0) -> np.ndarray:
    """Aberrant fibres: each along its own random spine, with every point moved by
    ``offset`` mm along each axis, away from the bundles of ``fibers``."""
    x = fibers(n, n, spine_seed=seed, seed=seed + 1, points=points)
    return (x + np.float32(offset / np.sqrt(points))).astype(np.float32)


def fiber_pair(n: int, n_bundles: int, seed: int, points: int = 20):
    """Two clouds of the same anatomy: shared spines (seed), fibre jitter seeds seed+1 and seed+2."""
    x = fibers(n, n_bundles, spine_seed=seed, seed=seed + 1, points=points)
    y = fibers(n, n_bundles, spine_seed=seed, seed=seed + 2, points=points)
    return x, uniform_weights(n), y, uniform_weights(n)


def blob_pair(n: int, seed: int, d: int = 3):
    """Config-1 style pair: x from ``seed``, y from ``seed + 1`` (centres redrawn)."""
    x = blobs(n, seed, d=d)
    y = blobs(n, seed + 1, d=d)
    return x, uniform_weights(n), y, uniform_weights(n)


def random_weights(n: int, seed: int, total: float = 1.0, zero_frac: float = 0.0) -> np.ndarray:
    """Positive random weights summing to ``total``; a fraction may be set to exactly zero."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.2, 1.0, size=n)
    if zero_frac > 0 and n > 1:
        k = int(zero_frac * n)
        w[rng.choice(n, size=k, replace=False)] = 0.0
    if w.sum() <= 0:
        w[0] = 1.0
    return (w / w.sum() * total).astype(np.float32)


def random_cloud(n: int, d: int, seed: int, scale: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return (scale * rng.standard_normal((n, d))).astype(np.float32)


def density_maps(K: int, seed: int, grid: int = 128, n_tubes: int = 8, jitter: float = 3.0,
                 nonzero=(250_000, 350_000), sigma=(2.0, 4.0), samples_per_voxel: float = 16.0):
    """K track-density maps on a grid^3 voxel grid (voxel = 1 unit).

    Template spines (cubic Bezier, control points ~ U[0.05 grid, 0.95 grid]^3) are
    shared; map k jitters every control point by N(0, jitter^2) and gives each tube a
    cross-section sigma ~ U[sigma].  Density = histogram of points drawn uniformly
    along each spine parameter plus an isotropic N(0, sigma^2) offset (a Gaussian
    tube).  Map k keeps its N_k ~ U[nonzero] densest voxels (fewer if fewer are
    nonzero); weights = density / sum.  Returns a list of (centres (N_k, 3) FP32
    at voxel centres, weights (N_k,) FP32).
    """
    rng = np.random.default_rng(seed)
    lo, hi = 0.05 * grid, 0.95 * grid
    spines = rng.uniform(lo, hi, size=(n_tubes, 4, 3))
    maps = []
    for k in range(K):
        ctrl = spines + jitter * rng.standard_normal(spines.shape)
        sig = rng.uniform(sigma[0], sigma[1], size=n_tubes)
        target = int(rng.integers(nonzero[0], nonzero[1] + 1))
        n_samp = int(samples_per_voxel * target)
        tube = rng.integers(0, n_tubes, size=n_samp)
        t = rng.uniform(0.0, 1.0, size=n_samp)
        s = 1.0 - t
        basis = np.stack([s ** 3, 3 * s * s * t, 3 * s * t * t, t ** 3], axis=1)
        pts = np.einsum("nk,nkc->nc", basis, ctrl[tube])
        pts += sig[tube][:, None] * rng.standard_normal((n_samp, 3))
        idx = np.floor(pts).astype(np.int64)
        ok = np.all((idx >= 0) & (idx < grid), axis=1)
        flat = (idx[ok, 0] * grid + idx[ok, 1]) * grid + idx[ok, 2]
        counts = np.bincount(flat, minlength=grid ** 3)
        nz = np.flatnonzero(counts)
        keep = nz[np.argsort(-counts[nz], kind="stable")[:target]]
        keep.sort()
        cz = keep % grid
        cy = (keep // grid) % grid
        cx = keep // (grid * grid)
        centres = np.stack([cx, cy, cz], axis=1).astype(np.float64) + 0.5
        w = counts[keep].astype(np.float64)
        maps.append((centres.astype(np.float32), (w / w.sum()).astype(np.float32)))
    return maps


def barycenter_support(maps, n: int, seed: int):
    """n support points drawn from the average of the maps (each map equally likely,
    then a voxel by its weight), jittered uniformly inside the voxel; weights 1/n."""
    rng = np.random.default_rng(seed)
    which = rng.integers(0, len(maps), size=n)
    out = np.empty((n, 3))
    for k, (c, w) in enumerate(maps):
        sel = np.flatnonzero(which == k)
        if len(sel) == 0:
            continue
        p = w.astype(np.float64)
        vox = rng.choice(len(c), size=len(sel), p=p / p.sum())
        out[sel] = c[vox].astype(np.float64) + rng.uniform(-0.5, 0.5, size=(len(sel), 3))
    return out.astype(np.float32), uniform_weights(n)
