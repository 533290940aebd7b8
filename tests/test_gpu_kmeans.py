"""GPU checks of the K-means coarse scale (Section 2, coarse-to-fine strategy).

Cluster labels are not unique (ties, local optima), so parity is checked on what
is fixed: with zero updates the labels are the nearest of the known initial
centres (brute force, FP64; near-ties within the FP32 error are accepted either
way); the sort is a stable permutation consistent with the offsets; centres and
masses are the weighted means and sums of the members; and Lloyd's inertia does
not increase with the number of iterations.
"""
import numpy as np
import pytest

import synth
from gpu_common import cuda, note

pytestmark = pytest.mark.gpu


def _km(x, w, k, iters):
    import paper_2107_02010_amd as skh
    note(f"kmeans n={len(x)} d={x.shape[1]} k={k} iters={iters}")
    r = skh.kmeans(cuda(x), cuda(w) if w is not None else None, k=k, iters=iters)
    return {key: v.cpu().numpy() for key, v in r.items()}


def _check_structure(x, w, k, r):
    n = len(x)
    off, perm, lab = r["offsets"], r["perm"], r["labels"]
    assert off[0] == 0 and off[-1] == n and np.all(np.diff(off) >= 0)
    assert np.array_equal(np.sort(perm), np.arange(n))
    for c in range(k):
        members = perm[off[c]:off[c + 1]]
        assert np.all(np.diff(members) > 0)  # stable: point order within a cluster
        assert np.all(lab[members] == c)
        ww = np.ones(len(members)) if w is None else w[members].astype(np.float64)
        if ww.sum() > 0:
            mean = (ww[:, None] * x[members].astype(np.float64)).sum(0) / ww.sum()
            scale = np.abs(x).max() + 1.0
            np.testing.assert_allclose(r["centres"][c], mean, atol=2e-6 * scale)
            assert r["masses"][c] == pytest.approx(ww.sum(), rel=1e-6)


@pytest.mark.parametrize("n,d,k", [(5000, 3, 71), (3000, 60, 55), (257, 2, 16), (64, 5, 64)])
def test_kmeans_structure_and_means(n, d, k):
    x = synth.random_cloud(n, d, seed=n + d, scale=3.0) if d != 60 else \
        synth.fibers(n, 10, spine_seed=1, seed=2)
    w = synth.random_weights(n, seed=3)
    r = _km(x, w, k, 10)
    _check_structure(x, w, k, r)


def test_kmeans_zero_iterations_is_nearest_initial_centre():
    n, d, k = 4000, 60, 63
    x = synth.fibers(n, 12, spine_seed=4, seed=5)
    r = _km(x, None, k, 0)
    init = x[(np.arange(k) * n) // k].astype(np.float64)
    x64 = x.astype(np.float64)
    dist = 0.5 * ((x64[:, None, :] - init[None]) ** 2).sum(-1)
    best = dist.min(1)
    lab = r["labels"]
    chosen = dist[np.arange(n), lab]
    # the library compares |c|^2/2 - <x, c> in FP32 on centred data: accept near-ties
    slack = 64 * 2.0 ** -24 * (0.5 * (x64 ** 2).sum(1) + (init ** 2).sum(1).max())
    assert np.all(chosen <= best + slack)
    exact = lab == dist.argmin(1)
    assert exact.mean() > 0.99


def test_kmeans_inertia_non_increasing():
    n, d, k = 6000, 3, 40
    x = synth.blobs(n, seed=6, n_blobs=7, sigma=0.05)
    w = synth.random_weights(n, seed=7)
    prev = np.inf
    for iters in (0, 1, 2, 4, 8):
        r = _km(x, w, k, iters)
        c = r["centres"].astype(np.float64)[r["labels"]]
        inertia = float((w * ((x - c) ** 2).sum(1)).sum())
        assert inertia <= prev * (1 + 1e-5)
        prev = inertia


def test_kmeans_rejects_bad_k():
    import paper_2107_02010_amd as skh
    x = synth.random_cloud(10, 3, seed=8)
    note("kmeans bad k")
    with pytest.raises(skh.SkhError):
        skh.kmeans(cuda(x), k=11)
    with pytest.raises(skh.SkhError):
        skh.kmeans(cuda(x), k=0)
