"""GPU parity of the softmin kernel against the FP64 oracle, element by element.

One softmin pass on arbitrary inputs needs no iteration, so it pins the kernel
exactly: the library's FP32 result must lie within the FP32 error bound of
``gpu_common.softmin_fp32_bound`` around the oracle's FP64 value.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import cuda, host, note, softmin_fp32_bound

pytestmark = pytest.mark.gpu


def _case(n, m, d, seed, scale=1.0, zero_frac=0.1):
    rng = np.random.default_rng(seed)
    x = (scale * rng.standard_normal((n, d))).astype(np.float32)
    y = (scale * rng.standard_normal((m, d)) + 0.3 * scale).astype(np.float32)
    w = synth.random_weights(m, seed + 1, zero_frac=zero_frac if m > 2 else 0.0)
    h = (0.5 * scale ** 2 * rng.standard_normal(m)).astype(np.float32)
    return x, y, w, h


def _check(x, y, w, h, eps, lam, tag):
    import paper_2107_02010_amd as skh
    note(f"softmin {tag} n={x.shape[0]} m={y.shape[0]} d={x.shape[1]} eps={eps} lam={lam}")
    out = host(skh.softmin(cuda(x), cuda(y), cuda(w), cuda(h), eps, lam))
    ref = oracle.softmin(x, y, w, h, eps, lam)
    bound = softmin_fp32_bound(x, y, w.astype(np.float64), h.astype(np.float64), eps, lam, ref)
    err = np.abs(out - ref)
    assert np.all(np.isfinite(out))
    worst = int(np.argmax(err / bound))
    assert np.all(err <= bound), (tag, worst, out[worst], ref[worst], bound[worst])
    return float(np.max(err / bound))


@pytest.mark.parametrize("n,m,d", [
    (1, 1, 3), (5, 7, 1), (300, 517, 3), (129, 129, 2), (1000, 1300, 60), (257, 4000, 16),
    (33, 2500, 60), (640, 64, 7), (2000, 2000, 3), (70, 300, 31), (100, 200, 63),
])
@pytest.mark.parametrize("eps_rel", [1e-2, 1.0])
def test_softmin_matches_oracle(n, m, d, eps_rel):
    x, y, w, h = _case(n, m, d, seed=n * 7 + m + d)
    eps = eps_rel * d
    _check(x, y, w, h, eps, 1.0, "random")
    _check(x, y, w, h, eps, 0.8, "damped")


def test_softmin_small_eps_and_far_points():
    # tiny eps: the max term dominates; far clusters exercise the online maximum
    x, y, w, h = _case(500, 700, 3, seed=3, scale=10.0)
    _check(x, y, w, h, 1e-3, 1.0, "small-eps")


def test_softmin_row_without_mass_is_inf():
    import paper_2107_02010_amd as skh
    x, y, w, h = _case(10, 20, 3, seed=4)
    w = np.zeros_like(w)
    note("softmin zero weights")
    out = host(skh.softmin(cuda(x), cuda(y), cuda(w), cuda(h), 0.5, 1.0))
    assert np.all(np.isinf(out)) and np.all(out > 0)


def test_softmin_blob_config_full_size():
    # 3-D blobs, n = m = 2000, eps = blur^2 = 1e-4 and at the first scale
    x, a, y, b = synth.blob_pair(2000, seed=0)
    rng = np.random.default_rng(5)
    h = (0.01 * rng.standard_normal(2000)).astype(np.float32)
    for eps in (1e-4, 1.0):
        _check(x, y, b, h, eps, 1.0, "blobs")


def test_softmin_fiber_full_size_sampled_rows():
    # 200k x 200k, 60-D fibres (the bench workload's shape); the oracle evaluates a
    # sample of rows, each against all 200k columns.
    import paper_2107_02010_amd as skh
    x, a, y, b = synth.fiber_pair(200_000, 50, seed=11)
    rng = np.random.default_rng(6)
    h = (2.0 * rng.standard_normal(200_000)).astype(np.float32)
    rows = np.sort(rng.choice(200_000, size=96, replace=False))
    rows[-1] = 199_999
    for eps in (1.0, 400.0):
        note(f"softmin fibres 200k eps={eps}")
        out = host(skh.softmin(cuda(x), cuda(y), cuda(b), cuda(h), eps, 1.0))
        ref = oracle.softmin(x[rows], y, b, h, eps, 1.0)
        # the bound needs the centre of the full clouds
        bound_all = softmin_fp32_bound(np.concatenate([x[rows], x]), y, b.astype(np.float64),
                                       h.astype(np.float64), eps, 1.0,
                                       np.concatenate([ref, np.zeros(len(x))]))[:len(rows)]
        err = np.abs(out[rows] - ref)
        assert np.all(err <= bound_all), (eps, np.max(err / bound_all))


# ------------------------------------------------------------- BF16 split ---
#
# The split contraction of one pair errs by at most 3 * 2^-16 |k x_i| |y_j - c_J| in
# log2 units (bf16 unit 2^-8: the dropped lo.lo product and the residuals of the two
# splits), i.e. 3 * 2^-16 lam |x_i| |y_j - c_J| in cost units, and log-sum-exp is
# 1-Lipschitz in the max norm, so a row errs by at most that for its worst column plus
# the FP32 bound of the rest of the arithmetic.  c_J is the centre of column j's
# K-means cluster.  For points inside the bounding box of the columns the library
# centres both clouds on the midpoint of that box, exactly as skh.kmeans centres the
# columns alone, so the clustering skh.kmeans returns (ceil(sqrt(m)) clusters, 10 Lloyd
# steps, the same packed width at d = 60) is the one the split path uses.

def _inside(x, y):
    """x clipped into the bounding box of y (see above)."""
    return np.clip(x, y.min(0), y.max(0)).astype(np.float32)


def _offset_radius(y, w):
    """max |y_j - c_J| over the columns with positive weight, from the clustering of
    the split path (FP64, from the centres skh.kmeans returns)."""
    import math

    import paper_2107_02010_amd as skh
    km = skh.kmeans(cuda(y), cuda(w), k=math.ceil(math.sqrt(len(y))), iters=10)
    c = host(km["centres"])
    lab = km["labels"].cpu().numpy()
    off = np.linalg.norm(y.astype(np.float64) - c[lab], axis=1)
    return float(off[w > 0].max())


def _split_bound(xc_rows, radius, lam):
    # 1.25: the FP32 rounding of the split terms themselves
    return 1.25 * 3 * 2.0 ** -16 * lam * np.linalg.norm(xc_rows, axis=1) * radius


def test_softmin_bf16_fiber_full_size_sampled_rows():
    # the benchmark's 200k x 200k fibre shape on the BF16 split path (its chosen
    # precision): sampled rows against all 200k columns in FP64, within the FP32 bound
    # plus the split bound on the actual cluster offsets
    import paper_2107_02010_amd as skh
    from gpu_common import centred
    x, a, y, b = synth.fiber_pair(200_000, 50, seed=12)
    x = _inside(x, y)
    rng = np.random.default_rng(8)
    h = (2.0 * rng.standard_normal(200_000)).astype(np.float32)
    rows = np.sort(rng.choice(200_000, size=64, replace=False))
    rows[-1] = 199_999
    xc, yc = centred(x, y)
    note("softmin bf16 fibres 200k: column clustering")
    radius = _offset_radius(y, b)
    for eps in (1.0, 400.0):
        note(f"softmin bf16 fibres 200k eps={eps}")
        out = host(skh.softmin(cuda(x), cuda(y), cuda(b), cuda(h), eps, 1.0,
                               precision="bf16x3"))
        ref = oracle.softmin(x[rows], y, b, h, eps, 1.0)
        split = _split_bound(xc[rows], radius, 1.0)
        # the split term is a small part of the scale of the problem
        assert split.max() <= 0.05 * eps, (eps, radius, split.max())
        bound = softmin_fp32_bound(np.concatenate([x[rows], x]), y, b.astype(np.float64),
                                   h.astype(np.float64), eps, 1.0,
                                   np.concatenate([ref, np.zeros(len(x))]))[:len(rows)] + split
        err = np.abs(out[rows] - ref)
        print(f"bf16 200k eps={eps}: radius {radius:.3f}, max err {err.max():.3e}, "
              f"max bound {bound.max():.3e} (split {split.max():.3e}), |out| >= "
              f"{np.abs(ref).min():.3f}")
        assert np.all(np.isfinite(out))
        assert np.all(err <= bound), (eps, np.max(err / bound))
        # a 1 % error of any sampled row is far outside what the kernel shows
        assert np.all(err <= 1e-3 * np.abs(ref) + 1e-3 * eps), (eps, np.max(err / np.abs(ref)))


def test_softmin_bf16_fiber_1m_sampled_rows():
    # 1M x 1M fibres (the time-to-S workload: 200 bundles, 1000 column clusters), one
    # dense BF16 split launch, sampled rows against all 1M columns in FP64
    import paper_2107_02010_amd as skh
    from gpu_common import centred
    x, a, y, b = synth.fiber_pair(1_000_000, 200, seed=0)
    x = _inside(x, y)
    rng = np.random.default_rng(10)
    h = (2.0 * rng.standard_normal(len(y))).astype(np.float32)
    rows = np.sort(rng.choice(len(x), size=24, replace=False))
    rows[-1] = len(x) - 1
    xc, yc = centred(x, y)
    note("softmin bf16 fibres 1M: column clustering")
    radius = _offset_radius(y, b)
    eps = 1.0
    note(f"softmin bf16 fibres 1M eps={eps}")
    out = host(skh.softmin(cuda(x), cuda(y), cuda(b), cuda(h), eps, 1.0, precision="bf16x3"))
    ref = oracle.softmin(x[rows], y, b, h, eps, 1.0)
    split = _split_bound(xc[rows], radius, 1.0)
    assert split.max() <= 0.05 * eps, (radius, split.max())
    bound = softmin_fp32_bound(np.concatenate([x[rows], x]), y, b.astype(np.float64),
                               h.astype(np.float64), eps, 1.0,
                               np.concatenate([ref, np.zeros(len(x))]))[:len(rows)] + split
    err = np.abs(out[rows] - ref)
    print(f"bf16 1M: radius {radius:.3f}, max err {err.max():.3e}, max bound {bound.max():.3e}")
    assert np.all(np.isfinite(out))
    assert np.all(err <= bound), np.max(err / bound)
    assert np.all(err <= 1e-3 * np.abs(ref) + 1e-3 * eps), np.max(err / np.abs(ref))


def _check_bf16(x, y, w, h, eps, lam, tag, radius=None):
    """BF16 hi/lo split against the oracle: the FP32 bound plus the split bound, on the
    actual cluster offsets when `radius` is given (see _offset_radius), otherwise with
    |y_j - c_J| <= 2 max |y| for any cluster centre c_J inside the cloud's hull."""
    import paper_2107_02010_amd as skh
    from gpu_common import centred
    note(f"softmin bf16 {tag} n={x.shape[0]} m={y.shape[0]} d={x.shape[1]} eps={eps}")
    out = host(skh.softmin(cuda(x), cuda(y), cuda(w), cuda(h), eps, lam, precision="bf16x3"))
    ref = oracle.softmin(x, y, w, h, eps, lam)
    xc, yc = centred(x, y)
    if radius is None:
        radius = 2 * np.linalg.norm(yc, axis=1).max()
    split = _split_bound(xc, radius, lam)
    bound = softmin_fp32_bound(x, y, w.astype(np.float64), h.astype(np.float64), eps, lam, ref) + split
    err = np.abs(out - ref)
    assert np.all(np.isfinite(out))
    worst = int(np.argmax(err / bound))
    assert np.all(err <= bound), (tag, worst, out[worst], ref[worst], bound[worst])
    return err


@pytest.mark.parametrize("n,m,d", [(300, 517, 3), (1000, 1300, 60), (257, 4000, 16), (33, 2500, 60),
                                   (5, 7, 1), (640, 64, 29)])
@pytest.mark.parametrize("eps_rel", [1e-2, 1.0])
def test_softmin_bf16_matches_oracle(n, m, d, eps_rel):
    x, y, w, h = _case(n, m, d, seed=n * 3 + m + d)
    _check_bf16(x, y, w, h, eps_rel * d, 1.0, "random")
    _check_bf16(x, y, w, h, eps_rel * d, 0.7, "damped")


def test_softmin_bf16_fibres_is_close_to_fp32_accuracy():
    # clustered fibres: the split error scales with the cluster radius
    x, a, y, b = synth.fiber_pair(6000, 20, seed=3)
    x = _inside(x, y)
    rng = np.random.default_rng(9)
    h = (rng.standard_normal(6000)).astype(np.float32)
    err = _check_bf16(x, y, b, h, 1.0, 1.0, "fibres", radius=_offset_radius(y, b))
    assert np.max(err) < 5e-3


def test_softmin_bf16_rejects_wide_points():
    import paper_2107_02010_amd as skh
    for d in (61, 62):
        x, y, w, h = _case(10, 10, d, seed=1)
        note(f"softmin bf16 d={d}")
        with pytest.raises(skh.SkhError):
            skh.softmin(cuda(x), cuda(y), cuda(w), cuda(h), 1.0, precision="bf16x3")


def test_softmin_bf16_no_mass_and_far_clusters():
    # zero weights (no mass: +inf), and far-apart clusters with a tiny eps, so the
    # running reference must be re-levelled many times inside a row's sweep
    import paper_2107_02010_amd as skh
    x, y, w, h = _case(40, 300, 8, seed=5)
    note("softmin bf16 zero weights")
    out = host(skh.softmin(cuda(x), cuda(y), cuda(np.zeros_like(w)), cuda(h), 0.5,
                           precision="bf16x3"))
    assert np.all(np.isinf(out)) and np.all(out > 0)
    rng = np.random.default_rng(7)
    centres = rng.uniform(-50, 50, size=(12, 8))
    y = (centres[rng.integers(0, 12, 3000)] + rng.standard_normal((3000, 8))).astype(np.float32)
    x = (centres[rng.integers(0, 12, 700)] + rng.standard_normal((700, 8))).astype(np.float32)
    w = synth.random_weights(3000, 8)
    h = (20.0 * rng.standard_normal(3000)).astype(np.float32)
    for eps in (0.05, 3.0):
        _check_bf16(x, y, w, h, eps, 1.0, "far-clusters")
