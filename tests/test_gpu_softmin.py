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

def test_softmin_bf16_fiber_full_size_sampled_rows():
    # the benchmark's 200k x 200k fibre shape on the BF16 split path (its chosen
    # precision): sampled rows against all 200k columns in FP64, within the FP32 bound
    # plus the split bound of _check_bf16 (any cluster centre lies in the cloud's hull)
    import paper_2107_02010_amd as skh
    from gpu_common import centred
    x, a, y, b = synth.fiber_pair(200_000, 50, seed=12)
    rng = np.random.default_rng(8)
    h = (2.0 * rng.standard_normal(200_000)).astype(np.float32)
    rows = np.sort(rng.choice(200_000, size=64, replace=False))
    rows[-1] = 199_999
    xc, yc = centred(x, y)
    for eps in (1.0, 400.0):
        note(f"softmin bf16 fibres 200k eps={eps}")
        out = host(skh.softmin(cuda(x), cuda(y), cuda(b), cuda(h), eps, 1.0,
                               precision="bf16x3"))
        ref = oracle.softmin(x[rows], y, b, h, eps, 1.0)
        bound = softmin_fp32_bound(np.concatenate([x[rows], x]), y, b.astype(np.float64),
                                   h.astype(np.float64), eps, 1.0,
                                   np.concatenate([ref, np.zeros(len(x))]))[:len(rows)]
        bound += 8 * 3 * 2.0 ** -16 * np.linalg.norm(xc[rows], axis=1) * 2 * \
            np.linalg.norm(yc, axis=1).max()
        err = np.abs(out[rows] - ref)
        assert np.all(np.isfinite(out))
        assert np.all(err <= bound), (eps, np.max(err / bound))


def _check_bf16(x, y, w, h, eps, lam, tag):
    """BF16 hi/lo split: the contraction error of one pair is at most
    3 * 2^-16 |x_i| |y_j - c_J| (dropped lo.lo product and the two split residuals),
    with |y_j - c_J| <= 2 max |y| for any cluster centre c_J inside the cloud's hull."""
    import paper_2107_02010_amd as skh
    from gpu_common import centred
    note(f"softmin bf16 {tag} n={x.shape[0]} m={y.shape[0]} d={x.shape[1]} eps={eps}")
    out = host(skh.softmin(cuda(x), cuda(y), cuda(w), cuda(h), eps, lam, precision="bf16x3"))
    ref = oracle.softmin(x, y, w, h, eps, lam)
    xc, yc = centred(x, y)
    split = 8 * 3 * 2.0 ** -16 * lam * np.linalg.norm(xc, axis=1) * 2 * np.linalg.norm(yc, axis=1).max()
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
    # clustered fibres: the split error scales with the cluster radius, so the
    # result is far inside the generic bound
    x, a, y, b = synth.fiber_pair(6000, 20, seed=3)
    rng = np.random.default_rng(9)
    h = (rng.standard_normal(6000)).astype(np.float32)
    err = _check_bf16(x, y, b, h, 1.0, 1.0, "fibres")
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
