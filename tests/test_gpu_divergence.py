"""GPU parity of the full symmetric Sinkhorn loop and of eq. (6) against the FP64 oracle.

Both sides run the same schedule (same diameter reading, same scale list, same
number of iterations) on the same FP32 inputs.  The FP32 path must match the
oracle's S to 1e-5 relative; potentials are compared after fixing the
balanced gauge (f + c, g - c) and within an FP32-propagation tolerance.
"""
import math

import numpy as np
import pytest

import oracle
import synth
from gpu_common import cuda, host, note

pytestmark = pytest.mark.gpu

S_RTOL_FP32 = 1e-5
S_RTOL_BF16 = 1e-3


def _run(x, a, y, b, blur, reach, scaling, extra=0, **kw):
    import paper_2107_02010_amd as skh
    note(f"divergence n={len(x)} m={len(y)} d={x.shape[1]} blur={blur} reach={reach} "
         f"q={scaling} extra={extra} {kw}")
    S, pot, st = skh.sinkhorn_divergence(cuda(x), cuda(a), cuda(y), cuda(b), blur=blur,
                                         reach=reach, scaling=scaling, extra_iters=extra,
                                         potentials=True, **kw)
    return S, {k: host(v) for k, v in pot.items()}, st


def _compare(x, a, y, b, blur, reach, scaling, extra=0, pot_atol=None, precision="fp32"):
    S, pot, st = _run(x, a, y, b, blur, reach, scaling, extra, precision=precision)
    Sr, r = oracle.sinkhorn_divergence(x, a, y, b, blur, reach, scaling=scaling, extra_iters=extra)
    assert st["iters"] == r["iters"] and st["n_scales"] == r["n_scales"]
    assert st["diameter"] == pytest.approx(r["diameter"], rel=1e-12)
    rtol = S_RTOL_FP32 if precision == "fp32" else S_RTOL_BF16
    assert S == pytest.approx(Sr, rel=rtol), (S, Sr)
    # potentials: compare after removing the mean (gauge), scale-aware tolerance
    if pot_atol is None:
        pot_atol = (1e-4 if precision == "fp32" else 1e-2) * max(blur ** 2, np.abs(r["f"]).max())
    for k in ("f", "g", "p", "q"):
        dg = pot[k] - r[k]
        dg -= dg.mean() if reach is None else 0.0
        assert np.max(np.abs(dg)) <= pot_atol, (k, np.max(np.abs(dg)), pot_atol)
    return S, Sr, st


def test_blob_config_full_size_balanced():
    # 3 isotropic blobs, n = m = 2000 in R^3, blur 0.01, scaling 0.5, no multiscale.
    x, a, y, b = synth.blob_pair(2000, seed=0)
    _compare(x, a, y, b, blur=0.01, reach=None, scaling=0.5)
    _compare(x, a, y, b, blur=0.01, reach=None, scaling=0.5, extra=20)


def test_blob_unbalanced_unequal_masses():
    x, a, y, b = synth.blob_pair(1500, seed=2)
    b = synth.random_weights(1500, 3, total=1.3, zero_frac=0.05)
    _compare(x, a, y, b, blur=0.02, reach=0.3, scaling=0.5, extra=5)


def test_fiber_downscaled_balanced_fp32():
    # the 60-D fibre generator at n = m = 3000 (20 bundles), blur 1 mm
    x, a, y, b = synth.fiber_pair(3000, 20, seed=7)
    _compare(x, a, y, b, blur=1.0, reach=None, scaling=0.8)


def test_fiber_downscaled_unbalanced_fp32():
    x, a, y, b = synth.fiber_pair(2500, 20, seed=9)
    _compare(x, a, y, b, blur=1.0, reach=20.0, scaling=0.8, extra=3)


def test_fiber_200k_full_size_bf16_against_fp32():
    # The benchmark's default step at full size (200k x 200k 60-D fibres, 50 bundles,
    # blur 1 mm, balanced, scaling 0.9, dense): the BF16 split solve it times against
    # the FP32 solve (pinned to the oracle at small sizes) on the same schedule.
    import paper_2107_02010_amd as skh
    x, a, y, b = synth.fiber_pair(200_000, 50, seed=0)
    X, A, Y, B = cuda(x), cuda(a), cuda(y), cuda(b)
    kw = dict(blur=1.0, reach=None, scaling=0.9, potentials=True)
    note("fibres 200k full size: FP32 solve")
    S0, pot0, st0 = skh.sinkhorn_divergence(X, A, Y, B, precision="fp32", **kw)
    note("fibres 200k full size: BF16 split solve")
    S1, pot1, st1 = skh.sinkhorn_divergence(X, A, Y, B, precision="bf16x3", **kw)
    assert st0["iters"] == st1["iters"] > 40
    print(f"S fp32 {S0:.9g} bf16 {S1:.9g} rel {abs(S1 - S0) / abs(S0):.2e}")
    assert abs(S1 - S0) <= 1e-3 * abs(S0)
    scale = max(1.0, float(pot0["f"].abs().max()))
    for k in ("f", "g", "p", "q"):
        dg = host(pot1[k]).astype(np.float64) - host(pot0[k]).astype(np.float64)
        dg -= dg.mean()  # balanced: potentials are defined up to a constant
        assert np.max(np.abs(dg)) <= 1e-3 * scale, (k, np.max(np.abs(dg)))


@pytest.mark.parametrize("n,m,d", [(1, 1, 3), (1, 37, 2), (130, 1, 5), (257, 129, 1), (5, 300, 60)])
def test_edge_sizes(n, m, d):
    rng = np.random.default_rng(n + m + d)
    x = rng.standard_normal((n, d)).astype(np.float32)
    y = (rng.standard_normal((m, d)) + 0.5).astype(np.float32)
    a = synth.random_weights(n, 1)
    b = synth.random_weights(m, 2)
    _compare(x, a, y, b, blur=0.1 * math.sqrt(d), reach=None, scaling=0.6, extra=2)
    _compare(x, a, y, b, blur=0.1 * math.sqrt(d), reach=1.0, scaling=0.6, extra=2)


def test_converged_mode_meets_tolerance():
    x, a, y, b = synth.blob_pair(1000, seed=12)
    S, pot, st = _run(x, a, y, b, 0.05, None, 0.5, tol=1e-4, max_iters=3000, check_every=2)
    assert st["converged"] == 1 and st["marginal_err"] <= 1e-4
    Sr, r = oracle.sinkhorn_divergence(x, a, y, b, 0.05, None, scaling=0.5, tol=1e-4,
                                       max_iters=3000, check_every=2)
    assert S == pytest.approx(Sr, rel=1e-4)


def test_bitwise_reproducible():
    x, a, y, b = synth.blob_pair(1000, seed=13)
    S1, p1, _ = _run(x, a, y, b, 0.02, 0.5, 0.5, extra=3)
    S2, p2, _ = _run(x, a, y, b, 0.02, 0.5, 0.5, extra=3)
    assert S1 == S2
    for k in p1:
        assert np.array_equal(p1[k], p2[k])


def test_self_divergence_zero_and_symmetry():
    x, a, y, b = synth.blob_pair(800, seed=14)
    S, _, _ = _run(x, a, x, a, 0.02, None, 0.5)
    assert abs(S) < 1e-6
    S1, _, _ = _run(x, a, y, b, 0.02, None, 0.5)
    S2, _, _ = _run(y, b, x, a, 0.02, None, 0.5)
    assert S1 == pytest.approx(S2, rel=1e-6)


def test_invalid_arguments():
    import paper_2107_02010_amd as skh
    x, a, y, b = synth.blob_pair(50, seed=15)
    bad = a.copy()
    bad[3] = -1.0
    note("invalid arguments")
    with pytest.raises(skh.SkhError) as e:
        skh.sinkhorn_divergence(cuda(x), cuda(bad), cuda(y), cuda(b), blur=0.1)
    assert e.value.code == -1
    xn = x.copy()
    xn[2, 1] = np.nan
    with pytest.raises(skh.SkhError) as e:
        skh.sinkhorn_divergence(cuda(xn), cuda(a), cuda(y), cuda(b), blur=0.1)
    assert e.value.code == -4
    with pytest.raises(skh.SkhError):
        skh.sinkhorn_divergence(cuda(x), cuda(a), cuda(y), cuda(b), blur=-1.0)
    with pytest.raises(skh.SkhError):
        skh.sinkhorn_divergence(cuda(x), cuda(a), cuda(y), cuda(b), blur=0.1, scaling=1.5)
    big = np.zeros((10, 64), np.float32)
    with pytest.raises(skh.SkhError):
        skh.sinkhorn_divergence(cuda(big), cuda(a[:10] * 5), cuda(big), cuda(a[:10] * 5), blur=0.1)


def test_weight_failures_and_not_converged():
    # NaN weight and zero total mass are argument errors; an iteration cap below what
    # the tolerance needs returns valid results with converged = 0 (SKH_NOT_CONVERGED)
    import ctypes

    import paper_2107_02010_amd as skh
    from paper_2107_02010_amd import _lib
    x, a, y, b = synth.blob_pair(60, seed=16)
    note("weight failures, not converged")
    an = a.copy()
    an[5] = np.nan
    with pytest.raises(skh.SkhError) as e:
        skh.sinkhorn_divergence(cuda(x), cuda(an), cuda(y), cuda(b), blur=0.1)
    assert e.value.code == _lib.SKH_EINVAL
    with pytest.raises(skh.SkhError) as e:
        skh.sinkhorn_divergence(cuda(x), cuda(np.zeros_like(a)), cuda(y), cuda(b), blur=0.1)
    assert e.value.code == _lib.SKH_EINVAL
    S, pot, st = skh.sinkhorn_divergence(cuda(x), cuda(a), cuda(y), cuda(b), blur=0.01,
                                         scaling=0.5, tol=1e-9, max_iters=3, potentials=True)
    # max_iters counts the iterations at blur after the scale list
    assert st["converged"] == 0 and st["iters"] == st["n_scales"] + 3
    assert st["marginal_err"] > 1e-9
    assert math.isfinite(S) and all(bool(v.isfinite().all()) for v in pot.values())
    with pytest.raises(skh.SkhError) as e:  # empty cloud
        skh.sinkhorn_divergence(cuda(x[:0]), cuda(a[:0]), cuda(y), cuda(b), blur=0.1)
    assert e.value.code == _lib.SKH_EINVAL
    # the C entry itself reports the positive status code
    P = _lib.default_params()
    P.blur, P.scaling, P.tol, P.max_iters = 0.01, 0.5, 1e-9, 3
    X, A, Y, B = cuda(x), cuda(a), cuda(y), cuda(b)
    out = ctypes.c_double()
    ctx = skh._Ctx.get(X.device)
    rc = _lib.load().skh_sinkhorn_divergence(ctx, X.data_ptr(), A.data_ptr(), len(x),
                                             Y.data_ptr(), B.data_ptr(), len(y), x.shape[1],
                                             ctypes.byref(P), ctypes.byref(out), None, None, None,
                                             None, None)
    assert rc == _lib.SKH_NOT_CONVERGED and math.isfinite(out.value)


# ------------------------------------------------------------- BF16 split ---

def test_fiber_downscaled_bf16_split():
    x, a, y, b = synth.fiber_pair(3000, 20, seed=7)
    S, Sr, st = _compare(x, a, y, b, blur=1.0, reach=None, scaling=0.8, precision="bf16x3")
    print(f"bf16 fibres: S={S:.9g} oracle={Sr:.9g} rel={abs(S - Sr) / abs(Sr):.2e}")


def test_fiber_downscaled_bf16_split_unbalanced():
    x, a, y, b = synth.fiber_pair(2500, 20, seed=9)
    _compare(x, a, y, b, blur=1.0, reach=20.0, scaling=0.8, extra=3, precision="bf16x3")


def test_blob_config_bf16_split():
    x, a, y, b = synth.blob_pair(2000, seed=0)
    _compare(x, a, y, b, blur=0.01, reach=None, scaling=0.5, precision="bf16x3")


@pytest.mark.parametrize("n,m,d", [(1, 1, 3), (1, 37, 2), (130, 1, 5), (257, 129, 1), (5, 300, 60)])
def test_edge_sizes_bf16(n, m, d):
    rng = np.random.default_rng(n + m + d)
    x = rng.standard_normal((n, d)).astype(np.float32)
    y = (rng.standard_normal((m, d)) + 0.5).astype(np.float32)
    a = synth.random_weights(n, 1)
    b = synth.random_weights(m, 2)
    _compare(x, a, y, b, blur=0.1 * math.sqrt(d), reach=None, scaling=0.6, extra=2,
             precision="bf16x3")


def test_workspace_limit():
    # a cap below what a solve needs fails with SKH_ENOMEM before the workspace grows and
    # leaves the context usable; without the cap the same solve runs
    import paper_2107_02010_amd as skh
    from paper_2107_02010_amd import _lib
    x, a, y, b = synth.blob_pair(3000, seed=17)
    X, A, Y, B = cuda(x), cuda(a), cuda(y), cuda(b)
    note("workspace limit")
    try:
        skh.set_workspace_limit(64 << 10)  # 64 KiB: a larger holding is freed
        assert skh.workspace_bytes() <= 64 << 10
        with pytest.raises(skh.SkhError) as e:
            skh.sinkhorn_divergence(X, A, Y, B, blur=0.05)
        assert e.value.code == _lib.SKH_ENOMEM and "workspace limit" in str(e.value)
        assert skh.workspace_bytes() <= 64 << 10
        skh.set_workspace_limit(0)
        S0 = skh.sinkhorn_divergence(X, A, Y, B, blur=0.05)
        held = skh.workspace_bytes()
        assert held > 64 << 10
        skh.set_workspace_limit(held)  # enough: the same solve runs within it
        assert skh.sinkhorn_divergence(X, A, Y, B, blur=0.05) == S0
        assert skh.workspace_bytes() <= held
    finally:
        skh.set_workspace_limit(0)
