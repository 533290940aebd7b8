"""GPU checks of the coarse-to-fine path (Section 2): K-means coarse phase, jump to
the fine points, cluster-block kernel truncation and the block-sparse softmin.

* no coarse phase and every block kept: the block-sparse machinery must give the
  dense result (oracle, same schedule), FP32 and BF16 split;
* truncation alone (theta = 20): entries dropped are below e^-20 of their row, so
  the result stays at the dense FP32 tolerance;
* full multiscale in converged mode reaches the same fixed point as the dense
  oracle (the coarse start and the truncation change the path, not the limit).
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import cuda, host, note

pytestmark = pytest.mark.gpu


def _run(x, a, y, b, **kw):
    import paper_2107_02010_amd as skh
    note(f"multiscale n={len(x)} m={len(y)} d={x.shape[1]} {kw}")
    S, pot, st = skh.sinkhorn_divergence(cuda(x), cuda(a), cuda(y), cuda(b), potentials=True, **kw)
    return S, {k: host(v) for k, v in pot.items()}, st


@pytest.mark.parametrize("precision,rtol", [("fp32", 1e-5), ("bf16x3", 1e-3)])
@pytest.mark.parametrize("reach", [None, 20.0])
def test_block_sparse_keep_all_equals_dense(precision, rtol, reach):
    x, a, y, b = synth.fiber_pair(3000, 20, seed=21)
    kw = dict(blur=1.0, reach=reach, scaling=0.8, extra_iters=2)
    S, pot, st = _run(x, a, y, b, multiscale=True, jump_scale=-1.0, trunc_theta=0.0,
                      precision=precision, **kw)
    Sr, r = oracle.sinkhorn_divergence(x, a, y, b, 1.0, reach, scaling=0.8, extra_iters=2)
    assert st["coarse_iters"] == 0 and st["iters"] == r["iters"]
    assert st["pairs"] == pytest.approx(st["dense_pairs"], rel=1e-12)
    assert S == pytest.approx(Sr, rel=rtol)


@pytest.mark.parametrize("reach", [None, 20.0])
def test_truncation_only_stays_at_fp32_tolerance(reach):
    x, a, y, b = synth.fiber_pair(4000, 25, seed=22)
    kw = dict(blur=1.0, reach=reach, scaling=0.8, extra_iters=3)
    S, pot, st = _run(x, a, y, b, multiscale=True, jump_scale=-1.0, trunc_theta=20.0, **kw)
    Sr, r = oracle.sinkhorn_divergence(x, a, y, b, 1.0, reach, scaling=0.8, extra_iters=3)
    print(f"truncation: kept {st['pairs'] / st['dense_pairs']:.3f} of the pairs, "
          f"S={S:.9g} oracle={Sr:.9g}")
    assert st["pairs"] < st["dense_pairs"]
    assert S == pytest.approx(Sr, rel=1e-5)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_full_multiscale_converges_to_dense_fixed_point(precision):
    # The averaged loop needs thousands of iterations at this tolerance, beyond
    # what the FP64 oracle finishes in seconds; the dense FP32 GPU path (pinned to
    # the oracle in schedule and converged mode elsewhere) is the reference here.
    x, a, y, b = synth.fiber_pair(4000, 25, seed=23)
    kw = dict(blur=1.0, reach=20.0, scaling=0.9, tol=1e-4, max_iters=20000, check_every=5)
    S, pot, st = _run(x, a, y, b, multiscale=True, precision=precision, **kw)
    Sd, potd, std = _run(x, a, y, b, **kw)
    print(f"multiscale {precision}: coarse iters {st['coarse_iters']}, fine iters "
          f"{st['iters'] - st['coarse_iters']}, kept {st['pairs'] / max(st['dense_pairs'], 1):.3f}, "
          f"S={S:.9g} dense={Sd:.9g} (dense iters {std['iters']})")
    assert st["converged"] == 1 and std["converged"] == 1
    assert st["coarse_iters"] > 0
    assert S == pytest.approx(Sd, rel=1e-5 if precision == "fp32" else 1e-3)
    # At a marginal tolerance tol the unbalanced potentials are pinned only up to
    # near-gauge shifts of about rho * tol (the e^{-f/rho} restoring term), per weakly
    # coupled group of points (here: per bundle), so only that bound is checked.
    rho, tol = 20.0 ** 2, 1e-4
    assert np.abs(pot["f"] - potd["f"]).max() <= 4 * rho * tol
    assert np.abs(pot["g"] - potd["g"]).max() <= 4 * rho * tol


def test_multiscale_200k_fibres_matches_dense_fp32():
    # The same comparison at the 200k-fibre shape of the benchmark (50 bundles, reach
    # 20 mm, marginal tolerance 1e-4): one dense FP32 solve against the multiscale
    # solves in FP32 and BF16 split.
    x, a, y, b = synth.fiber_pair(200_000, 50, seed=25)
    kw = dict(blur=1.0, reach=20.0, scaling=0.9, tol=1e-4, max_iters=20000, check_every=1)
    Sd, potd, std = _run(x, a, y, b, **kw)
    assert std["converged"] == 1
    rho, tol = 20.0 ** 2, 1e-4
    for precision, rtol in (("fp32", 1e-5), ("bf16x3", 1e-3)):
        S, pot, st = _run(x, a, y, b, multiscale=True, precision=precision, **kw)
        print(f"200k multiscale {precision}: kept {st['pairs'] / max(st['dense_pairs'], 1):.4f}, "
              f"S={S:.9g} dense={Sd:.9g} ({st['iters']} / {std['iters']} iterations)")
        assert st["converged"] == 1 and st["coarse_iters"] > 0
        assert st["pairs"] < 0.1 * st["dense_pairs"]
        assert S == pytest.approx(Sd, rel=rtol)
        assert np.abs(pot["f"] - potd["f"]).max() <= 4 * rho * tol
        assert np.abs(pot["g"] - potd["g"]).max() <= 4 * rho * tol


def test_multiscale_blob_config_balanced():
    x, a, y, b = synth.blob_pair(2000, seed=0)
    kw = dict(blur=0.01, reach=None, scaling=0.5)
    S, pot, st = _run(x, a, y, b, multiscale=True, jump_scale=-1.0, trunc_theta=20.0, **kw)
    Sr, r = oracle.sinkhorn_divergence(x, a, y, b, 0.01, None, scaling=0.5)
    assert S == pytest.approx(Sr, rel=1e-5)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_multiscale_fixed_self_loops_keep_the_cross_vectors(precision):
    # The self loops are independent of the cross loop (coarse loop, jump, masks and
    # fine loop alike): holding p, q fixed at any given values leaves f, g as in the
    # full multiscale solve with the same scale list, and drops the self problems'
    # pairs.
    import torch

    import paper_2107_02010_amd as skh
    x, a, y, b = synth.fiber_pair(5000, 25, seed=24)
    X, A, Y, B = cuda(x), cuda(a), cuda(y), cuda(b)
    kw = dict(blur=1.0, reach=20.0, scaling=0.8, extra_iters=3, multiscale=True,
              precision=precision, n_clusters=40)
    note(f"multiscale fixed self loops {precision}")
    S0, pot0, st0 = skh.sinkhorn_divergence(X, A, Y, B, potentials=True, **kw)
    zp, zq = torch.zeros(len(x), device="cuda"), torch.zeros(len(y), device="cuda")
    S1, pot1, st1 = skh.sinkhorn_divergence(X, A, Y, B, potentials=True,
                                            init=(None, None, zp, zq),
                                            fixed=skh.SKH_FIX_P | skh.SKH_FIX_Q, **kw)
    assert st1["iters"] == st0["iters"] and st1["coarse_iters"] == st0["coarse_iters"]
    assert st1["coarse_iters"] > 0
    assert st1["pairs"] < 0.75 * st0["pairs"]
    scale = max(1.0, float(torch.abs(pot0["f"]).max()))
    for k in ("f", "g"):
        assert torch.max(torch.abs(pot1[k] - pot0[k])).item() <= 1e-6 * scale
    assert torch.equal(pot1["p"], zp) and torch.equal(pot1["q"], zq)
    with pytest.raises(ValueError):  # a fixed vector left out
        skh.sinkhorn_divergence(X, A, Y, B, init=(None, None, None, zq),
                                fixed=skh.SKH_FIX_P | skh.SKH_FIX_Q, **kw)
    with pytest.raises(skh.SkhError):  # the cross loop cannot be fixed on this path
        skh.sinkhorn_divergence(X, A, Y, B, init=(pot0["f"], pot0["g"], None, None),
                                fixed=skh.SKH_FIX_CROSS, **kw)


def _fixed_point_deviation(rows_pts, cols_pts, cols_w, pot_rows, pot_cols, eps, rho):
    """Relative deviation of sampled rows from the unbalanced fixed point, with the FP64
    oracle's dense softmin over every column: the row mass of the plan over its target,
    r_i / (w_i e^{-f_i / rho}) - 1 = expm1((f_i - f~_i) / eps + f_i / rho), where
    f~_i = -eps log sum_j w_j exp((g_j - C_ij) / eps) (eq. (4) and the Algorithm's update
    with lambda = rho / (rho + eps): at the fixed point f = lambda f~)."""
    ft = oracle.softmin(rows_pts, cols_pts, cols_w, pot_cols, eps, 1.0)
    return np.abs(np.expm1((pot_rows - ft) / eps + pot_rows / rho))


def test_multiscale_1m_fibres_full_size():
    # The 1M x 1M fibre workload of the benchmark (200 bundles, blur 1 mm, reach 20 mm,
    # K-means sqrt(n) clusters, truncation theta 20, marginal tolerance 1e-4) in the two
    # configurations it times: plain FP32 multiscale and BF16 split + learned warm start.
    # S agrees within 1e-3; sampled rows and columns of every dual vector sit at the
    # fixed point of the dense problem, checked by the FP64 oracle against all 1M points
    # (no clustering, no truncation).
    import paper_2107_02010_amd as skh
    from paper_2107_02010_amd.warm_start import (DEFAULT_CHECKPOINT, WarmStartNet,
                                                 sinkhorn_divergence_warm)
    n = 1_000_000
    note("multiscale 1M fibres: generating the clouds")
    x, a, y, b = synth.fiber_pair(n, 200, seed=0)
    X, A, Y, B = cuda(x), cuda(a), cuda(y), cuda(b)
    kw = dict(reach=20.0, tol=1e-4, check_every=5, max_iters=20000, multiscale=True)
    note("multiscale 1M fibres: plain FP32 solve")
    S0, pot0, st0 = skh.sinkhorn_divergence(X, A, Y, B, blur=1.0, scaling=0.9, potentials=True,
                                            precision="fp32", **kw)
    note("multiscale 1M fibres: BF16 split + warm start")
    net = WarmStartNet.load(DEFAULT_CHECKPOINT, "cuda:0")
    S1, pot1, st1 = sinkhorn_divergence_warm(net, X, A, Y, B, 1.0, scaling=0.9,
                                             precision="bf16x3", **kw)
    assert st0["converged"] and st1["converged"] and st1["warm_fallback"] == 0
    assert st0["pairs"] < 0.2 * st0["dense_pairs"]
    print(f"S fp32 {S0:.9g} bf16+warm {S1:.9g} rel {abs(S1 - S0) / abs(S0):.2e}")
    assert abs(S1 - S0) <= 1e-3 * abs(S0)
    rng = np.random.default_rng(17)
    ri = np.sort(rng.choice(n, size=40, replace=False))
    ri[-1] = n - 1
    eps, rho = 1.0, 400.0
    # The stopping rule bounds the relative L1 marginal error by 1e-4 (measured by the
    # solver in its own precision): a sample's mean deviation stays within a few times
    # that, single rows within 50 times; the BF16 split adds its contraction error
    # (about 1e-4 of eps in f~ on clustered fibres).
    for tag, pot, mean_bound, max_bound in (("fp32", pot0, 5e-4, 5e-3),
                                            ("bf16x3+warm", pot1, 1e-3, 1e-2)):
        P = {k: host(v).astype(np.float64) for k, v in pot.items()}
        devs = [
            _fixed_point_deviation(x[ri], y, b, P["f"][ri], P["g"], eps, rho),  # f vs g
            _fixed_point_deviation(y[ri], x, a, P["g"][ri], P["f"], eps, rho),  # g vs f
            _fixed_point_deviation(x[ri], x, a, P["p"][ri], P["p"], eps, rho),  # p vs p
            _fixed_point_deviation(y[ri], y, b, P["q"][ri], P["q"], eps, rho),  # q vs q
        ]
        for name, dv in zip("fgpq", devs):
            print(f"{tag} {name}: mean deviation {dv.mean():.2e}, max {dv.max():.2e}")
            assert np.all(np.isfinite(dv))
            assert dv.mean() <= mean_bound and dv.max() <= max_bound, (tag, name)
