"""Pins of the oracle's trajectory (not only its fixed point) and of its barycenter descent.

The fixed point of the symmetric loop does not depend on the weight of the averaging
step of the Algorithm (a <- (a + a~)/2): every fixed-point pin holds for any weight in
(0, 1].  The schedule-mode GPU parity tests, however, compare trajectories at equal
iteration counts, so the weight and the order of the updates are pinned here by
iterates written out by hand from the Algorithm's definition on single Diracs, where
each softmin has one term and the log-sum-exp is exact:

  one point y of weight b seen from x:  -lam eps log(b exp((h - C)/eps)) = lam (C - h - eps log b).

The barycenter descent of Section 3 (track density atlas) is pinned on Dirac maps, where
the balanced cross plan moves all of the support's mass to the map's point, so that
grad_x S = x - y for each map and a unit step lands on the maps' mean.
"""
import math

import numpy as np
import pytest

import oracle


def _dirac_iterates(C, a, b, sigmas, reach):
    """f, g, p, q after one iteration per scale in `sigmas`, from zero, for alpha = a delta_x
    and beta = b delta_y with C = C(x, y): the Algorithm's four tilde updates from the same
    old values (Jacobi), then the half-way averages."""
    f = g = p = q = 0.0
    for s in sigmas:
        eps = s * s
        lam = 1.0 if reach is None else 1.0 / (1.0 + eps / reach ** 2)
        pt = lam * (0.0 - p - eps * math.log(a))      # alpha <-> alpha: C(x, x) = 0
        qt = lam * (0.0 - q - eps * math.log(b))      # beta <-> beta
        gt = lam * (C - f - eps * math.log(a))        # alpha -> beta
        ft = lam * (C - g - eps * math.log(b))        # beta -> alpha
        f, g, p, q = 0.5 * (f + ft), 0.5 * (g + gt), 0.5 * (p + pt), 0.5 * (q + qt)
    return f, g, p, q


@pytest.mark.parametrize("reach", [None, 0.7])
def test_first_iteration_is_half_of_the_softmin(reach):
    # One iteration at sigma = blur from zero: every vector is half its softmin,
    # p = -lam eps log(a) / 2, f = lam (C - eps log b) / 2, and so on.
    x = np.array([[0.3, -0.2]])
    y = np.array([[1.1, 0.4]])
    a, b, blur = 0.6, 1.7, 0.5
    C = 0.5 * float(np.sum((x - y) ** 2))
    r = oracle.sinkhorn(x, [a], y, [b], blur, reach, scaling=0.5, diam=0.1 * blur)
    assert r["iters"] == 1 and r["n_scales"] == 1
    eps = blur * blur
    lam = 1.0 if reach is None else 1.0 / (1.0 + eps / reach ** 2)
    assert r["p"][0] == pytest.approx(-0.5 * lam * eps * math.log(a), rel=1e-14)
    assert r["q"][0] == pytest.approx(-0.5 * lam * eps * math.log(b), rel=1e-14)
    assert r["f"][0] == pytest.approx(0.5 * lam * (C - eps * math.log(b)), rel=1e-14)
    assert r["g"][0] == pytest.approx(0.5 * lam * (C - eps * math.log(a)), rel=1e-14)


@pytest.mark.parametrize("reach", [None, 0.7])
@pytest.mark.parametrize("extra", [1, 3])
def test_iterates_on_two_scales_written_out(reach, extra):
    # Scale list [d, blur] (d = 2 blur, q = 1/2), then `extra` iterations at blur: the
    # iterates of the Dirac problem by hand, including the change of eps and lambda.
    x = np.array([[0.0, 0.0, 0.5]])
    y = np.array([[0.9, -0.3, 0.1]])
    a, b, blur = 0.45, 2.2, 0.8
    C = 0.5 * float(np.sum((x - y) ** 2))
    r = oracle.sinkhorn(x, [a], y, [b], blur, reach, scaling=0.5, diam=2.0 * blur,
                        extra_iters=extra)
    assert r["n_scales"] == 2 and r["iters"] == 2 + extra
    f, g, p, q = _dirac_iterates(C, a, b, [2.0 * blur] + [blur] * (1 + extra), reach)
    for got, want in ((r["f"][0], f), (r["g"][0], g), (r["p"][0], p), (r["q"][0], q)):
        assert got == pytest.approx(want, rel=1e-13, abs=1e-15)


def test_second_iteration_balanced_closed_form():
    # Balanced, one scale, two iterations: f2 = C/2 - 3/4 eps log b + 1/4 eps log a and
    # g2 = C/2 - 3/4 eps log a + 1/4 eps log b; p and q sit at -eps log(.)/2 from the
    # first iteration on.  A weight w != 1/2 in the averaging step moves every one.
    x = np.array([[0.2]])
    y = np.array([[-0.9]])
    a, b, blur = 0.3, 1.9, 0.6
    C = 0.5 * (0.2 + 0.9) ** 2
    eps = blur * blur
    r = oracle.sinkhorn(x, [a], y, [b], blur, None, scaling=0.5, diam=0.5 * blur, extra_iters=1)
    assert r["iters"] == 2
    la, lb = math.log(a), math.log(b)
    assert r["f"][0] == pytest.approx(0.5 * C - 0.75 * eps * lb + 0.25 * eps * la, rel=1e-14)
    assert r["g"][0] == pytest.approx(0.5 * C - 0.75 * eps * la + 0.25 * eps * lb, rel=1e-14)
    assert r["p"][0] == pytest.approx(-0.5 * eps * la, rel=1e-14)
    assert r["q"][0] == pytest.approx(-0.5 * eps * lb, rel=1e-14)


def test_two_point_cloud_first_iteration():
    # Two points against one: after one iteration from zero each vector is half its
    # softmin, where the two-term log-sum-exp of a point against its own cloud is
    # log(a_1 + a_2 e^{-c/eps}) with c = |x_1 - x_2|^2 / 2.
    x = np.array([[0.0, 0.0], [0.6, 0.8]])      # |x_1 - x_2| = 1
    y = np.array([[2.0, 0.0]])
    a = np.array([0.25, 0.5])
    b = np.array([0.75])
    blur = 0.9
    eps = blur * blur
    r = oracle.sinkhorn(x, a, y, b, blur, None, scaling=0.5, diam=0.5 * blur)
    assert r["iters"] == 1
    c12 = 0.5
    p1 = -0.5 * eps * math.log(a[0] + a[1] * math.exp(-c12 / eps))
    p2 = -0.5 * eps * math.log(a[1] + a[0] * math.exp(-c12 / eps))
    C1, C2 = 0.5 * 4.0, 0.5 * (1.4 ** 2 + 0.8 ** 2)
    f1 = 0.5 * (C1 - eps * math.log(b[0]))
    f2 = 0.5 * (C2 - eps * math.log(b[0]))
    g = -0.5 * eps * math.log(a[0] * math.exp(-C1 / eps) + a[1] * math.exp(-C2 / eps))
    q = -0.5 * eps * math.log(b[0])
    np.testing.assert_allclose(r["p"], [p1, p2], rtol=1e-14)
    np.testing.assert_allclose(r["f"], [f1, f2], rtol=1e-14)
    np.testing.assert_allclose(r["g"], [g], rtol=1e-14)
    np.testing.assert_allclose(r["q"], [q], rtol=1e-14)


# ------------------------------------------------------------- barycenter --

def test_barycenter_step_on_dirac_maps_lands_on_their_mean():
    # Support: two coincident points of weight 1/2 (one unit Dirac split in two); maps:
    # three unit Diracs y_k.  Balanced, so each cross plan sends all of a_i to y_k and
    # the self plan moves nothing: grad_{x_i} S_k = a_i (x - y_k).  The step
    # x <- x - lr mean_k grad / a_i gives x - lr (x - mean_k y_k); S_k = |x - y_k|^2 / 2.
    x0 = np.array([[0.5, -1.0, 2.0], [0.5, -1.0, 2.0]])
    a = np.array([0.5, 0.5])
    ys = [np.array([[1.5, 0.0, 2.0]]), np.array([[0.0, -2.0, 3.0]]), np.array([[-1.0, 1.0, 1.0]])]
    maps = [(y, np.array([1.0])) for y in ys]
    ybar = np.mean(np.concatenate(ys), axis=0)
    for lr in (1.0, 0.25):
        x1, hist = oracle.barycenter_steps(x0, a, maps, 1, blur=0.3, lr=lr, scaling=0.5)
        want = x0[0] - lr * (x0[0] - ybar)
        np.testing.assert_allclose(x1, np.stack([want, want]), rtol=0, atol=1e-12)
        S_want = np.mean([0.5 * np.sum((x0[0] - y[0]) ** 2) for y in ys])
        assert hist[0] == pytest.approx(S_want, rel=1e-12)


def test_barycenter_two_steps_geometric_approach():
    # With lr = 1/2 on one Dirac map the distance to y halves at every step, and the
    # S history is |x_t - y|^2 / 2 = |x_0 - y|^2 / 2 * 4^{-t}.
    x0 = np.array([[1.0, 2.0]])
    y = np.array([[-1.0, 0.0]])
    x2, hist = oracle.barycenter_steps(x0, np.array([1.0]), [(y, np.array([1.0]))], 2,
                                       blur=0.2, lr=0.5, scaling=0.5)
    np.testing.assert_allclose(x2, y + 0.25 * (x0 - y), rtol=0, atol=1e-12)
    S0 = 0.5 * float(np.sum((x0 - y) ** 2))
    assert hist[0] == pytest.approx(S0, rel=1e-12)
    assert hist[1] == pytest.approx(S0 / 4.0, rel=1e-12)


def test_barycenter_warm_steps_on_dirac_maps_stay_geometric():
    # A warm start changes where each step's loops begin, not what the Dirac gradient is:
    # the distance to y still halves at every step with lr = 1/2.
    x0 = np.array([[1.0, 2.0]])
    y = np.array([[-1.0, 0.0]])
    x3, hist = oracle.barycenter_steps(x0, np.array([1.0]), [(y, np.array([1.0]))], 3,
                                       blur=0.2, lr=0.5, scaling=0.5, start_scale=0.4)
    np.testing.assert_allclose(x3, y + 0.125 * (x0 - y), rtol=0, atol=1e-12)
    S0 = 0.5 * float(np.sum((x0 - y) ** 2))
    np.testing.assert_allclose(hist, [S0, S0 / 4.0, S0 / 16.0], rtol=1e-12)


def test_barycenter_warm_steps_reach_the_cold_fixed_points():
    # With enough iterations at blur every step's loops converge, so the warm-started
    # descent (loops started from the previous step's vectors, q_k held) takes the same
    # steps as the cold one.  S differs only by the balanced gauge of (f, g), which the
    # warm start inherits: c * (sum a - sum b), with the FP32 weights' sums off 1 by ~1e-8.
    import synth
    maps = synth.density_maps(2, seed=1, grid=12, n_tubes=2, nonzero=(60, 90),
                              sigma=(1.0, 1.5), jitter=1.0)
    x0, a = synth.barycenter_support(maps, 40, seed=2)
    kw = dict(blur=1.0, scaling=0.7, extra_iters=1000, diam=20.0)
    xc, hc = oracle.barycenter_steps(x0, a, maps, 2, **kw)
    xw, hw = oracle.barycenter_steps(x0, a, maps, 2, start_scale=3.0, **kw)
    np.testing.assert_allclose(xw, xc, rtol=0, atol=1e-10)
    np.testing.assert_allclose(hw, hc, rtol=1e-8)
    # the warm start matters on the Algorithm's schedule alone (one iteration per scale)
    xs, _ = oracle.barycenter_steps(x0, a, maps, 2, start_scale=3.0,
                                    **dict(kw, extra_iters=0))
    assert np.abs(xs - xc).max() > 1e-3
