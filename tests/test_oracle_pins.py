"""Pins of the FP64 oracle against facts fixed by the paper and by the mathematics.

Each test names what pins it: a closed form, an invariant, a limit, a special
case reducing to a textbook routine, or brute force on tiny inputs.  Together
they are chosen so that a dropped term, a wrong sign, a wrong index or a
transposed operand anywhere in the oracle fails at least one of them.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
import synth


def _conv(x, a, y, b, blur, reach=None, scaling=0.5, tol=1e-13, max_iters=20000):
    S, r = oracle.sinkhorn_divergence(x, a, y, b, blur, reach, scaling=scaling, tol=tol,
                                      max_iters=max_iters, check_every=1)
    assert r["converged"] or tol >= 1e-6, r["marginal_err"]
    return S, r


def _w(n, seed, total=1.0):
    """Random positive FP64 weights summing to ``total`` exactly enough for a balanced
    problem (FP32 weights normalised in FP32 leave a mass gap near 1e-8, and the
    balanced problem has no fixed point unless the two masses agree)."""
    w = synth.random_weights(n, seed).astype(np.float64)
    return w * (total / w.sum())


def _u(n):
    return np.full(n, 1.0 / n)


# ---------------------------------------------------------------- schedule --

def test_schedule_worked_example():
    # Algorithm loop header: [d, d q, d q^2, ..., blur] with ceil(log(d/blur)/log(1/q))
    # multiplicative steps; d = 1.9, blur = 0.01, q = 0.5 gives ceil(7.57) = 8 steps.
    s = oracle.schedule(1.9, 0.01, 0.5)
    expect = [1.9, 0.95, 0.475, 0.2375, 0.11875, 0.059375, 0.0296875, 0.01484375, 0.01]
    np.testing.assert_allclose(s, expect, rtol=1e-15)


def test_schedule_default_scaling_length():
    # q = 0.9 (the Algorithm's default), d = 260, blur = 1: ceil(52.78) = 53 steps.
    s = oracle.schedule(260.0, 1.0, 0.9)
    assert len(s) == 54 and s[-1] == 1.0 and s[0] == 260.0
    assert np.all(s[:-1] > 1.0)
    np.testing.assert_allclose(s[1:-1] / s[:-2], 0.9, rtol=1e-12)


def test_schedule_degenerate():
    assert list(oracle.schedule(0.5, 1.0, 0.9)) == [1.0]
    assert list(oracle.schedule(1.0, 1.0, 0.9)) == [1.0]


def test_diameter_is_box_diagonal():
    x = np.array([[0.0, 0.0, 0.0], [0.5, 0.1, 0.2]])
    y = np.array([[1.0, 2.0, 2.0]])
    assert oracle.diameter(x, y) == pytest.approx(3.0, rel=1e-15)
    # upper bound on the largest pairwise distance
    rng = np.random.default_rng(0)
    x, y = rng.normal(size=(30, 4)), rng.normal(size=(20, 4))
    dmax = np.sqrt(((x[:, None] - y[None]) ** 2).sum(-1)).max()
    assert oracle.diameter(x, y) >= dmax


# ----------------------------------------------------------------- softmin --

def test_softmin_single_column_closed_form():
    # m = 1: -lam eps log(w exp((h - C)/eps)) = lam (C - h - eps log w)
    rng = np.random.default_rng(1)
    r = rng.normal(size=(7, 5))
    c = rng.normal(size=(1, 5))
    w, h, eps, lam = np.array([0.3]), np.array([0.7]), 0.05, 0.8
    C = 0.5 * ((r - c) ** 2).sum(1)
    out = oracle.softmin(r, c, w, h, eps, lam)
    np.testing.assert_allclose(out, lam * (C - h[0] - eps * math.log(w[0])), rtol=1e-13)


def test_softmin_small_eps_is_hard_min():
    # eps -> 0 with uniform weights 1/m: min_j (C_ij - h_j) <= out/lam <= min + eps log m
    rng = np.random.default_rng(2)
    r, c = rng.normal(size=(9, 3)), rng.normal(size=(11, 3))
    h = rng.normal(size=11)
    w = np.full(11, 1.0 / 11)
    C = 0.5 * ((r[:, None] - c[None]) ** 2).sum(-1)
    hard = (C - h[None]).min(1)
    for eps in (1e-2, 1e-4):
        out = oracle.softmin(r, c, w, h, eps, 1.0)
        assert np.all(out >= hard - 1e-12)
        assert np.all(out <= hard + eps * math.log(11) + 1e-12)
    np.testing.assert_allclose(oracle.softmin(r, c, w, h, 1e-6, 0.5), 0.5 * hard, atol=1e-5)


def test_softmin_large_eps_expansion():
    # eps -> inf: out/lam = -eps log W + <w/W, C - h> - Var_w(C - h)/(2 eps) + O(eps^-2)
    rng = np.random.default_rng(3)
    r, c = rng.normal(size=(4, 2)), rng.normal(size=(6, 2))
    w, h = rng.uniform(0.1, 1, 6), rng.normal(size=6)
    W = w.sum()
    t = 0.5 * ((r[:, None] - c[None]) ** 2).sum(-1) - h[None]
    mean = (t * w).sum(1) / W
    var = ((t - mean[:, None]) ** 2 * w).sum(1) / W
    eps = 1e3
    out = oracle.softmin(r, c, w, h, eps, 1.0)
    approx = -eps * math.log(W) + mean - var / (2 * eps)
    np.testing.assert_allclose(out, approx, atol=1e-6)


def test_softmin_invariances():
    rng = np.random.default_rng(4)
    r, c = rng.normal(size=(8, 3)), rng.normal(size=(10, 3))
    w, h = rng.uniform(0.1, 1, 10), rng.normal(size=10)
    eps, lam = 0.3, 0.7
    base = oracle.softmin(r, c, w, h, eps, lam)
    # shift of the potential: out(h + s) = out(h) - lam s
    np.testing.assert_allclose(oracle.softmin(r, c, w, h + 0.25, eps, lam), base - lam * 0.25,
                               rtol=1e-12, atol=1e-12)
    # scaling of the weights: out(t w) = out(w) - lam eps log t
    np.testing.assert_allclose(oracle.softmin(r, c, 3.0 * w, h, eps, lam),
                               base - lam * eps * math.log(3.0), rtol=1e-12, atol=1e-12)
    # column order is irrelevant, rows are independent
    perm = rng.permutation(10)
    np.testing.assert_allclose(oracle.softmin(r, c[perm], w[perm], h[perm], eps, lam), base,
                               rtol=1e-13)
    np.testing.assert_allclose(oracle.softmin(r[::-1], c, w, h, eps, lam), base[::-1], rtol=1e-13)
    # zero-weight columns drop out; translation of both clouds changes nothing
    w0 = w.copy()
    w0[[1, 4]] = 0.0
    keep = np.array([k not in (1, 4) for k in range(10)])
    np.testing.assert_allclose(oracle.softmin(r, c, w0, h, eps, lam),
                               oracle.softmin(r, c[keep], w[keep], h[keep], eps, lam), rtol=1e-13)
    shift = np.array([5.0, -3.0, 2.0])
    np.testing.assert_allclose(oracle.softmin(r + shift, c + shift, w, h, eps, lam), base,
                               rtol=1e-11, atol=1e-11)


def test_softmin_no_mass_row_is_inf():
    out = oracle.softmin(np.zeros((2, 2)), np.ones((3, 2)), np.zeros(3), np.zeros(3), 1.0)
    assert np.all(np.isinf(out)) and np.all(out > 0)


# ------------------------------------------------------- single Diracs ------

@pytest.mark.parametrize("blur", [0.05, 0.5, 3.0])
def test_dirac_balanced(blur):
    # n = m = 1, unit masses: the only plan moves all mass, S = |x - y|^2 / 2 for any eps;
    # the symmetric loop started at zero keeps f = g, so f = g = C/2 and p = q = 0.
    x = np.array([[0.1, 0.2, 0.3, -1.0]])
    y = np.array([[0.5, -0.1, 0.7, 0.2]])
    C = 0.5 * ((x - y) ** 2).sum()
    S, r = _conv(x, [1.0], y, [1.0], blur)
    assert S == pytest.approx(C, rel=1e-12)
    np.testing.assert_allclose([r["f"][0], r["g"][0]], [C / 2, C / 2], rtol=1e-12)
    np.testing.assert_allclose([r["p"][0], r["q"][0]], [0.0, 0.0], atol=1e-14)


def _dirac_ot(a, b, C, eps, rho):
    # Minimiser of eq. (2) for one Dirac each (masses a, b): setting the derivative of
    # pi C + eps KL(pi, ab) + rho KL(pi, a) + rho KL(pi, b) to zero gives
    # pi = (ab)^((eps+rho)/(eps+2rho)) exp(-C/(eps+2rho)), value eps ab + rho(a+b) - (eps+2rho) pi.
    pi = (a * b) ** ((eps + rho) / (eps + 2 * rho)) * math.exp(-C / (eps + 2 * rho))
    return eps * a * b + rho * (a + b) - (eps + 2 * rho) * pi


@pytest.mark.parametrize("a,b", [(1.0, 1.0), (0.6, 1.7), (2.0, 0.3)])
@pytest.mark.parametrize("blur,reach", [(0.1, 0.5), (0.4, 0.3), (1.0, 5.0)])
def test_dirac_unbalanced_closed_form(a, b, blur, reach):
    # eq. (5) from the closed-form minimiser of eq. (2), including the mass term
    # eps/2 (a - b)^2; the oracle computes S by eq. (6) from the loop's fixed point.
    x = np.array([[0.3, -0.2]])
    y = np.array([[-0.1, 0.4]])
    C = 0.5 * ((x - y) ** 2).sum()
    eps, rho = blur ** 2, reach ** 2
    expect = (_dirac_ot(a, b, C, eps, rho) - 0.5 * _dirac_ot(a, a, 0.0, eps, rho)
              - 0.5 * _dirac_ot(b, b, 0.0, eps, rho) + 0.5 * eps * (a - b) ** 2)
    S, r = _conv(x, [a], y, [b], blur, reach)
    assert S == pytest.approx(expect, rel=1e-11, abs=1e-14)
    if a == b == 1.0:
        # f = g = rho C / (eps + 2 rho): fixed point of f = lam (C - g), lam = rho/(rho+eps)
        np.testing.assert_allclose(r["f"], rho * C / (eps + 2 * rho), rtol=1e-11)
        assert S == pytest.approx((eps + 2 * rho) * (1 - math.exp(-C / (eps + 2 * rho))),
                                  rel=1e-11)


# ------------------------------------------------- identities, symmetry ------

@pytest.mark.parametrize("blur", [0.2, 0.3])
def test_translation_identity(blur):
    # Translations are retrieved exactly (Introduction): for unit masses,
    # S(alpha, alpha + t) = |t|^2 / 2 for any eps, and more generally
    # S(alpha, beta + t) = S(alpha, beta) - (xbar - ybar).t + |t|^2/2.
    x = synth.random_cloud(12, 3, seed=5, scale=0.3).astype(np.float64)
    a = _w(12, seed=6)
    t = np.array([0.4, -0.25, 0.1])
    S, _ = _conv(x, a, x + t, a, blur)
    assert S == pytest.approx(0.5 * (t ** 2).sum(), rel=1e-9)
    y = synth.random_cloud(9, 3, seed=7, scale=0.3).astype(np.float64) + 0.2
    b = np.full(9, 1.0 / 9)
    S0, _ = _conv(x, a, y, b, blur)
    S1, _ = _conv(x, a, y + t, b, blur)
    xbar, ybar = (a[:, None] * x).sum(0), (b[:, None] * y).sum(0)
    assert S1 == pytest.approx(S0 - (xbar - ybar) @ t + 0.5 * (t ** 2).sum(), rel=1e-9)


@pytest.mark.parametrize("reach", [None, 0.4])
def test_self_zero_symmetry_positivity(reach):
    x, _, y, _ = synth.blob_pair(40, seed=8)
    a, b = _u(40), _u(40)
    x, y = x.astype(np.float64), y.astype(np.float64)
    a = _u(40)
    b = _w(40, seed=9, total=1.3 if reach else 1.0)
    Sxx, _ = _conv(x, a, x, a, 0.05, reach)
    assert abs(Sxx) < 1e-12
    Sxy, _ = _conv(x, a, y, b, 0.05, reach)
    Syx, _ = _conv(y, b, x, a, 0.05, reach)
    assert Sxy > 0
    assert Sxy == pytest.approx(Syx, rel=1e-11)


def test_zero_weight_points_drop_out():
    x, _, y, _ = synth.blob_pair(20, seed=10)
    a, b = _u(20), _u(20)
    a = a.copy()
    a[[3, 7]] = 0.0
    a /= a.sum()
    keep = a > 0
    S0, _ = _conv(x, a, y, b, 0.1)
    S1, _ = _conv(x[keep], a[keep], y, b, 0.1, tol=1e-13)
    # the diameter is the same (box of all points); the fixed point does not depend on it
    assert S0 == pytest.approx(S1, rel=1e-10)


# -------------------------------------------------------- limits of eps ------

def test_small_eps_brute_force_permutations():
    # eps -> 0: OT_0 <= OT_eps <= OT_0 + eps log n for uniform n = m (a permutation plan
    # has KL = log n), and 0 <= OT_eps(alpha, alpha) <= eps log n, so
    # |S_eps - OT_0| <= eps log n.  OT_0 of eq. (1) by enumerating all n! permutations.
    n = 6
    rng = np.random.default_rng(11)
    x, y = rng.uniform(size=(n, 2)), rng.uniform(size=(n, 2))
    C = 0.5 * ((x[:, None] - y[None]) ** 2).sum(-1)
    ot0 = min(sum(C[i, s[i]] for i in range(n)) / n for s in itertools.permutations(range(n)))
    w = np.full(n, 1.0 / n)
    for blur in (0.05, 0.02):
        eps = blur ** 2
        S, _ = _conv(x, w, y, w, blur, scaling=0.7, tol=1e-6)
        assert abs(S - ot0) <= eps * math.log(n) + 1e-12
    S, _ = _conv(x, w, y, w, 0.005, scaling=0.7, tol=1e-6)
    assert S == pytest.approx(ot0, rel=2e-3)


def test_small_eps_sorted_matching_1d():
    # 1-D, uniform, equal sizes: the optimal matching pairs sorted samples.
    n = 40
    rng = np.random.default_rng(12)
    x, y = rng.normal(size=n), rng.normal(0.5, 1.3, size=n)
    ot0 = 0.5 * np.mean((np.sort(x) - np.sort(y)) ** 2)
    w = np.full(n, 1.0 / n)
    blur = 0.02
    S, _ = _conv(x, w, y, w, blur, scaling=0.7, tol=1e-6)
    assert abs(S - ot0) <= blur ** 2 * math.log(n) + 1e-12


def test_large_eps_mmd_limit():
    # eps -> inf: S_eps -> |xbar - ybar|^2 / 2 for unit masses (energy-distance limit
    # of the debiased divergence); the gap is O(diam^4 / eps).
    x, _, y, _ = synth.blob_pair(30, seed=13)
    x, y, a, b = x.astype(np.float64), y.astype(np.float64), _u(30), _u(30)
    xbar, ybar = (a[:, None] * x).sum(0), (b[:, None] * y).sum(0)
    S, _ = _conv(x, a, y, b, blur=200.0)
    assert S == pytest.approx(0.5 * ((xbar - ybar) ** 2).sum(), rel=1e-4)


def test_reach_to_infinity_recovers_balanced():
    x, _, y, _ = synth.blob_pair(25, seed=14)
    a, b = _u(25), _u(25)
    Sb, _ = _conv(x, a, y, b, 0.1)
    Su, _ = _conv(x, a, y, b, 0.1, reach=1e4, tol=1e-10)
    assert Su == pytest.approx(Sb, rel=1e-6)


# ------------------------------------------------------------ fixed point ----

@pytest.mark.parametrize("reach", [None, 0.3])
def test_fixed_point_marginals(reach):
    # First-order conditions of eq. (3): pi 1 = alpha e^{-f/rho}, pi^T 1 = beta e^{-g/rho}
    # (alpha, beta when balanced), pi from eq. (4).
    x, _, y, _ = synth.blob_pair(30, seed=15)
    a, b = _u(30), _u(30)
    a = _u(30)
    b = _w(30, seed=16, total=1.0 if reach is None else 0.8)
    blur = 0.08
    S, r = _conv(x, a, y, b, blur, reach, tol=1e-14)
    row, col = oracle.marginals(x, a, y, b, r["f"], r["g"], blur ** 2)
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    ta = a64 if reach is None else a64 * np.exp(-r["f"] / reach ** 2)
    tb = b64 if reach is None else b64 * np.exp(-r["g"] / reach ** 2)
    np.testing.assert_allclose(row, ta, rtol=1e-9)
    np.testing.assert_allclose(col, tb, rtol=1e-9)
    # same for the two symmetric problems
    rp, _ = oracle.marginals(x, a, x, a, r["p"], r["p"], blur ** 2)
    ta_p = a64 if reach is None else a64 * np.exp(-r["p"] / reach ** 2)
    np.testing.assert_allclose(rp, ta_p, rtol=1e-9)


@pytest.mark.parametrize("reach", [None, 0.3])
def test_strong_duality(reach):
    # Primal eq. (2) at the plan of eq. (4) equals the dual eq. (3) at the optimum.
    x, _, y, _ = synth.blob_pair(25, seed=17)
    a, b = _u(25), _u(25)
    a = _u(25)
    b = _w(25, seed=18, total=1.0 if reach is None else 1.4)
    blur = 0.1
    S, r = _conv(x, a, y, b, blur, reach, tol=1e-14)
    eps = blur ** 2
    dual = oracle.ot_dual(x, a, y, b, r["f"], r["g"], eps, reach)
    primal = oracle.ot_primal(x, a, y, b, r["f"], r["g"], eps, reach)
    assert primal == pytest.approx(dual, rel=1e-9)


@pytest.mark.parametrize("reach,mb", [(None, 1.0), (0.3, 1.5), (1.0, 0.7)])
def test_eq5_equals_eq6(reach, mb):
    # The dual form eq. (6) and the definition eq. (5) (each OT by eq. (3)) agree at the
    # fixed point, including the mass term when the total masses differ.
    x, _, y, _ = synth.blob_pair(20, seed=19)
    a, b = _u(20), _u(20)
    a = _u(20)
    b = _w(20, seed=20, total=mb)
    blur = 0.1
    S6, r = _conv(x, a, y, b, blur, reach, tol=1e-14)
    S5 = oracle.divergence_eq5(x, a, y, b, r["f"], r["g"], r["p"], r["q"], blur, reach)
    assert S6 == pytest.approx(S5, rel=1e-9)


def _alternating_sinkhorn(x, a, y, b, eps, rho, iters=20000):
    """Textbook alternating (IPFP) Sinkhorn in the log domain, written here with numpy.

    For the unbalanced problem each half-step is damped by rho/(rho+eps)
    (Chizat et al.); it shares no code with the oracle and reaches the optimum
    of eq. (3) by a different route than the symmetric averaged loop."""
    C = 0.5 * ((x[:, None] - y[None]) ** 2).sum(-1)
    lam = 1.0 if rho is None else rho / (rho + eps)
    f, g = np.zeros(len(a)), np.zeros(len(b))
    la, lb = np.log(a), np.log(b)
    for _ in range(iters):
        s = lb[None] + (g[None] - C) / eps
        mx = s.max(1)
        f = -lam * eps * (mx + np.log(np.exp(s - mx[:, None]).sum(1)))
        s = la[:, None] + (f[:, None] - C) / eps
        mx = s.max(0)
        g_new = -lam * eps * (mx + np.log(np.exp(s - mx[None]).sum(0)))
        if np.max(np.abs(g_new - g)) < 1e-15:
            g = g_new
            break
        g = g_new
    return f, g


@pytest.mark.parametrize("reach", [None, 0.5])
def test_alternating_sinkhorn_reaches_same_ot(reach):
    x, _, y, _ = synth.blob_pair(15, seed=21)
    a, b = _u(15), _u(15)
    x, y = x.astype(np.float64), y.astype(np.float64)
    a, b = _u(15), _w(15, 22)
    blur = 0.15
    eps = blur ** 2
    rho = None if reach is None else reach ** 2
    f1, g1 = _alternating_sinkhorn(x, a, y, b, eps, rho)
    S, r = _conv(x, a, y, b, blur, reach, tol=1e-14)
    d_alt = oracle.ot_dual(x, a, y, b, f1, g1, eps, reach)
    d_sym = oracle.ot_dual(x, a, y, b, r["f"], r["g"], eps, reach)
    assert d_sym == pytest.approx(d_alt, rel=1e-10)
    if reach is not None:  # unique potentials when unbalanced
        np.testing.assert_allclose(r["f"], f1, rtol=1e-8, atol=1e-12)


def test_schedule_mode_iteration_count():
    x, _, y, _ = synth.blob_pair(10, seed=23)
    a, b = _u(10), _u(10)
    r = oracle.sinkhorn(x, a, y, b, blur=0.01, scaling=0.5, extra_iters=3)
    assert r["iters"] == r["n_scales"] + 3
    assert r["n_scales"] == len(oracle.schedule(oracle.diameter(x, y), 0.01, 0.5))


# ---------------------------------------------------------------- gradient ---

@pytest.mark.parametrize("reach", [None, 0.6])
def test_gradient_finite_differences(reach):
    rng = np.random.default_rng(24)
    x, y = rng.uniform(size=(5, 2)), rng.uniform(size=(6, 2))
    a, b = _u(5), _w(6, 25)
    blur = 0.2
    S, r = _conv(x, a, y, b, blur, reach, tol=1e-15, scaling=0.5)
    G = oracle.grad_x(x, a, y, b, r["f"], r["g"], r["p"], blur ** 2)
    h = 1e-5
    fd = np.zeros_like(x)
    for i in range(5):
        for k in range(2):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            Sp, _ = _conv(xp, a, y, b, blur, reach, tol=1e-15)
            Sm, _ = _conv(xm, a, y, b, blur, reach, tol=1e-15)
            fd[i, k] = (Sp - Sm) / (2 * h)
    np.testing.assert_allclose(G, fd, rtol=1e-5, atol=1e-9)


def test_gradient_sum_and_dirac():
    # Balanced, unit masses: sum_i grad_i = xbar - ybar (derivative of the translation identity).
    x, _, y, _ = synth.blob_pair(20, seed=26)
    x, y, a, b = x.astype(np.float64), y.astype(np.float64), _u(20), _u(20)
    S, r = _conv(x, a, y, b, 0.1)
    G = oracle.grad_x(x, a, y, b, r["f"], r["g"], r["p"], 0.01)
    np.testing.assert_allclose(G.sum(0), (a[:, None] * x).sum(0) - (b[:, None] * y).sum(0),
                               rtol=1e-9, atol=1e-12)
    # One Dirac each: grad = (x - y) when balanced, (x - y) exp(-C/(eps + 2 rho)) otherwise.
    x1, y1 = np.array([[0.2, 0.1]]), np.array([[-0.3, 0.5]])
    C = 0.5 * ((x1 - y1) ** 2).sum()
    S, r = _conv(x1, [1.0], y1, [1.0], 0.3)
    np.testing.assert_allclose(oracle.grad_x(x1, [1.0], y1, [1.0], r["f"], r["g"], r["p"], 0.09),
                               x1 - y1, rtol=1e-11)
    S, r = _conv(x1, [1.0], y1, [1.0], 0.3, reach=0.5)
    eps, rho = 0.09, 0.25
    np.testing.assert_allclose(oracle.grad_x(x1, [1.0], y1, [1.0], r["f"], r["g"], r["p"], eps),
                               (x1 - y1) * math.exp(-C / (eps + 2 * rho)), rtol=1e-10)


@pytest.mark.parametrize("reach", [None, 0.6])
def test_gradient_y_finite_differences(reach):
    rng = np.random.default_rng(28)
    x, y = rng.uniform(size=(5, 2)), rng.uniform(size=(4, 2))
    a, b = _w(5, 29), _u(4)
    blur = 0.25
    S, r = _conv(x, a, y, b, blur, reach, tol=1e-15)
    G = oracle.grad_y(x, a, y, b, r["f"], r["g"], r["q"], blur ** 2)
    h = 1e-5
    fd = np.zeros_like(y)
    for j in range(4):
        for k in range(2):
            yp, ym = y.copy(), y.copy()
            yp[j, k] += h
            ym[j, k] -= h
            fd[j, k] = (_conv(x, a, yp, b, blur, reach, tol=1e-15)[0]
                        - _conv(x, a, ym, b, blur, reach, tol=1e-15)[0]) / (2 * h)
    np.testing.assert_allclose(G, fd, rtol=1e-5, atol=1e-9)


def test_weight_gradient_finite_differences_unbalanced():
    # Each weight moved alone (unbalanced: the masses need not agree).
    rng = np.random.default_rng(31)
    x, y = rng.uniform(size=(5, 2)), rng.uniform(size=(6, 2))
    a, b = _w(5, 32), _w(6, 33, total=1.3)
    blur, reach = 0.2, 0.6
    S, r = _conv(x, a, y, b, blur, reach, tol=1e-15)
    Ga = oracle.grad_weights(r["f"], r["p"], blur, reach)
    Gb = oracle.grad_weights(r["g"], r["q"], blur, reach)
    h = 1e-6
    for i in range(5):
        ap, am = a.copy(), a.copy()
        ap[i] += h
        am[i] -= h
        fd = (_conv(x, ap, y, b, blur, reach, tol=1e-15)[0]
              - _conv(x, am, y, b, blur, reach, tol=1e-15)[0]) / (2 * h)
        assert fd == pytest.approx(Ga[i], rel=1e-6, abs=1e-10)
    for j in range(6):
        bp, bm = b.copy(), b.copy()
        bp[j] += h
        bm[j] -= h
        fd = (_conv(x, a, y, bp, blur, reach, tol=1e-15)[0]
              - _conv(x, a, y, bm, blur, reach, tol=1e-15)[0]) / (2 * h)
        assert fd == pytest.approx(Gb[j], rel=1e-6, abs=1e-10)


def test_weight_gradient_balanced_mass_preserving():
    # Balanced: only mass-preserving moves stay feasible, and f, g carry a free constant;
    # moving mass h from point k to point i changes S by h (G_i - G_k), free of that constant.
    rng = np.random.default_rng(34)
    x, y = rng.uniform(size=(5, 2)), rng.uniform(size=(6, 2))
    a, b = _w(5, 35), _w(6, 36)
    blur = 0.2
    S, r = _conv(x, a, y, b, blur, None, tol=1e-15)
    Ga = oracle.grad_weights(r["f"], r["p"], blur)
    Gb = oracle.grad_weights(r["g"], r["q"], blur)
    h = 1e-6
    for i, k in ((0, 1), (2, 4), (3, 0)):
        ap, am = a.copy(), a.copy()
        ap[i] += h
        ap[k] -= h
        am[i] -= h
        am[k] += h
        fd = (_conv(x, ap, y, b, blur, None, tol=1e-15)[0]
              - _conv(x, am, y, b, blur, None, tol=1e-15)[0]) / (2 * h)
        assert fd == pytest.approx(Ga[i] - Ga[k], rel=1e-6, abs=1e-10)
    for j, k in ((0, 5), (3, 2)):
        bp, bm = b.copy(), b.copy()
        bp[j] += h
        bp[k] -= h
        bm[j] -= h
        bm[k] += h
        fd = (_conv(x, a, y, bp, blur, None, tol=1e-15)[0]
              - _conv(x, a, y, bm, blur, None, tol=1e-15)[0]) / (2 * h)
        assert fd == pytest.approx(Gb[j] - Gb[k], rel=1e-6, abs=1e-10)


@pytest.mark.parametrize("a,b", [(1.0, 1.0), (0.6, 1.7), (2.0, 0.3)])
def test_weight_gradient_dirac_closed_form(a, b):
    # One Dirac each: dS/da and dS/db by central differences of the closed-form S of
    # eq. (5) (minimiser of eq. (2) for one Dirac each, mass term included).
    x, y = np.array([[0.3, -0.2]]), np.array([[-0.1, 0.4]])
    C = 0.5 * ((x - y) ** 2).sum()
    blur, reach = 0.3, 0.5
    eps, rho = blur ** 2, reach ** 2

    def S_closed(a, b):
        return (_dirac_ot(a, b, C, eps, rho) - 0.5 * _dirac_ot(a, a, 0.0, eps, rho)
                - 0.5 * _dirac_ot(b, b, 0.0, eps, rho) + 0.5 * eps * (a - b) ** 2)

    h = 1e-5
    da = (S_closed(a + h, b) - S_closed(a - h, b)) / (2 * h)
    db = (S_closed(a, b + h) - S_closed(a, b - h)) / (2 * h)
    S, r = _conv(x, [a], y, [b], blur, reach)
    assert oracle.grad_weights(r["f"], r["p"], blur, reach)[0] == pytest.approx(da, rel=1e-8)
    assert oracle.grad_weights(r["g"], r["q"], blur, reach)[0] == pytest.approx(db, rel=1e-8)
    if a == b == 1.0:
        # (eps + rho)(1 - e^{-C/(eps + 2 rho)}), differentiating the closed form by hand
        assert da == pytest.approx((eps + rho) * (1 - math.exp(-C / (eps + 2 * rho))), rel=1e-8)


# ------------------------------------------------------------- plan apply ----

def test_plan_apply_marginal_and_labels():
    x, _, y, _ = synth.blob_pair(30, seed=27)
    a, b = _u(30), _u(30)
    blur = 0.1
    S, r = _conv(x, a, y, b, blur, tol=1e-14)
    ones = np.ones((30, 1))
    out = oracle.plan_apply(x, a, y, b, r["f"], r["g"], blur ** 2, ones)
    np.testing.assert_allclose(out[:, 0], a, rtol=1e-9)
    # eq. (7): soft labels of one-hot vectors sum to one (balanced) and lie in the simplex
    labels = np.eye(4)[np.arange(30) % 4]
    lab = oracle.plan_apply(x, a, y, b, r["f"], r["g"], blur ** 2, labels, divide_by_a=True)
    assert np.all(lab >= 0)
    np.testing.assert_allclose(lab.sum(1), 1.0, rtol=1e-9)


@pytest.mark.parametrize("reach", [None, 0.5])
def test_self_and_cross_loops_are_independent(reach):
    # In the Algorithm every update reads the previous values of one loop only:
    # p~ from p (alpha<->alpha), q~ from q (beta<->beta), f~ from g and g~ from f.
    # With the same scale list, the p of the pair (alpha, beta) is therefore the p of
    # the pair (alpha, alpha), whatever beta is; the barycenter shares it over maps.
    rng = np.random.default_rng(41)
    x = rng.uniform(0, 1, (30, 2))
    y = rng.uniform(0, 1, (25, 2)) + 0.3
    y2 = rng.normal(0.5, 0.2, (40, 2))
    a, b, b2 = _w(30, 1), _w(25, 2), _w(40, 3)
    kw = dict(blur=0.05, reach=reach, scaling=0.7, diam=3.0, extra_iters=4)
    _, r1 = oracle.sinkhorn_divergence(x, a, y, b, **kw)
    _, r2 = oracle.sinkhorn_divergence(x, a, y2, b2, **kw)
    _, r3 = oracle.sinkhorn_divergence(x, a, x, a, **kw)
    np.testing.assert_array_equal(r1["p"], r2["p"])
    np.testing.assert_array_equal(r1["p"], r3["p"])
    _, r4 = oracle.sinkhorn_divergence(y, b, y, b, **kw)
    np.testing.assert_array_equal(r1["q"], r4["q"])


# ---------------------------------------------------------- label transfer ---

def test_flip_fibers_reverses_points():
    x = np.arange(18, dtype=np.float64).reshape(2, 9)  # 2 fibres of 3 points in 3-D
    fx = oracle.flip_fibers(x, 3)
    np.testing.assert_array_equal(fx[0], [6, 7, 8, 3, 4, 5, 0, 1, 2])
    np.testing.assert_array_equal(oracle.flip_fibers(fx, 3), x)


def _label_case(n_out=0, frac=0.5, points=4):
    y = synth.fibers(60, 3, spine_seed=40, seed=41, points=points)
    ly = synth.fiber_labels(60, 3)
    x = synth.random_orientations(synth.fibers(45, 3, spine_seed=40, seed=42, points=points),
                                  points, seed=43, frac=frac)
    lx = synth.fiber_labels(45, 3)
    if n_out:
        x = np.concatenate([x, synth.outlier_fibers(n_out, seed=44, points=points)])
        lx = np.concatenate([lx, -np.ones(n_out, np.int32)])
    return x, _u(len(x)), y, _u(60), ly, lx


@pytest.mark.parametrize("flips", [0, 4])
def test_label_transfer_score_is_transported_mass(flips):
    # At the fixed point the row marginal of the plan is alpha_i e^{-f_i/rho} (optimality of
    # eq. (3) in f_i), so score_i = sum_l Lab_il = e^{-f_i/rho}, summed over both versions.
    x, a, y, b, ly, lx = _label_case(n_out=5)
    reach = 20.0
    lab, score, r = oracle.label_transfer(x, a, y, b, ly, 3, 1.0, reach, flip_points=flips,
                                          scaling=0.7, tol=1e-13, max_iters=50000)
    assert r["converged"]
    n = len(x)
    e = np.exp(-r["f"] / reach ** 2)
    np.testing.assert_allclose(score, e[:n] + e[n:] if flips else e, rtol=1e-8)
    np.testing.assert_allclose(score, lab.sum(1), rtol=1e-12)


def test_label_transfer_balanced_rows_on_simplex():
    x, a, y, b, ly, lx = _label_case(frac=0.0)
    lab, score, r = oracle.label_transfer(x, a, y, b, ly, 3, 1.0, None, scaling=0.7, tol=1e-13,
                                          max_iters=50000)
    assert r["converged"] and np.all(lab >= 0)
    np.testing.assert_allclose(score, 1.0, rtol=1e-9)
    assert np.all(np.argmax(lab, 1) == lx)


def test_label_transfer_flips_and_outliers():
    # Half the subject fibres are stored reversed, five are far from every bundle.  With the
    # flips every inlier recovers its bundle and keeps about its mass; without them the
    # reversed fibres (far from their bundle in that orientation) keep much less mass than
    # any forward fibre; the aberrant fibres lose all of it either way.
    x, a, y, b, ly, lx = _label_case(n_out=5)
    ids = np.arange(180, dtype=np.float32).reshape(45, 4)  # which fibres were stored reversed
    rev = synth.random_orientations(ids, 4, seed=43)[:, 0] != ids[:, 0]
    inl = lx >= 0
    lab, score, _ = oracle.label_transfer(x, a, y, b, ly, 3, 1.0, 20.0, flip_points=4,
                                          scaling=0.7, tol=1e-10, max_iters=50000)
    assert np.all(np.argmax(lab[inl], 1) == lx[inl])
    assert np.all((score[inl] > 0.9) & (score[inl] < 1.5)) and np.all(score[~inl] < 1e-6)
    lab0, score0, _ = oracle.label_transfer(x, a, y, b, ly, 3, 1.0, 20.0, scaling=0.7,
                                            tol=1e-10, max_iters=50000)
    assert rev.sum() > 10
    assert score0[:45][rev].max() < 0.6 < 1.2 < score0[:45][~rev].min()
    assert np.all(score0[~inl] < 1e-6)


# ------------------------------------------------------ general exponent p ---

@pytest.mark.parametrize("pexp", [1.0, 1.5])
def test_cost_p_softmin_single_column(pexp):
    # m = 1: out_i = lam (C(x_i, y) - h - eps log w) with C = |x - y|^p / p
    rng = np.random.default_rng(80)
    x, y = rng.uniform(size=(7, 3)), rng.uniform(size=(1, 3))
    eps, lam, w, h = 0.04, 0.8, 0.3, 0.25
    C = np.sqrt(((x - y) ** 2).sum(1)) ** pexp / pexp
    out = oracle.softmin(x, y, [w], [h], eps, lam, p=pexp)
    np.testing.assert_allclose(out, lam * (C - h - eps * math.log(w)), rtol=1e-13)


@pytest.mark.parametrize("pexp", [1.0, 1.5])
def test_cost_p_dirac_balanced_and_unbalanced(pexp):
    # One Dirac each: balanced S = C for any eps; unbalanced from the closed-form minimiser of
    # eq. (2), whose derivation only uses the scalars C, eps = blur^p and rho = reach^p.
    x, y = np.array([[0.3, -0.2]]), np.array([[-0.1, 0.4]])
    C = np.sqrt(((x - y) ** 2).sum()) ** pexp / pexp
    S, r = oracle.sinkhorn_divergence(x, [1.0], y, [1.0], 0.3, scaling=0.5, tol=1e-14,
                                      max_iters=20000, p=pexp)
    assert S == pytest.approx(C, rel=1e-12)
    blur, reach = 0.3, 0.7
    eps, rho = blur ** pexp, reach ** pexp
    for a, b in ((1.0, 1.0), (0.6, 1.7)):
        expect = (_dirac_ot(a, b, C, eps, rho) - 0.5 * _dirac_ot(a, a, 0.0, eps, rho)
                  - 0.5 * _dirac_ot(b, b, 0.0, eps, rho) + 0.5 * eps * (a - b) ** 2)
        S, r = oracle.sinkhorn_divergence(x, [a], y, [b], blur, reach, scaling=0.5, tol=1e-14,
                                          max_iters=20000, p=pexp)
        assert r["converged"]
        assert S == pytest.approx(expect, rel=1e-10)


@pytest.mark.parametrize("pexp", [1.0, 1.5])
def test_cost_p_sorted_matching_1d(pexp):
    # Uniform 1-D measures: OT_0 is the sorted matching for any convex cost (p >= 1), and
    # |S_eps - OT_0| <= eps log n (entropic bounds of the three OT terms).
    rng = np.random.default_rng(81)
    n = 6
    x, y = rng.uniform(size=(n, 1)), rng.uniform(size=(n, 1)) + 0.3
    ot0 = np.mean(np.abs(np.sort(x[:, 0]) - np.sort(y[:, 0])) ** pexp / pexp)
    blur = 0.01 ** (1.0 / pexp)  # eps = 0.01
    S, r = oracle.sinkhorn_divergence(x, _u(n), y, _u(n), blur, scaling=0.7, tol=1e-10,
                                      max_iters=200000, p=pexp)
    assert r["converged"]
    assert abs(S - ot0) <= blur ** pexp * math.log(n)


@pytest.mark.parametrize("reach", [None, 0.5])
def test_cost_p_strong_duality(reach):
    # At the fixed point of the loop for p = 1, the primal eq. (2) at the plan of eq. (4)
    # equals the dual eq. (3) (strong duality), for the cross and both self problems.
    rng = np.random.default_rng(82)
    x, y = rng.uniform(size=(7, 2)), rng.uniform(size=(8, 2))
    a, b = _w(7, 83), _w(8, 84)
    blur = 0.15
    S, r = oracle.sinkhorn_divergence(x, a, y, b, blur, reach, scaling=0.6, tol=1e-14,
                                      max_iters=50000, p=1.0)
    assert r["converged"]
    eps = blur
    for (u, wu, v, wv, fu, fv) in ((x, a, y, b, r["f"], r["g"]), (x, a, x, a, r["p"], r["p"]),
                                   (y, b, y, b, r["q"], r["q"])):
        prim = oracle.ot_primal(u, wu, v, wv, fu, fv, eps, reach, p=1.0)
        dual = oracle.ot_dual(u, wu, v, wv, fu, fv, eps, reach, p=1.0)
        assert prim == pytest.approx(dual, rel=1e-9, abs=1e-12)
    # eq. (6) equals eq. (5) through the duals
    S5 = oracle.divergence_eq5(x, a, y, b, r["f"], r["g"], r["p"], r["q"], blur, reach, pexp=1.0)
    assert S == pytest.approx(S5, rel=1e-9, abs=1e-12)


def test_label_transfer_flip_copies_carry_the_fibre_weight():
    # A palindromic fibre equals its flip, so the augmented subject holds every point twice
    # at weight a_i: the same measure as the points once at 2 a_i.  Each copy's label is
    # normalised by its own weight a_i, so Lab with flips = 2 Lab of the doubled subject.
    P = 4
    x0 = synth.fibers(30, 3, spine_seed=40, seed=45, points=P).astype(np.float64)
    x = 0.5 * (x0 + oracle.flip_fibers(x0, P))  # palindromic
    np.testing.assert_array_equal(oracle.flip_fibers(x, P), x)
    y = synth.fibers(40, 3, spine_seed=40, seed=46, points=P)
    ly = synth.fiber_labels(40, 3)
    a, b = _u(30), _u(40)
    kw = dict(blur=1.0, reach=20.0, scaling=0.7, tol=1e-13, max_iters=100000)
    lab_f, score_f, r1 = oracle.label_transfer(x, a, y, b, ly, 3, flip_points=P, **kw)
    lab_2, score_2, r2 = oracle.label_transfer(x, 2 * a, y, b, ly, 3, **kw)
    assert r1["converged"] and r2["converged"]
    np.testing.assert_allclose(lab_f, 2 * lab_2, rtol=1e-8, atol=1e-12)
    np.testing.assert_allclose(score_f, 2 * score_2, rtol=1e-8)


# ------------------------------------------------ gradients, cost exponent p --

def _conv_p(x, a, y, b, blur, reach, cost_p, tol=1e-14):
    S, r = oracle.sinkhorn_divergence(x, a, y, b, blur, reach, scaling=0.5, tol=tol,
                                      max_iters=50000, check_every=1, p=cost_p)
    assert r["converged"], r["marginal_err"]
    return S, r


@pytest.mark.parametrize("cost_p,reach", [(1.5, None), (1.5, 0.7), (1.0, None), (1.0, 0.7),
                                          (1.25, 0.9)])
def test_gradient_p_finite_differences(cost_p, reach):
    # grad_x S for |x - y|^p / p (eps = blur^p) against central differences of the
    # oracle's converged S; the self term's zero-distance pairs do not move with x
    rng = np.random.default_rng(61)
    x, y = rng.uniform(size=(5, 2)), rng.uniform(size=(6, 2))
    a, b = _u(5), _w(6, 62)
    blur = 0.3
    S, r = _conv_p(x, a, y, b, blur, reach, cost_p)
    G = oracle.grad_x_p(x, a, y, b, r["f"], r["g"], r["p"], blur, cost_p)
    h = 1e-5
    fd = np.zeros_like(x)
    for i in range(5):
        for k in range(2):
            xp, xm = x.copy(), x.copy()
            xp[i, k] += h
            xm[i, k] -= h
            fd[i, k] = (_conv_p(xp, a, y, b, blur, reach, cost_p)[0]
                        - _conv_p(xm, a, y, b, blur, reach, cost_p)[0]) / (2 * h)
    np.testing.assert_allclose(G, fd, rtol=2e-5, atol=1e-9)


@pytest.mark.parametrize("cost_p", [1.5, 1.0])
def test_weight_gradient_p_finite_differences(cost_p):
    rng = np.random.default_rng(63)
    x, y = rng.uniform(size=(4, 2)), rng.uniform(size=(5, 2))
    a, b = _w(4, 64), _w(5, 65, total=1.2)
    blur, reach = 0.3, 0.8
    S, r = _conv_p(x, a, y, b, blur, reach, cost_p)
    Ga = oracle.grad_weights(r["f"], r["p"], blur, reach, cost_p=cost_p)
    h = 1e-6
    for i in range(4):
        ap, am = a.copy(), a.copy()
        ap[i] += h
        am[i] -= h
        fd = (_conv_p(x, ap, y, b, blur, reach, cost_p)[0]
              - _conv_p(x, am, y, b, blur, reach, cost_p)[0]) / (2 * h)
        assert fd == pytest.approx(Ga[i], rel=1e-6, abs=1e-10)


def test_gradient_p_reduces_to_p2_and_dirac():
    # p = 2: the same numbers as the p = 2 gradient (a separate implementation, in C)
    rng = np.random.default_rng(66)
    x, y = rng.uniform(size=(6, 3)), rng.uniform(size=(7, 3))
    a, b = _u(6), _w(7, 67)
    S, r = _conv(x, a, y, b, 0.25, 0.9)
    np.testing.assert_allclose(oracle.grad_x_p(x, a, y, b, r["f"], r["g"], r["p"], 0.25, 2.0),
                               oracle.grad_x(x, a, y, b, r["f"], r["g"], r["p"], 0.0625),
                               rtol=1e-12, atol=1e-15)
    # one balanced Dirac each: the plan moves the unit mass, grad = |x - y|^{p-2} (x - y)
    x1, y1 = np.array([[0.2, 0.1]]), np.array([[-0.3, 0.5]])
    for P in (1.0, 1.5):
        S, r = _conv_p(x1, [1.0], y1, [1.0], 0.3, None, P)
        D = float(np.linalg.norm(x1 - y1))
        np.testing.assert_allclose(oracle.grad_x_p(x1, [1.0], y1, [1.0], r["f"], r["g"], r["p"],
                                                   0.3, P), D ** (P - 2.0) * (x1 - y1),
                                   rtol=1e-10)
