"""Pins of the FP64 warm-start network reference: its hand-derived backward pass
against central finite differences, permutation equivariance of the set encoder,
exact special cases, and the Adam update against its closed form on a quadratic."""
import numpy as np
import pytest

from oracle import network as net


def _case(T=11, na=5, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((T, net.IN))
    w = rng.uniform(0.1, 1.0, T)
    target = rng.standard_normal((T, net.OUT))
    theta = net.init_params(seed + 1) * 0.7
    return theta, X, w, na, target


def test_param_count_and_packing():
    assert net.n_params() == 256 * 64 + 256 + 2 * (256 * 256 + 256) + 256 * 768 + 256 + 2 * 256 + 2
    theta = net.init_params(3)
    assert np.array_equal(net.pack(net.unpack(theta)), theta)


def test_backward_matches_finite_differences():
    theta, X, w, na, target = _case()
    loss, g = net.loss_and_grad(theta, X, w, na, target)
    rng = np.random.default_rng(5)
    idx = rng.choice(net.n_params(), size=60, replace=False)
    # include every bias block and the last layer
    idx = np.concatenate([idx, [16384, 16384 + 255, net.n_params() - 1, net.n_params() - 3]])
    h = 1e-6
    for k in idx:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (net.loss_and_grad(tp, X, w, na, target)[0] - net.loss_and_grad(tm, X, w, na, target)[0]) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-9), k


def test_permutation_equivariance():
    theta, X, w, na, target = _case(T=9, na=4)
    y = net.forward(theta, X, w, na)
    pa = np.random.default_rng(1).permutation(4)
    pb = 4 + np.random.default_rng(2).permutation(5)
    perm = np.concatenate([pa, pb])
    y2 = net.forward(theta, X[perm], w[perm], na)
    np.testing.assert_allclose(y2, y[perm], rtol=1e-12, atol=1e-12)
    # swapping the roles of the clouds changes the pooled context order only
    assert not np.allclose(net.forward(theta, X, w, 5), y)


def test_zero_weights_give_biases():
    theta, X, w, na, _ = _case()
    P = net.unpack(theta)
    for k in ("W1", "W2", "W3", "W4", "W5"):
        P[k] = np.zeros_like(P[k])
    P["b5"] = np.array([0.25, -1.5])
    y = net.forward(net.pack(P), X, w, na)
    np.testing.assert_allclose(y, np.tile([0.25, -1.5], (X.shape[0], 1)))


def test_adam_closed_form_first_step():
    # first step: m = (1-b1) g, v = (1-b2) g^2, bias-corrected ratio = sign(g) (up to eps)
    theta = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    t, m, v = net.adam_step(theta, g, np.zeros(3), np.zeros(3), 1, lr=0.1, eps=0.0)
    np.testing.assert_allclose(t, theta - 0.1 * np.sign(g), rtol=1e-12)
