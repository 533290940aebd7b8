"""GPU parity of the solve for the cost |x - y|^p / p with p != 2 (eps = blur^p,
rho = reach^p) against the FP64 oracle: same schedule, same inputs, S to 1e-5
relative and the potentials within an FP32-propagation tolerance, as for p = 2."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import cuda, host, note

pytestmark = pytest.mark.gpu

S_RTOL_FP32 = 1e-5


def _compare(x, a, y, b, blur, reach, pexp, scaling=0.5, extra=3):
    import paper_2107_02010_amd as skh
    note(f"p-cost n={len(x)} m={len(y)} d={x.shape[1]} p={pexp} blur={blur} reach={reach}")
    S, pot, st = skh.sinkhorn_divergence(cuda(x), cuda(a), cuda(y), cuda(b), blur=blur,
                                         reach=reach, scaling=scaling, extra_iters=extra,
                                         potentials=True, p=pexp)
    pot = {k: host(v) for k, v in pot.items()}
    Sr, r = oracle.sinkhorn_divergence(x, a, y, b, blur, reach, scaling=scaling,
                                       extra_iters=extra, p=pexp)
    assert st["iters"] == r["iters"] and st["n_scales"] == r["n_scales"]
    assert st["eps"] == pytest.approx(blur ** pexp, rel=1e-12)
    assert S == pytest.approx(Sr, rel=S_RTOL_FP32), (S, Sr)
    tol = 1e-4 * max(blur ** pexp, np.abs(r["f"]).max())
    for k in ("f", "g", "p", "q"):
        dg = pot[k] - r[k]
        dg -= dg.mean() if reach is None else 0.0
        assert np.max(np.abs(dg)) <= tol, (k, np.max(np.abs(dg)), tol)
    return S, Sr


@pytest.mark.parametrize("pexp", [1.0, 1.5])
@pytest.mark.parametrize("reach", [None, 0.3])
def test_blobs_match_oracle(pexp, reach):
    x, a, y, b = synth.blob_pair(700, seed=90)
    y, b = y[:513], synth.random_weights(513, 91)
    if reach is None:
        a = (a / a.astype(np.float64).sum()).astype(np.float32)
        b = (b / b.astype(np.float64).sum()).astype(np.float32)
    _compare(x, a, y, b, 0.05, reach, pexp)


@pytest.mark.parametrize("n,m,d", [(1, 1, 3), (129, 300, 7), (257, 130, 12), (200, 230, 60)])
def test_edge_sizes_and_widths(n, m, d):
    # ragged tiles, a single point, and every packed width (4, 8, 16, 64)
    x = synth.random_cloud(n, d, seed=92, scale=0.3)
    y = synth.random_cloud(m, d, seed=93, scale=0.3) + np.float32(0.1)
    a, b = synth.random_weights(n, 94), synth.random_weights(m, 95, total=1.2)
    _compare(x, a, y, b, 0.1, 0.5, 1.0)


def test_p_two_is_the_standard_path():
    # p = 2 given explicitly runs the contraction kernels: bitwise the default call
    import paper_2107_02010_amd as skh
    x, a, y, b = synth.blob_pair(300, seed=96)
    note("p = 2 explicit")
    S1 = skh.sinkhorn_divergence(cuda(x), cuda(a), cuda(y), cuda(b), blur=0.05, p=2.0)
    S2 = skh.sinkhorn_divergence(cuda(x), cuda(a), cuda(y), cuda(b), blur=0.05)
    assert S1 == S2


def test_rejects_unsupported_combinations():
    import paper_2107_02010_amd as skh
    x, a, y, b = synth.blob_pair(100, seed=97)
    note("p-cost argument checks")
    for kw in (dict(p=0.5), dict(p=2.5), dict(p=1.0, multiscale=True),
               dict(p=1.0, precision="bf16x3")):
        with pytest.raises(skh.SkhError):
            skh.sinkhorn_divergence(cuda(x), cuda(a), cuda(y), cuda(b), blur=0.05, **kw)


def _converged_p(x, a, y, b, blur, reach, pexp):
    Sr, r = oracle.sinkhorn_divergence(x, a, y, b, blur, reach, scaling=0.5, tol=1e-9,
                                       max_iters=5000, check_every=5, p=pexp)
    return {k: r[k].astype(np.float32) for k in ("f", "g", "p", "q")}


@pytest.mark.parametrize("pexp,reach", [(1.0, None), (1.0, 0.4), (1.5, None), (1.5, 0.4),
                                        (1.25, 0.4)])
@pytest.mark.parametrize("n,m,d", [(400, 300, 3), (129, 257, 7), (200, 230, 60), (1, 90, 3)])
def test_gradients_match_oracle(pexp, reach, n, m, d):
    # dS/da, dS/db at eps = blur^p, rho = reach^p; dS/dx and dS/dy with the pair weights
    # |x_i - y_j|^{p-2}, on the same FP32 inputs and potentials as the oracle
    import paper_2107_02010_amd as skh
    x = synth.random_cloud(n, d, seed=100 + d, scale=0.3)
    y = synth.random_cloud(m, d, seed=101 + d, scale=0.3) + np.float32(0.05)
    a, b = synth.random_weights(n, 102), synth.random_weights(m, 103)
    if reach is None:
        a = (a / a.astype(np.float64).sum()).astype(np.float32)
        b = (b / b.astype(np.float64).sum()).astype(np.float32)
    blur = 0.1
    pot = _converged_p(x, a, y, b, blur, reach, pexp)
    note(f"p-cost gradients n={n} m={m} d={d} p={pexp} reach={reach}")
    G = skh.gradients(cuda(x), cuda(a), cuda(y), cuda(b), {k: cuda(v) for k, v in pot.items()},
                      blur, reach, p=pexp)
    G = {k: host(v) for k, v in G.items()}
    ga = oracle.grad_weights(pot["f"], pot["p"], blur, reach, cost_p=pexp)
    gb = oracle.grad_weights(pot["g"], pot["q"], blur, reach, cost_p=pexp)
    np.testing.assert_allclose(G["a"], ga, rtol=2 ** -23, atol=1e-37)
    np.testing.assert_allclose(G["b"], gb, rtol=2 ** -23, atol=1e-37)
    rx = oracle.grad_x_p(x, a, y, b, pot["f"], pot["g"], pot["p"], blur, pexp)
    ry = oracle.grad_x_p(y, b, x, a, pot["g"], pot["f"], pot["q"], blur, pexp)
    # |grad_x C| = |x - y|^{p-1}: the plan sums carry terms up to a_i (span^{p-1}), and
    # FP32 rounding of the differences, the weights and the exponentials at ~1e-6 each
    span = (np.abs(x).max() + np.abs(y).max()) ** (pexp - 1.0) + 1.0
    assert np.all(np.abs(G["x"] - rx) <= 1e-4 * (a[:, None] * span) + 1e-4 * np.abs(rx))
    assert np.all(np.abs(G["y"] - ry) <= 1e-4 * (b[:, None] * span) + 1e-4 * np.abs(ry))


def test_loss_backward_uses_the_cost_exponent():
    # the autograd Function passes the solve's exponent to the gradient kernels:
    # backward equals gradients(..., p) on the same potentials
    import torch

    import paper_2107_02010_amd as skh
    x, a, y, b = synth.blob_pair(300, seed=104)
    a = (a / a.astype(np.float64).sum()).astype(np.float32)
    b = (b / b.astype(np.float64).sum()).astype(np.float32)
    note("p-cost loss backward")
    X = cuda(x).requires_grad_(True)
    kw = dict(blur=0.05, scaling=0.5, extra_iters=5, p=1.5)
    L = skh.sinkhorn_loss(X, cuda(a), cuda(y), cuda(b), **kw)
    L.backward()
    S, pot, _ = skh.sinkhorn_divergence(cuda(x), cuda(a), cuda(y), cuda(b), potentials=True, **kw)
    G = skh.gradients(cuda(x), cuda(a), cuda(y), cuda(b), pot, 0.05, None, wrt=("x",), p=1.5)
    assert float(L) == pytest.approx(S, rel=0, abs=0)
    assert torch.equal(X.grad, G["x"])
    G2 = skh.gradients(cuda(x), cuda(a), cuda(y), cuda(b), pot, 0.05, None, wrt=("x",))
    assert not torch.allclose(G2["x"], G["x"])  # the p = 2 formula is another gradient


def test_gradient_exponent_checks():
    import paper_2107_02010_amd as skh
    x, a, y, b = synth.blob_pair(50, seed=105)
    z = {k: cuda(np.zeros(50, np.float32)) for k in "fgpq"}
    note("p-cost gradient argument checks")
    for pexp in (0.5, 2.5, float("nan")):
        with pytest.raises(skh.SkhError):
            skh.gradients(cuda(x), cuda(a), cuda(y), cuda(b), z, 0.1, None, p=pexp)
