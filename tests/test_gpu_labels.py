"""GPU parity of the label transfer (eq. (7), Section 3) with mirror-flip augmentation
and outlier scores, against the FP64 oracle run the same number of iterations."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import cuda, host, note

pytestmark = pytest.mark.gpu


def _case(n, m, bundles, n_out, points, seed):
    y = synth.fibers(m, bundles, spine_seed=seed, seed=seed + 1, points=points)
    ly = synth.fiber_labels(m, bundles)
    x = synth.random_orientations(synth.fibers(n, bundles, spine_seed=seed, seed=seed + 2,
                                               points=points), points, seed=seed + 3)
    lx = synth.fiber_labels(n, bundles)
    if n_out:
        x = np.concatenate([x, synth.outlier_fibers(n_out, seed=seed + 4, points=points)])
        lx = np.concatenate([lx, -np.ones(n_out, np.int32)])
    return x, synth.uniform_weights(len(x)), y, synth.uniform_weights(m), ly, lx


def _labels(ly):
    import torch
    return torch.as_tensor(ly, dtype=torch.int32).cuda()


@pytest.mark.parametrize("flips", [0, 4])
@pytest.mark.parametrize("n,m,bundles,n_out", [(300, 400, 3, 10), (97, 130, 5, 3)])
def test_label_transfer_matches_oracle(n, m, bundles, n_out, flips):
    import paper_2107_02010_amd as skh
    x, a, y, b, ly, lx = _case(n, m, bundles, n_out, 4, seed=50 + n)
    kw = dict(blur=1.0, reach=20.0, scaling=0.7, extra_iters=30)
    note(f"label transfer n={len(x)} m={m} L={bundles} flips={flips}")
    lab, score = skh.label_transfer(cuda(x), cuda(a), cuda(y), cuda(b), _labels(ly), bundles,
                                    flip_points=flips, tol=0.0, **kw)
    lab, score = host(lab), host(score)
    ref, rscore, r = oracle.label_transfer(x, a, y, b, ly, bundles, flip_points=flips, **kw)
    # Lab_i carries exp((f_i + g_j)/eps): each iteration of the FP32 loop leaves a few ulps
    # of rounding in f and g (at most 4 per iteration, carried through the averaging), so
    # row i is off by up to 4 k ulps of (|f_i| + max|g|) over eps after k iterations
    fi = np.abs(r["f"][:len(x)])
    if flips:
        fi = np.maximum(fi, np.abs(r["f"][len(x):]))
    rel = 4 * r["iters"] * 2.0 ** -24 * (fi + np.abs(r["g"]).max()) / kw["blur"] ** 2
    err = np.abs(lab - ref) / (rel[:, None] * rscore[:, None] + 1e-30)
    assert np.all(err <= 1.0), (rel.max(), err.max())
    assert np.all(np.abs(score - rscore) <= rel * rscore + 1e-30)
    np.testing.assert_allclose(score, lab.sum(1), rtol=1e-5, atol=1e-30)
    # the decided labels agree wherever the oracle's margin is clear (rows that carry mass:
    # an outlier's labels, ~1e-140, are below the FP32 range)
    top2 = np.sort(ref, 1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0] > 1e-2 * rscore) & (rscore > 1e-20)
    assert clear.sum() >= 0.9 * n
    assert np.array_equal(np.argmax(lab, 1)[clear], np.argmax(ref, 1)[clear])


def test_label_transfer_multiscale_fibres():
    # 20k-fibre atlas of 10 bundles, 60-D fibres; the subject's fibres stored in random
    # directions plus 1 % aberrant fibres; multiscale solve to the usual tolerance
    import paper_2107_02010_amd as skh
    x, a, y, b, ly, lx = _case(20000, 20000, 10, 200, 20, seed=60)
    note("label transfer multiscale 20k flips")
    lab, score, st = skh.label_transfer(cuda(x), cuda(a), cuda(y), cuda(b), _labels(ly), 10,
                                        flip_points=20, multiscale=True, tol=1e-4, stats=True)
    lab, score = host(lab), host(score)
    inl = lx >= 0
    assert st["iters"] > 0
    assert np.mean(np.argmax(lab[inl], 1) == lx[inl]) > 0.999
    assert np.all(score[~inl] < 1e-3)
    assert np.all(score[inl] > 0.5)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("theta", [20.0, 0.0])
def test_label_transfer_multiscale_plan_matches_dense(theta, precision):
    # The multiscale path applies the plan over the cluster blocks kept at the final
    # potentials (theta <= 0 keeps every block); the dense plan on the same potentials
    # (the solve is deterministic: same inputs, same vectors) differs by the dropped
    # blocks, whose entries are below e^{-theta} each, and by FP32 rounding.
    import torch

    import paper_2107_02010_amd as skh
    x, a, y, b, ly, lx = _case(2500, 3100, 5, 37, 4, seed=80)
    kw = dict(blur=1.0, reach=20.0, scaling=0.7, multiscale=True, trunc_theta=theta,
              n_clusters=24, tol=0.0, precision=precision)
    note(f"label transfer multiscale plan vs dense theta={theta} {precision}")
    lab, score = skh.label_transfer(cuda(x), cuda(a), cuda(y), cuda(b), _labels(ly), 5,
                                    flip_points=4, **kw)
    xa = np.ascontiguousarray(np.concatenate([x, oracle.flip_fibers(x, 4)]), np.float32)
    aa = np.ascontiguousarray(np.concatenate([a, a]), np.float32)
    _, pot, _ = skh.sinkhorn_divergence(cuda(xa), cuda(aa), cuda(y), cuda(b), potentials=True,
                                        **kw)
    V = torch.nn.functional.one_hot(_labels(ly).long(), 5).float()
    aug = host(skh.plan_apply(cuda(xa), cuda(aa), cuda(y), cuda(b), pot["f"], pot["g"], 1.0, V,
                              divide_by_a=True))
    n = len(x)
    ref = aug[:n] + aug[n:]
    rs = ref.sum(1)
    lab, score = host(lab), host(score)
    tol = 1e-4 * rs[:, None] + (1e-7 if theta > 0 else 1e-30)
    assert np.all(np.abs(lab - ref) <= tol), np.abs(lab - ref).max()
    np.testing.assert_allclose(score, rs, rtol=1e-4, atol=1e-7 if theta > 0 else 1e-30)


def test_label_transfer_rejects_bad_arguments():
    import torch

    import paper_2107_02010_amd as skh
    x, a, y, b, ly, lx = _case(50, 60, 3, 0, 4, seed=70)
    note("label transfer argument checks")
    bad = ly.copy()
    bad[7] = 3
    with pytest.raises(skh.SkhError):
        skh.label_transfer(cuda(x), cuda(a), cuda(y), cuda(b), _labels(bad), 3)
    with pytest.raises(skh.SkhError):  # 12 coordinates are not fibres of 5 points
        skh.label_transfer(cuda(x), cuda(a), cuda(y), cuda(b), _labels(ly), 3, flip_points=5)
    with pytest.raises(ValueError):
        skh.label_transfer(cuda(x), cuda(a), cuda(y), cuda(b),
                           torch.as_tensor(ly, dtype=torch.int64).cuda(), 3)
    lab, score = skh.label_transfer(cuda(x), cuda(a), cuda(y), cuda(b), _labels(ly), 3)
    assert torch.isfinite(lab).all() and torch.isfinite(score).all()


@pytest.mark.parametrize("n,m,L,flips", [(1, 50, 1, 0), (3, 40, 2, 4), (130, 70, 64, 4)])
def test_label_transfer_multiscale_edge_sizes(n, m, L, flips):
    # tiny subjects, more clusters requested than points, one label and the largest
    # label count: the block-sparse plan inside the multiscale solve against the dense
    # plan on the same potentials
    import torch

    import paper_2107_02010_amd as skh
    rng = np.random.default_rng(n + m + L)
    x = (5.0 * rng.standard_normal((n, 12))).astype(np.float32)
    y = (5.0 * rng.standard_normal((m, 12))).astype(np.float32)
    a, b = synth.uniform_weights(n), synth.uniform_weights(m)
    ly = rng.integers(0, L, m).astype(np.int32)
    kw = dict(blur=1.0, reach=20.0, scaling=0.7, multiscale=True, n_clusters=200, tol=0.0)
    note(f"label transfer multiscale edge n={n} m={m} L={L} flips={flips}")
    lab, score = skh.label_transfer(cuda(x), cuda(a), cuda(y), cuda(b), _labels(ly), L,
                                    flip_points=flips, **kw)
    if flips:
        xa = np.ascontiguousarray(np.concatenate([x, oracle.flip_fibers(x, flips)]), np.float32)
        aa = np.ascontiguousarray(np.concatenate([a, a]), np.float32)
    else:
        xa, aa = x, a
    _, pot, _ = skh.sinkhorn_divergence(cuda(xa), cuda(aa), cuda(y), cuda(b), potentials=True,
                                        **kw)
    V = torch.nn.functional.one_hot(_labels(ly).long(), L).float()
    aug = host(skh.plan_apply(cuda(xa), cuda(aa), cuda(y), cuda(b), pot["f"], pot["g"], 1.0, V,
                              divide_by_a=True))
    ref = aug[:n] + aug[n:] if flips else aug
    rs = ref.sum(1)
    lab, score = host(lab), host(score)
    assert lab.shape == (n, L) and score.shape == (n,)
    assert np.all(np.abs(lab - ref) <= 1e-4 * rs[:, None] + 1e-7)
    np.testing.assert_allclose(score, rs, rtol=1e-4, atol=1e-7)
