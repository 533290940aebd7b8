"""GPU barycenter gradient descent (Section 3) against the oracle's trajectory on
a downscaled instance of the density-map generator, plus the full-size
workload's shape through one step (ragged map sizes)."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import cuda, host, note

pytestmark = pytest.mark.gpu


def test_barycenter_steps_match_oracle():
    import torch

    from paper_2107_02010_amd.barycenter import wasserstein_barycenter
    maps = synth.density_maps(3, seed=1, grid=24, n_tubes=3, nonzero=(500, 900),
                              sigma=(1.0, 2.0), jitter=1.5)
    x0, a = synth.barycenter_support(maps, 400, seed=2)
    kw = dict(blur=1.0, reach=None, scaling=0.7, lr=1.0)
    note("barycenter 3 maps 24^3, 400 support, 2 steps")
    xg, hg = wasserstein_barycenter(cuda(x0), cuda(a), [(cuda(c), cuda(w)) for c, w in maps],
                                    steps=2, **kw)
    xr, hr = oracle.barycenter_steps(x0, a, maps, 2, **kw)
    assert hg[0] == pytest.approx(hr[0], rel=1e-4)
    assert hg[1] == pytest.approx(hr[1], rel=1e-3)
    assert hg[1] < hg[0]  # the loss decreases
    np.testing.assert_allclose(host(xg), xr, atol=2e-3 * 24)
    assert torch.isfinite(xg).all()


def test_barycenter_full_shape_one_step():
    from paper_2107_02010_amd.barycenter import barycenter_step
    maps = synth.density_maps(2, seed=3)
    x0, a = synth.barycenter_support(maps, 200_000, seed=4)
    note("barycenter 128^3 maps, 200k support, one step")
    ym = [(cuda(c), cuda(w)) for c, w in maps]
    x1, S, pots = barycenter_step(cuda(x0), cuda(a), ym, blur=1.0, scaling=0.9)
    g = host(x1)
    assert np.all(np.isfinite(g)) and S > 0
    # balanced, unit masses: the mean of the support moves to the mean of the maps' means
    # (sum_i grad_i = xbar - mean_k ybar_k, step lr/a_i with a_i = 1/n)
    ybar = np.mean([(w[:, None].astype(np.float64) * c).sum(0) for c, w in maps], axis=0)
    print("support mean after one step", g.astype(np.float64).mean(0), "target", ybar)
    np.testing.assert_allclose(g.astype(np.float64).mean(0), ybar, atol=0.5)
