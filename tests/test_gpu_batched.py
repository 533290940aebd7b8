"""GPU parity of the batched multi-pair solve: K independent pairs in one launch per
iteration (block-diagonal softmins) against the FP64 oracle run pair by pair with the
same scale list, against single GPU solves, and with fixed self loops."""
import numpy as np
import pytest

import oracle
import synth
from gpu_common import cuda, host, note

pytestmark = pytest.mark.gpu

SIZES = [(1, 2), (37, 64), (129, 200), (300, 257), (513, 400)]


def _pairs(reach, seed=100):
    xs, as_, ys, bs = [], [], [], []
    for k, (n, m) in enumerate(SIZES):
        x = synth.blobs(n, seed + 2 * k, sigma=0.08)
        y = synth.blobs(m, seed + 2 * k + 1, sigma=0.08)
        if reach is None:
            a, b = synth.uniform_weights(n), synth.uniform_weights(m)
        else:
            a, b = synth.random_weights(n, seed + 50 + k), synth.random_weights(m, seed + 70 + k, 1.3)
        xs.append(x); as_.append(a); ys.append(y); bs.append(b)
    return xs, as_, ys, bs


def _diam(xs, ys):
    allp = np.concatenate(xs + ys).astype(np.float64)
    return float(np.sqrt(((allp.max(0) - allp.min(0)) ** 2).sum()))


@pytest.mark.parametrize("reach", [None, 0.3])
def test_batched_matches_oracle_and_single_solves(reach):
    import paper_2107_02010_amd as skh
    xs, as_, ys, bs = _pairs(reach)
    blur, scaling, extra = 0.05, 0.5, 3
    note(f"batched K={len(xs)} reach={reach}")
    S, pot, st = skh.sinkhorn_divergence_batched([cuda(v) for v in xs], [cuda(v) for v in as_],
                                                 [cuda(v) for v in ys], [cuda(v) for v in bs],
                                                 blur=blur, reach=reach, scaling=scaling,
                                                 extra_iters=extra, potentials=True)
    diam = st["diameter"]
    assert diam == pytest.approx(_diam(xs, ys), rel=1e-6)
    for k in range(len(xs)):
        Sr, r = oracle.sinkhorn_divergence(xs[k], as_[k], ys[k], bs[k], blur, reach,
                                           scaling=scaling, diam=diam, extra_iters=extra)
        assert st["iters"] == r["iters"]
        assert S[k] == pytest.approx(Sr, rel=1e-5, abs=1e-9), (k, S[k], Sr)
        tol = 1e-4 * max(blur ** 2, np.abs(r["f"]).max())
        for nm in ("f", "g", "p", "q"):
            dg = host(pot[nm][k]) - r[nm]
            dg -= dg.mean() if reach is None else 0.0
            assert np.max(np.abs(dg)) <= tol, (k, nm, np.max(np.abs(dg)), tol)
        S1 = skh.sinkhorn_divergence(cuda(xs[k]), cuda(as_[k]), cuda(ys[k]), cuda(bs[k]),
                                     blur=blur, reach=reach, scaling=scaling, diameter=diam,
                                     extra_iters=extra)
        assert S[k] == pytest.approx(S1, rel=1e-5, abs=1e-9)


def test_batched_fixed_self_loops_reproduce_the_full_batched_solve():
    # the Jacobi loops are independent: holding p, q at the full solve's values and
    # running only the cross loops gives the same f, g and S bit for bit
    import torch

    import paper_2107_02010_amd as skh
    xs, as_, ys, bs = _pairs(0.3, seed=120)
    args = ([cuda(v) for v in xs], [cuda(v) for v in as_], [cuda(v) for v in ys],
            [cuda(v) for v in bs])
    kw = dict(blur=0.05, reach=0.3, scaling=0.5, extra_iters=2)
    note("batched fixed self loops")
    S, pot, st = skh.sinkhorn_divergence_batched(*args, potentials=True, **kw)
    n, m = sum(len(v) for v in xs), sum(len(v) for v in ys)
    init = (torch.zeros(n, device="cuda"), torch.zeros(m, device="cuda"), torch.cat(pot["p"]),
            torch.cat(pot["q"]))
    S2, pot2, st2 = skh.sinkhorn_divergence_batched(*args, potentials=True, init=init,
                                                    fixed=skh.SKH_FIX_P | skh.SKH_FIX_Q, **kw)
    assert S2 == S
    for nm in ("f", "g"):
        assert all(torch.equal(u, v) for u, v in zip(pot[nm], pot2[nm]))


def test_batched_rejects_bad_arguments():
    import paper_2107_02010_amd as skh
    from paper_2107_02010_amd import _lib
    xs, as_, ys, bs = _pairs(None, seed=130)
    args = ([cuda(v) for v in xs], [cuda(v) for v in as_], [cuda(v) for v in ys],
            [cuda(v) for v in bs])
    note("batched argument checks")
    with pytest.raises(ValueError):
        skh.sinkhorn_divergence_batched(args[0], args[1][:-1], args[2], args[3])
    # empty pair, multiscale, BF16 split and p != 2 go through the C checks
    import ctypes
    x, y = args[0][0], args[2][0]
    P = _lib.default_params()
    S = (ctypes.c_double * 2)()
    ctx = skh._Ctx.get(x.device)
    xo = (ctypes.c_int64 * 3)(0, 1, 1)
    yo = (ctypes.c_int64 * 3)(0, 1, 2)
    rc = _lib.load().skh_sinkhorn_divergence_batched(ctx, x.data_ptr(), args[1][0].data_ptr(), xo,
                                                     y.data_ptr(), args[3][0].data_ptr(), yo, 2, 3,
                                                     ctypes.byref(P), S, None, None, None, None,
                                                     None)
    assert rc == _lib.SKH_EINVAL
    xo = (ctypes.c_int64 * 2)(0, 1)
    yo = (ctypes.c_int64 * 2)(0, 2)
    for field, val in (("multiscale", 1), ("precision", _lib.SKH_BF16_SPLIT), ("cost_p", 1.0)):
        P = _lib.default_params()
        setattr(P, field, val)
        rc = _lib.load().skh_sinkhorn_divergence_batched(ctx, x.data_ptr(), args[1][0].data_ptr(),
                                                         xo, y.data_ptr(), args[3][0].data_ptr(),
                                                         yo, 1, 3, ctypes.byref(P), S, None, None,
                                                         None, None, None)
        assert rc == _lib.SKH_EINVAL, field
