"""GPU parity of the adjoint gradients against the oracle.

The reference is the dense implicit-function gradient of the exact solutions
(oracle.dense.exact_gradients, itself pinned to torch CPU autograd and finite
differences); the autograd wrapper is checked with central finite differences
of the GPU forward map on a 24 x 24 copy of the differentiation workload.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2306_15049_amd import rsr, synth
from conftest import to_dev, to_host

pytestmark = pytest.mark.gpu


def _case():
    cfg = synth.config("C5_small")
    pr = cfg.problems[0]
    _, b = oracle.rhs(pr)
    wh, wv = oracle.weights(pr.x_true + 0.05 * pr.noise_dir)
    return cfg, pr, b, wh, wv


def test_adjoint_matches_dense_gradient(ctx):
    cfg, pr, b, wh, wv = _case()
    gammas = cfg.gammas[::4]          # 4 shifts across 1e-5..1e1
    ctx.set_operators([(24, 24)], [pr.psf])
    ctx.update_weights(0, to_dev(wh), to_dev(wv))
    X = to_dev(np.zeros((len(gammas), 24, 24)))
    opts = rsr.SolveOptions(tol=1e-12)
    rc, st = ctx.solve(gammas, to_dev(b), X, opts=opts)
    assert rc == 0
    Gbar = 2.0 * (X - to_dev(np.broadcast_to(pr.x_true, (len(gammas), 24, 24)).copy()))
    Lam = to_dev(np.zeros((len(gammas), 24, 24)))
    rc, dg, dwh, dwv, db, sta = ctx.adjoint(gammas, X, Gbar.contiguous(), Lam, opts=opts)
    assert rc == 0
    Xr, dg_r, dwh_r, dwv_r = dense.exact_gradients(pr.psf, wh, wv, gammas, b, pr.x_true)
    np.testing.assert_allclose(dg, dg_r, rtol=1e-6)
    sc = max(np.abs(dwh_r).max(), np.abs(dwv_r).max())
    np.testing.assert_allclose(to_host(dwh), dwh_r, rtol=0, atol=1e-6 * sc)
    np.testing.assert_allclose(to_host(dwv), dwv_r, rtol=0, atol=1e-6 * sc)
    assert not to_host(dwh)[:, -1].any() and not to_host(dwv)[-1, :].any()
    # dL/db = sum_l lambda_l = sum_l B_l^{-1} Gbar_l
    Am, Em = dense.dense_A(pr.psf, 24, 24), dense.dense_E(wh, wv)
    G = to_host(Gbar)
    db_r = sum(dense.cholesky_solve(Am + g * Em, G[l]) for l, g in enumerate(gammas))
    np.testing.assert_allclose(to_host(db), db_r, rtol=0, atol=1e-7 * np.abs(db_r).max())


def test_autograd_function_finite_differences(ctx, torch_cuda):
    torch = torch_cuda
    from paper_2306_15049_amd.autograd import RecycledShiftSolve
    cfg, pr, b, wh, wv = _case()
    ctx.set_operators([(24, 24)], [pr.psf])
    gam = torch.tensor([1e-3, 1e-1, 2.0], dtype=torch.float64, requires_grad=True)
    twh = to_dev(wh).requires_grad_(True)
    twv = to_dev(wv).requires_grad_(True)
    tb = to_dev(b).requires_grad_(True)
    xt = to_dev(pr.x_true)
    opts = rsr.SolveOptions(tol=1e-13)

    def loss(g, h, v, bb):
        X = RecycledShiftSolve.apply(ctx, g, h, v, bb, 0, opts)
        return ((X - xt) ** 2).sum()

    L = loss(gam, twh, twv, tb)
    L.backward()
    # central differences, relative step for gamma, directional for w and b
    with torch.no_grad():
        for l in range(3):
            h = 1e-6 * float(gam[l])
            gp = gam.detach().clone(); gp[l] += h
            gm = gam.detach().clone(); gm[l] -= h
            fd = (loss(gp, twh.detach(), twv.detach(), tb.detach()) - loss(gm, twh.detach(), twv.detach(), tb.detach())) / (2 * h)
            assert abs(float(fd) - float(gam.grad[l])) <= 1e-5 * abs(float(gam.grad[l])) + 1e-12
        rng = np.random.default_rng(7)
        vh = to_dev(rng.standard_normal((24, 24)) * (wh != 0))
        vv = to_dev(rng.standard_normal((24, 24)) * (wv != 0))
        eps = 1e-6 * float(twh.abs().max())
        fd = (loss(gam.detach(), twh.detach() + eps * vh, twv.detach() + eps * vv, tb.detach()) -
              loss(gam.detach(), twh.detach() - eps * vh, twv.detach() - eps * vv, tb.detach())) / (2 * eps)
        an = float((twh.grad * vh).sum() + (twv.grad * vv).sum())
        assert abs(float(fd) - an) <= 1e-5 * abs(an)
        vb = to_dev(rng.standard_normal((24, 24)))
        eps = 1e-6 * float(tb.abs().max())
        fd = (loss(gam.detach(), twh.detach(), twv.detach(), tb.detach() + eps * vb) -
              loss(gam.detach(), twh.detach(), twv.detach(), tb.detach() - eps * vb)) / (2 * eps)
        an = float((tb.grad * vb).sum())
        assert abs(float(fd) - an) <= 1e-5 * abs(an)
