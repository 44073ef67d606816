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


def _recycled_setup(ctx, cfg, pr, b, mode):
    """Outer step 0 (plain, W = I), then W_1 from the middle shift's solution and
    the principal space from the step-0 solutions, as the outer loop's step 1 does."""
    n = pr.ny
    M = len(cfg.gammas)
    ctx.set_operators([(n, n)], [pr.psf])
    X0 = to_dev(np.zeros((M, n, n)))
    rc, _ = ctx.solve(cfg.gammas, to_dev(b), X0, opts=rsr.SolveOptions(tol=1e-10, mode=mode))
    assert rc == 0
    lstar = (M + 1) // 2 - 1
    ctx.weights_from_image(0, X0[lstar].contiguous(), 1e-4)
    p = ctx.set_recycle_space(0, X0, p_max=cfg.p)
    assert p > 0
    split = int(np.ceil(0.75 * M))
    return rsr.SolveOptions(tol=1e-12, mode=mode, init=rsr.INIT_MR, n_ritz=3, use_prev_k=True,
                            use_prev_shift=mode == rsr.SEQUENTIAL, split_I=split,
                            gamma_JL=float(cfg.gammas[split - 1]), gamma_JR=float(cfg.gammas[M - 1]))


@pytest.mark.parametrize("mode", [rsr.BATCHED, rsr.SEQUENTIAL])
def test_recycled_adjoint_matches_dense_gradient(ctx, torch_cuda, mode):
    # forward and adjoint both recycled (principal space, minimum-residual guess,
    # Ritz vectors, previous corrections), through the autograd wrapper; two
    # backward passes so that the second adjoint also has its own previous
    # corrections; against the dense implicit gradient at the same weights
    torch = torch_cuda
    from paper_2306_15049_amd.autograd import RecycledShiftSolve
    cfg, pr, b, _, _ = _case()
    opts = _recycled_setup(ctx, cfg, pr, b, mode)
    wh_d, wv_d = ctx.get_weights(0)
    wh, wv = to_host(wh_d), to_host(wv_d)
    gam = torch.tensor(cfg.gammas, dtype=torch.float64, requires_grad=True)
    twh = wh_d.clone().requires_grad_(True)
    twv = wv_d.clone().requires_grad_(True)
    xt = to_dev(pr.x_true)
    Xr, dg_r, dwh_r, dwv_r = dense.exact_gradients(pr.psf, wh, wv, cfg.gammas, b, pr.x_true)
    sc = max(np.abs(dwh_r).max(), np.abs(dwv_r).max())
    for rep in range(2):
        for t in (gam, twh, twv):
            t.grad = None
        X = RecycledShiftSolve.apply(ctx, gam, twh, twv, to_dev(b), 0, opts)
        ((X - xt) ** 2).sum().backward()
        p, _, _ = ctx.recycle_info(0)
        assert p > 0                              # the principal space survived both passes
        np.testing.assert_allclose(to_host(X), Xr, rtol=0, atol=1e-6 * np.abs(Xr).max())
        np.testing.assert_allclose(gam.grad.numpy(), dg_r, rtol=1e-6, atol=1e-9 * np.abs(dg_r).max())
        np.testing.assert_allclose(to_host(twh.grad), dwh_r, rtol=0, atol=1e-6 * sc)
        np.testing.assert_allclose(to_host(twv.grad), dwv_r, rtol=0, atol=1e-6 * sc)


def test_recycled_adjoint_uses_the_recycle_spaces(ctx):
    # the adjoint systems start from the principal space and carry local spaces
    # (Ritz block + the forward correction of their shift), and their groups
    # follow the shift index, not the adjoint slot
    cfg, pr, b, _, _ = _case()
    opts = _recycled_setup(ctx, cfg, pr, b, rsr.BATCHED)
    M = len(cfg.gammas)
    X = to_dev(np.zeros((M, 24, 24)))
    rc, st = ctx.solve(cfg.gammas, to_dev(b), X, opts=opts)
    assert rc == 0
    Gbar = (2.0 * (X - to_dev(np.broadcast_to(pr.x_true, (M, 24, 24)).copy()))).contiguous()
    Lam = to_dev(np.zeros((M, 24, 24)))
    rc, dg, dwh, dwv, db, sta = ctx.adjoint(cfg.gammas, X, Gbar, Lam, opts=opts)
    assert rc == 0
    assert all(s["local_dim"] == 4 for s in sta)   # 3 Ritz vectors + the forward correction
    assert all(s["relres_init"] < 1.0 for s in sta)
    wh, wv = (to_host(t) for t in ctx.get_weights(0))
    G, L = to_host(Gbar), to_host(Lam)
    for l, g in enumerate(cfg.gammas):
        assert oracle.true_relres(pr.psf, wh, wv, g, G[l], L[l]) <= 1e-12, l


def test_c5_recycled_adjoint_full_size(ctx, torch_cuda):
    # 512 x 512, 16 shifts: recycled forward and adjoint.  Every adjoint solution
    # passes the residual gate with the oracle operator; dL/dgamma and dL/dw are
    # recomputed on the CPU from (x, lambda) with the oracle's E and D; central
    # differences of the GPU forward map (relative step for gamma, a random
    # direction for w) agree with the gradient
    torch = torch_cuda
    from paper_2306_15049_amd.autograd import RecycledShiftSolve
    cfg = synth.config("C5")
    pr = cfg.problems[0]
    _, b = oracle.rhs(pr)
    M = len(cfg.gammas)
    print("C5 setup (512^2, 16 shifts)", flush=True)
    opts = _recycled_setup(ctx, cfg, pr, b, rsr.BATCHED)
    wh_d, wv_d = ctx.get_weights(0)
    wh, wv = to_host(wh_d), to_host(wv_d)
    gam = torch.tensor(cfg.gammas, dtype=torch.float64, requires_grad=True)
    twh = wh_d.clone().requires_grad_(True)
    twv = wv_d.clone().requires_grad_(True)
    xt = to_dev(pr.x_true)
    bd = to_dev(b)
    print("C5 recycled forward + adjoint", flush=True)
    X = RecycledShiftSolve.apply(ctx, gam, twh, twv, bd, 0, opts)
    ((X - xt) ** 2).sum().backward()
    Xh = to_host(X)
    # the adjoint solutions, by a direct call with the same options
    Gbar = (2.0 * (X.detach() - xt)).contiguous()
    Lam = torch.zeros_like(Gbar)
    rc, dg, dwh, dwv, db, sta = ctx.adjoint(cfg.gammas, X.detach().contiguous(), Gbar, Lam, opts=opts)
    assert rc == 0 and all(s["local_dim"] > 0 for s in sta)
    Gh, Lh = to_host(Gbar), to_host(Lam)
    for l in (0, 5, 10, 15):
        assert oracle.true_relres(pr.psf, wh, wv, cfg.gammas[l], Gh[l], Lh[l]) <= 1e-12, l
        ex = oracle.apply_E(wh, wv, Xh[l]).ravel()
        np.testing.assert_allclose(dg[l], -(Lh[l].ravel() @ ex), rtol=1e-10)
    dwh_c = np.zeros_like(wh)
    dwv_c = np.zeros_like(wv)
    for l, g in enumerate(cfg.gammas):
        lh, lv = oracle.diff(Lh[l])
        xh, xv = oracle.diff(Xh[l])
        dwh_c -= g * lh * xh
        dwv_c -= g * lv * xv
    sc = max(np.abs(dwh_c).max(), np.abs(dwv_c).max())
    np.testing.assert_allclose(to_host(dwh), dwh_c, rtol=0, atol=1e-10 * sc)
    np.testing.assert_allclose(to_host(dwv), dwv_c, rtol=0, atol=1e-10 * sc)
    np.testing.assert_allclose(gam.grad.numpy(), dg, rtol=1e-8)
    # central differences of the forward map (plain CG at tight tolerance, so the
    # difference quotient sees the exact solutions, not the recycled history)
    fopts = rsr.SolveOptions(tol=1e-13, mode=rsr.BATCHED)
    h_rel = cfg.extra["fd_h"]

    def loss(g, h_, v_):
        ctx.update_weights(0, h_, v_)
        Xf = to_dev(np.zeros((len(g), 512, 512)))
        rc, _ = ctx.solve(g, bd, Xf, opts=fopts)
        assert rc in (0, 1)
        return ((Xf - xt) ** 2).sum(dim=(1, 2))

    with torch.no_grad():
        for l in (2, 8, 14):
            h = h_rel * cfg.gammas[l]
            Lp = float(loss([cfg.gammas[l] + h], wh_d, wv_d)[0])
            Lm = float(loss([cfg.gammas[l] - h], wh_d, wv_d)[0])
            fd = (Lp - Lm) / (2 * h)
            print(f"C5 dL/dgamma[{l}] fd {fd:.10e} adjoint {dg[l]:.10e}", flush=True)
            assert abs(fd - dg[l]) <= 1e-5 * abs(dg[l]), (l, fd, dg[l])
        rng = np.random.default_rng(9)
        vh = to_dev(rng.standard_normal((512, 512)) * (wh != 0))
        vv = to_dev(rng.standard_normal((512, 512)) * (wv != 0))
        eps = h_rel * float(wh_d.abs().max())
        sel = [3, 12]
        g_sel = [cfg.gammas[l] for l in sel]
        Lp = loss(g_sel, (wh_d + eps * vh).contiguous(), (wv_d + eps * vv).contiguous())
        Lm = loss(g_sel, (wh_d - eps * vh).contiguous(), (wv_d - eps * vv).contiguous())
        fd = float((Lp - Lm).sum()) / (2 * eps)
        # the directional derivative of the two selected terms of L
        an = 0.0
        for l in sel:
            lh, lv = oracle.diff(Lh[l])
            xh, xv = oracle.diff(Xh[l])
            an -= cfg.gammas[l] * float((lh * xh * to_host(vh)).sum() + (lv * xv * to_host(vv)).sum())
        print(f"C5 directional dL/dw fd {fd:.10e} adjoint {an:.10e}", flush=True)
        assert abs(fd - an) <= 1e-5 * abs(an)
