"""GPU parity of recycled MINRES (Sec. 2.3 and 4.2) with the oracle.

* A fixed number of Lanczos steps (1, 3, 8) from zero, no local space, on a
  ragged 37 x 29 image with two shifts batched: x after m steps is the
  oracle's (dense.recycled_minres, explicit Lanczos basis and least squares)
  element by element.  After a few steps the three-term recurrence and the
  oracle's fully re-orthogonalised basis agree to rounding.
* The same with a local space: the previous correction of the slot
  (use_prev_k), which the oracle takes as Ut; both sides build K, U from it
  (eq. localU) and assemble x by eq. xFinal.
* Converged solves against Cholesky on four shifts, with the number of
  Lanczos steps close to the oracle's (the GPU has no re-orthogonalisation, so
  it may take a few more).
* The recycled outer loop with MINRES as the inner solver on the 32 x 32
  workload (sequential: g^(k-1,l) and g^(k,l-1) in the local spaces) and on
  the 256 x 256 workload (batched, 20 shifts): residual gate of every shift at
  every step with the oracle's operator, and fewer matrix-vector products than
  plain MINRES from zero after the first step.
* Descriptor checks: an unknown solver, MINRES with principal-space seeding,
  MINRES on the device-only path -> RSR_E_ARG.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2306_15049_amd import irn, rsr, synth
from conftest import to_dev, to_host

pytestmark = pytest.mark.gpu

NY, NX = 37, 29


def _problem(ctx):
    pr = synth.make_problem(31, NY, NX, 1.5, 7, 5)
    _, b = oracle.rhs(pr)
    ctx.set_operators([(NY, NX)], [pr.psf])
    wh, wv = oracle.weights(pr.x_true + 0.05 * pr.noise_dir)
    ctx.update_weights(0, to_dev(wh), to_dev(wv))
    Am, Em = dense.dense_A(pr.psf, NY, NX), dense.dense_E(wh, wv)
    return pr, b, Am, Em


def _minres(**kw):
    return rsr.SolveOptions(solver=rsr.SOLVER_MINRES, **kw)


def test_fixed_steps_match_oracle(ctx):
    pr, b, Am, Em = _problem(ctx)
    gammas = [0.05, 0.8]
    for m in (1, 3, 8):
        print(f"MINRES {NY}x{NX}: {m} steps from zero", flush=True)
        X = to_dev(np.zeros((2, NY, NX)))
        rc, st = ctx.solve(gammas, to_dev(b), X, opts=_minres(tol=1e-15, maxit=m))
        Xh = to_host(X)
        for l, g in enumerate(gammas):
            assert st[l]["iters"] == m and st[l]["converged"] == 0
            assert st[l]["matvec_A"] == m + 1          # m Lanczos steps + the true residual
            xr, mr, _ = dense.recycled_minres(Am + g * Em, b, np.zeros(NY * NX), None, tol=1e-15, maxit=m)
            assert mr == m
            err = np.linalg.norm(Xh[l].ravel() - xr) / np.linalg.norm(xr)
            assert err <= 1e-11, (m, l, err)


def test_fixed_steps_with_local_space_match_oracle(ctx):
    pr, b, Am, Em = _problem(ctx)
    rng = np.random.default_rng(3)
    b2 = b + 0.2 * np.linalg.norm(b) / np.sqrt(b.size) * rng.standard_normal(b.shape)
    gammas = [0.3]
    Bm = Am + gammas[0] * Em
    for m in (1, 2, 6):
        # the first solve of slot 0 (from zero) leaves its correction g = x as the
        # slot's previous correction
        X = to_dev(np.zeros((1, NY, NX)))
        rc, _ = ctx.solve(gammas, to_dev(b), X, opts=rsr.SolveOptions(tol=1e-12))
        assert rc == 0
        g = to_host(X)[0].ravel()
        print(f"MINRES {NY}x{NX} with Ut = g: {m} steps", flush=True)
        X2 = to_dev(np.zeros((1, NY, NX)))
        rc, st = ctx.solve(gammas, to_dev(b2), X2, opts=_minres(tol=1e-15, maxit=m, use_prev_k=True))
        assert st[0]["local_dim"] == 1
        xr, mr, _ = dense.recycled_minres(Bm, b2, np.zeros(NY * NX), g[:, None], tol=1e-15, maxit=m)
        assert mr == m and st[0]["iters"] == m
        err = np.linalg.norm(to_host(X2)[0].ravel() - xr) / np.linalg.norm(xr)
        assert err <= 1e-11, (m, err)


def test_converged_against_cholesky(ctx):
    pr, b, Am, Em = _problem(ctx)
    gammas = [0.01, 0.1, 1.0, 10.0]
    X = to_dev(np.zeros((4, NY, NX)))
    print(f"MINRES {NY}x{NX}: converged, 4 shifts", flush=True)
    rc, st = ctx.solve(gammas, to_dev(b), X, opts=_minres(tol=1e-10))
    assert rc == 0
    Xh = to_host(X)
    for l, g in enumerate(gammas):
        Bm = Am + g * Em
        xs = dense.cholesky_solve(Bm, b)
        cond = np.linalg.cond(Bm)
        assert np.linalg.norm(Xh[l].ravel() - xs.ravel()) <= 1e-10 * cond * np.linalg.norm(xs), l
        assert oracle.true_relres(pr.psf, *ctx_weights(ctx), g, b, Xh[l]) <= 1e-10
        _, mr, _ = dense.recycled_minres(Bm, b, np.zeros(NY * NX), None, tol=1e-10)
        assert mr - 2 <= st[l]["iters"] <= int(1.3 * mr) + 5, (l, mr, st[l]["iters"])


def ctx_weights(ctx):
    return tuple(to_host(t) for t in ctx.get_weights(0))


@pytest.mark.parametrize("name,mode", [("C1", rsr.SEQUENTIAL), ("C2", rsr.BATCHED)])
def test_recycled_loop_with_minres(ctx, name, mode):
    cfg = synth.config(name)
    pr = cfg.problems[0]
    _, b = oracle.rhs(pr)
    loops = {}
    mv = {}
    for method in ("recycled", "plain"):
        loop = irn.OuterLoop(ctx, cfg, method, mode=mode, solver="minres")
        loop.b[0] = to_dev(b)
        mv[method] = []
        steps = min(cfg.outer_steps, 3)
        for k in range(steps):
            print(f"{name} {method} MINRES step {k}", flush=True)
            rec = loop.step()
            assert max(rec.relres) <= cfg.tol, (method, k)
            mv[method].append(rec.matvec_A)
            if method == "recycled" and k > 0:
                assert rec.p > 0 and max(rec.relres_init) < 1.0
            wh, wv = ctx_weights(ctx)
            Xh = to_host(loop.X[0])
            for l, g in enumerate(cfg.gammas):
                rel = oracle.true_relres(pr.psf, wh, wv, g, b, Xh[l])
                assert rel <= cfg.tol, (method, k, l, rel)
        loops[method] = loop
    # recycling saves products after the first step (same weights sequence: l* fixed)
    assert sum(mv["recycled"][1:]) < sum(mv["plain"][1:]), mv


def test_descriptor_checks(ctx):
    n = 16
    ctx.set_operators([(n, n)], [np.ones((1, 1))])
    b = to_dev(np.ones((n, n)))
    X = to_dev(np.zeros((2, n, n)))

    def status(fn):
        with pytest.raises(rsr.RsrError) as e:
            fn()
        return e.value.status

    assert status(lambda: ctx.solve([0.1, 1.0], b, X, opts=rsr.SolveOptions(solver=2))) == -1
    assert status(lambda: ctx.solve([0.1, 1.0], b, X, opts=_minres(mode=rsr.SEQUENTIAL, seed_lanczos=8,
                                                                   seed_p=4))) == -1
    import torch
    nb = ctx.workspace_size([0.1, 1.0], opts=rsr.SolveOptions(), kind=rsr.WS_DEVICE, ld_x=n * n)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    stats = torch.zeros((2, 4), dtype=torch.float64, device="cuda")
    assert status(lambda: ctx.solve_async([0.1, 1.0], b, X, ws, stats, opts=_minres())) == -1
    rc, st = ctx.solve([0.1, 1.0], b, X, opts=_minres(tol=1e-10))
    assert rc == 0
