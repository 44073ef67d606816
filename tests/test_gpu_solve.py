"""GPU solver parity against the oracle.

Gates (two, because a relative residual of 1e-8 does not bound the solution
error of an ill-conditioned shift to 1e-6):
  * residual gate: at tol 1e-8 every GPU solution has ||b - Bx|| / ||b|| <= tol
    recomputed by the oracle's loop operator on the CPU;
  * solution gate: at tol 1e-12 the GPU solution is within 1e-6 (relative) of
    the dense Cholesky solution (images up to 32 x 32) or of the oracle CG
    solution at the same tolerance.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2306_15049_amd import rsr, synth
from conftest import to_dev, to_host

pytestmark = pytest.mark.gpu


def _case(n, seed, sigma, s, rects=6):
    pr = synth.make_problem(seed, n, n, sigma, s, rects)
    _, b = oracle.rhs(pr)
    return pr, b


def _relres(h, wh, wv, g, b, x):
    return oracle.true_relres(h, wh, wv, g, b, x)


@pytest.mark.parametrize("mode", [rsr.BATCHED, rsr.SEQUENTIAL])
def test_plain_cg_matches_cholesky_16(ctx, mode):
    pr, b = _case(16, 21, 1.5, 7)
    wh, wv = oracle.weights(pr.x_true + 0.05 * pr.noise_dir)
    gammas = synth.shift_grid(-4, 0, 6)
    print(f"plain CG 16x16 mode={mode}", flush=True)
    ctx.set_operators([(16, 16)], [pr.psf])
    ctx.update_weights(0, to_dev(wh), to_dev(wv))
    bd = to_dev(b)
    X = to_dev(np.zeros((6, 16, 16)))
    rc, st = ctx.solve(gammas, bd, X, opts=rsr.SolveOptions(tol=1e-12, mode=mode))
    assert rc == 0
    Xh = to_host(X)
    Am, Em = dense.dense_A(pr.psf, 16, 16), dense.dense_E(wh, wv)
    for l, g in enumerate(gammas):
        ref = dense.cholesky_solve(Am + g * Em, b)
        assert np.linalg.norm(Xh[l] - ref) <= 1e-6 * np.linalg.norm(ref)
        assert _relres(pr.psf, wh, wv, g, b, Xh[l]) <= 1e-12 * 1.5
        assert st[l]["converged"] == 1


def test_plain_cg_c1_residual_gate_and_counts(ctx):
    cfg = synth.config("C1")
    pr = cfg.problems[0]
    _, b = oracle.rhs(pr)
    wh, wv = oracle.unit_weights(32, 32)
    print("plain CG C1 32x32, 8 shifts", flush=True)
    ctx.set_operators([(32, 32)], [pr.psf])
    X = to_dev(np.zeros((8, 32, 32)))
    rc, st = ctx.solve(cfg.gammas, to_dev(b), X, opts=rsr.SolveOptions(tol=1e-8))
    assert rc == 0
    Xh = to_host(X)
    Xo, so = oracle.cg_shifts(pr.psf, wh, wv, cfg.gammas, b, tol=1e-8)
    for l, g in enumerate(cfg.gammas):
        assert _relres(pr.psf, wh, wv, g, b, Xh[l]) <= 1e-8
        # same method; finite-precision CG on an ill-conditioned shift is sensitive
        # to the summation order, so counts agree only loosely (they are not pinned)
        assert abs(st[l]["iters"] - so[l]["iters"]) <= max(3, 0.15 * so[l]["iters"])


def test_plain_cg_c1_solution_gate(ctx):
    cfg = synth.config("C1")
    pr = cfg.problems[0]
    _, b = oracle.rhs(pr)
    wh, wv = oracle.weights(pr.x_true + 0.05 * pr.noise_dir)
    ctx.set_operators([(32, 32)], [pr.psf])
    ctx.update_weights(0, to_dev(wh), to_dev(wv))
    X = to_dev(np.zeros((8, 32, 32)))
    rc, st = ctx.solve(cfg.gammas, to_dev(b), X, opts=rsr.SolveOptions(tol=1e-12))
    Xh = to_host(X)
    Am, Em = dense.dense_A(pr.psf, 32, 32), dense.dense_E(wh, wv)
    for l, g in enumerate(cfg.gammas):
        ref = dense.cholesky_solve(Am + g * Em, b)
        assert np.linalg.norm(Xh[l] - ref) <= 1e-6 * np.linalg.norm(ref), l


def test_ragged_multi_tile_and_zero_rhs(ctx):
    pr, b = _case(45, 22, 2.0, 9)
    h = pr.psf
    ctx.set_operators([(45, 45)], [h])
    ctx.set_tile(0, 16, 16)
    wh, wv = oracle.unit_weights(45, 45)
    gam = [1e-3, 0.1, 5.0]
    B = np.stack([b, np.zeros_like(b), b])
    X = to_dev(np.zeros((3, 45, 45)))
    rc, st = ctx.solve(gam, to_dev(B), X, opts=rsr.SolveOptions(tol=1e-10), shared_b=False)
    Xh = to_host(X)
    assert not Xh[1].any() and st[1]["iters"] == 0
    for l in (0, 2):
        assert _relres(h, wh, wv, gam[l], b, Xh[l]) <= 1e-10
        xo, so = oracle.cg(h, wh, wv, gam[l], b, tol=1e-12)
        assert np.linalg.norm(Xh[l] - xo) <= 1e-6 * np.linalg.norm(xo)


def test_maxit_reports_not_converged(ctx):
    pr, b = _case(32, 23, 1.5, 7)
    ctx.set_operators([(32, 32)], [pr.psf])
    X = to_dev(np.zeros((2, 32, 32)))
    rc, st = ctx.solve([1e-4, 1e-3], to_dev(b), X, opts=rsr.SolveOptions(tol=1e-10, maxit=5))
    assert rc == 1
    assert all(s["iters"] == 5 and s["converged"] == 0 for s in st)


@pytest.mark.parametrize("recycled", [False, True])
def test_fused_and_two_pass_iterations_agree_bitwise(ctx, monkeypatch, recycled):
    # the two iteration forms of the persistent kernel compute the same values in
    # the same order (r_j, ph_j per cell; the stencil; the partial sums), so the
    # solutions agree to the last bit; ragged tiles, several systems, local spaces
    from paper_2306_15049_amd import irn
    pr = synth.make_problem(9, 150, 203, 2.0, 13, 12)
    _, b = oracle.rhs(pr)
    cfg = synth.Config("ragged", [pr], synth.shift_grid(-4, 1, 6), 3, 12, 5, "batched")
    out = {}
    # one grid size for every form (the forms may differ in occupancy, and the
    # chunking of the reductions follows the grid)
    monkeypatch.setenv("RSR_CG_MAX_BLOCKS", "256")
    for mode in ("1", "2", "3"):
        monkeypatch.setenv("RSR_CG_MODE", mode)
        loop = irn.OuterLoop(ctx, cfg, "recycled" if recycled else "plain")
        loop.b[0] = to_dev(b)
        recs = loop.run(3 if recycled else 1)
        out[mode] = (to_host(loop.X[0]), [r.iters for r in recs])
    assert out["1"][1] == out["2"][1] == out["3"][1]
    assert np.array_equal(out["1"][0], out["2"][0]) and np.array_equal(out["1"][0], out["3"][0])
    wh, wv = (to_host(t) for t in ctx.get_weights(0))
    X = out["3"][0]
    for l, g in enumerate(cfg.gammas):
        assert oracle.true_relres(pr.psf, wh, wv, g, b, X[l]) <= 1e-8


@pytest.mark.parametrize("tile,recycled", [((16, 16), False), ((32, 32), True), ((16, 32), True)])
def test_single_system_kernel_matches_general_kernel_bitwise(ctx, monkeypatch, tile, recycled):
    # one system per launch (sequential mode), a workgroup per tile: the
    # single-system kernel keeps the tile's x, p, W and Z in registers but forms
    # the general kernel's values in the same order, so the iterates agree to the
    # last bit (ragged tiles, local spaces of up to 5 columns, 4 pixels per thread
    # with 32 x 32 tiles)
    from paper_2306_15049_amd import irn
    pr = synth.make_problem(9, 150, 203, 2.0, 13, 12)
    _, b = oracle.rhs(pr)
    cfg = synth.Config("ragged", [pr], synth.shift_grid(-4, 1, 4), 3, 12, 5, "sequential")
    out = {}
    for mode in ("1", "4"):
        monkeypatch.setenv("RSR_CG_MODE", mode)
        loop = irn.OuterLoop(ctx, cfg, "recycled" if recycled else "plain", tiles={0: tile})
        loop.b[0] = to_dev(b)
        recs = loop.run(3 if recycled else 1)
        out[mode] = (to_host(loop.X[0]), [r.iters for r in recs])
    assert out["1"][1] == out["4"][1]
    assert np.array_equal(out["1"][0], out["4"][0])
    wh, wv = (to_host(t) for t in ctx.get_weights(0))
    for l, g in enumerate(cfg.gammas):
        assert oracle.true_relres(pr.psf, wh, wv, g, b, out["4"][0][l]) <= 1e-8


def test_single_system_kernel_records_lanczos_data_bitwise(ctx, monkeypatch):
    # the correction equation's solve records CG-Lanczos data (r_j and the step
    # coefficients); its one system runs the single-system kernel unless form 0
    # is forced, and the Krylov vectors built from the record agree to the last bit
    pr = synth.make_problem(9, 150, 203, 2.0, 13, 12)
    ny, nx = pr.ny, pr.nx
    wh0, wv0 = oracle.weights(pr.x_true)
    wh1, wv1 = oracle.weights(pr.x_true + 0.05 * pr.noise_dir)
    ctx.set_operators([(ny, nx)], [pr.psf])
    ctx.set_tile(0, 16, 32)
    ctx.update_weights(0, to_dev(wh1), to_dev(wv1))
    out = {}
    for mode in ("1", "0"):
        monkeypatch.setenv("RSR_CG_MODE", mode)
        print(f"correction space, mode {mode}", flush=True)
        V, nout = ctx.correction_space(0, to_dev(pr.x_true), to_dev(wh0), to_dev(wv0), 0.3, 30, 10)
        out[mode] = (to_host(V), nout)
    assert out["1"][1] == out["0"][1] == 11
    assert np.array_equal(out["1"][0], out["0"][0])


def test_rank_two_psf_solve_matches_cholesky(ctx):
    # the first example's two-term Kronecker PSF on a 24 x 20 image (rank-R path)
    # against dense Cholesky at tight tolerance
    h = synth.kronecker_sum_psf(synth.EXAMPLE1_TERMS)
    rng = np.random.default_rng(17)
    ny, nx = 24, 20
    b = rng.standard_normal((ny, nx))
    wh, wv = oracle.weights(rng.standard_normal((ny, nx)) * 0.3)
    ctx.set_operators([(ny, nx)], [h])
    ctx.update_weights(0, to_dev(wh), to_dev(wv))
    g = [1e-3, 0.1, 10.0]
    X = to_dev(np.zeros((3, ny, nx)))
    rc, st = ctx.solve(g, to_dev(b), X, opts=rsr.SolveOptions(tol=1e-13))
    assert rc == 0
    Am, Em = dense.dense_A(h, ny, nx), dense.dense_E(wh, wv)
    Xh = to_host(X)
    for l, gg in enumerate(g):
        xr = dense.cholesky_solve(Am + gg * Em, b)
        assert np.linalg.norm(Xh[l] - xr) <= 1e-8 * np.linalg.norm(xr), l
