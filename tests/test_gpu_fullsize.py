"""GPU parity at the full workload sizes, in the launch configuration the
benchmark uses.

* 1024 x 1024, delta PSF and W = 1: the exact solution is the closed form
  IDCT(DCT(b) / (1 + gamma lambda_ij)) (Neumann Laplacian), so the solution
  gate holds at full size.
* 1024 x 1024, Gaussian PSF sigma = 4 at 21 x 21, shifts batched: residual
  gate with the oracle's loop operator on the CPU.
* 256 x 256 benchmark workload, recycled outer loop: residual gate of every
  shift at every step with the oracle's operator, and a sampled solution gate
  against the oracle's own CG at tight tolerance.
"""
import numpy as np
import pytest

import oracle
from oracle import dense
from paper_2306_15049_amd import irn, rsr, synth
from conftest import to_dev, to_host

pytestmark = pytest.mark.gpu


def test_delta_psf_full_size_closed_form(ctx):
    n = 1024
    rng = np.random.default_rng(11)
    b = rng.standard_normal((n, n))
    ctx.set_operators([(n, n)], [np.ones((1, 1))])
    gammas = [1e-2, 1.0, 10.0]
    X = to_dev(np.zeros((3, n, n)))
    print("delta PSF 1024^2 batched", flush=True)
    rc, st = ctx.solve(gammas, to_dev(b), X, opts=rsr.SolveOptions(tol=1e-12))
    assert rc == 0
    Xh = to_host(X)
    for l, g in enumerate(gammas):
        ref = dense.neumann_dct_solve(b, g)
        assert np.linalg.norm(Xh[l] - ref) <= 1e-9 * np.linalg.norm(ref), l


def test_gaussian_full_size_residual_gate(ctx):
    cfg = synth.config("C3")
    pr = cfg.problems[0]
    _, b = oracle.rhs(pr)
    ctx.set_operators([(1024, 1024)], [pr.psf])
    wh, wv = oracle.weights(pr.x_true + 0.02 * pr.noise_dir)
    ctx.update_weights(0, to_dev(wh), to_dev(wv))
    gammas = [cfg.gammas[10], cfg.gammas[31]]
    X = to_dev(np.zeros((2, 1024, 1024)))
    print("C3-size Gaussian 2 shifts batched", flush=True)
    rc, st = ctx.solve(gammas, to_dev(b), X, opts=rsr.SolveOptions(tol=1e-8))
    assert rc == 0
    Xh = to_host(X)
    for l, g in enumerate(gammas):
        assert oracle.true_relres(pr.psf, wh, wv, g, b, Xh[l]) <= 1e-8


def test_benchmark_workload_recycled_steps(ctx):
    cfg = synth.config("C2")
    pr = cfg.problems[0]
    _, b = oracle.rhs(pr)
    loop = irn.OuterLoop(ctx, cfg, "recycled")
    loop.b[0] = to_dev(b)
    for k in range(3):
        print(f"C2 recycled step {k}", flush=True)
        loop.step()
        wh, wv = (to_host(t) for t in ctx.get_weights(0))
        X = to_host(loop.X[0])
        for l in (0, 9, 19):                # sampled shifts: both ends and the middle
            assert oracle.true_relres(pr.psf, wh, wv, cfg.gammas[l], b, X[l]) <= 1e-8, (k, l)
    # solution gate on the best-conditioned shift against the oracle CG at tight tolerance
    l = 13
    xo, so = oracle.cg(pr.psf, wh, wv, cfg.gammas[l], b, tol=1e-12)
    assert np.linalg.norm(X[l] - xo) <= 1e-6 * np.linalg.norm(xo)
