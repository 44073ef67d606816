"""The device-only solve (rsr_solve_shift_set_async) and its HIP graph.

* Eagerly it matches rsr_solve_shift_set's plain CG: same iteration counts,
  solutions within 1e-12 relative, the residual gate with the oracle operator.
* Recorded once into a graph (torch.cuda.graph stream capture) and replayed
  several times with eager work and synchronisations between the replays and a
  new right-hand side written into the recorded buffer before each replay:
  every replay equals an eager solve of that right-hand side and passes the
  residual gate; a warm-started graph (x0 = the previous replay's solution)
  passes it too with fewer iterations.
"""
import numpy as np
import pytest

import oracle
from paper_2306_15049_amd import rsr, synth
from conftest import to_dev, to_host

pytestmark = pytest.mark.gpu


def _setup(ctx, n=96, seed=13):
    pr = synth.make_problem(seed, n, n, 2.0, 13, 10)
    _, b = oracle.rhs(pr)
    ctx.set_operators([(n, n)], [pr.psf])
    wh, wv = oracle.weights(pr.x_true + 0.05 * pr.noise_dir)
    ctx.update_weights(0, to_dev(wh), to_dev(wv))
    return pr, b, wh, wv


def test_device_only_solve_matches_the_host_driven_one(ctx, torch_cuda):
    torch = torch_cuda
    n = 96
    pr, b, wh, wv = _setup(ctx, n)
    g = [1e-4, 1e-2, 0.3, 5.0]
    m = len(g)
    opts = rsr.SolveOptions(tol=1e-10, maxit=5000)
    Xr = to_dev(np.zeros((m, n, n)))
    rc, st = ctx.solve(g, to_dev(b), Xr, opts=opts)
    assert rc == 0
    nb = ctx.workspace_size(g, opts=opts, kind=rsr.WS_DEVICE, ld_x=n * n)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    stats = torch.zeros((m, 4), dtype=torch.float64, device="cuda")
    Xa = to_dev(np.full((m, n, n), 7.0))
    n0 = ctx.allocation_count()
    ctx.solve_async(g, to_dev(b), Xa, ws, stats, opts=opts)
    torch.cuda.synchronize()
    assert ctx.allocation_count() == n0
    S = to_host(stats)
    assert [int(v) for v in S[:, 0]] == [s["iters"] for s in st]
    assert np.all(S[:, 1] == 1) and np.all(S[:, 2] <= 1e-10)
    A, R = to_host(Xa), to_host(Xr)
    for l, gg in enumerate(g):
        assert np.linalg.norm(A[l] - R[l]) <= 1e-12 * np.linalg.norm(R[l])
        rel = oracle.true_relres(pr.psf, wh, wv, gg, b, A[l])
        assert rel <= 1e-10 and abs(rel - S[l, 2]) <= 1e-3 * rel + 1e-16


def test_recorded_graph_replays_match_eager_solves(ctx, torch_cuda):
    torch = torch_cuda
    n = 96
    pr, b, wh, wv = _setup(ctx, n)
    g = [1e-3, 3e-2, 1.0]
    m = len(g)
    opts = rsr.SolveOptions(tol=1e-10, maxit=5000)
    rng = np.random.default_rng(5)
    rhs = [b + 0.05 * np.abs(b).max() * rng.standard_normal(b.shape) for _ in range(3)]
    nb = ctx.workspace_size(g, opts=opts, kind=rsr.WS_DEVICE, ld_x=n * n)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    stats = torch.zeros((m, 4), dtype=torch.float64, device="cuda")
    bbuf = to_dev(rhs[0])
    X = to_dev(np.zeros((m, n, n)))
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        ctx.solve_async(g, bbuf, X, ws, stats, opts=opts)
    torch.cuda.synchronize()
    for k, bk in enumerate(rhs):
        bbuf.copy_(to_dev(bk))
        X.fill_(3.0)                                   # the ZERO start must overwrite it
        graph.replay()
        torch.cuda.synchronize()
        Xg, S = to_host(X), to_host(stats)
        # eager work between replays, on other buffers
        Xe = to_dev(np.zeros((m, n, n)))
        rc, st = ctx.solve(g, to_dev(bk), Xe, opts=opts)
        assert rc == 0
        E = to_host(Xe)
        assert [int(v) for v in S[:, 0]] == [s["iters"] for s in st], k
        for l, gg in enumerate(g):
            assert np.linalg.norm(Xg[l] - E[l]) <= 1e-12 * np.linalg.norm(E[l]), (k, l)
            assert oracle.true_relres(pr.psf, wh, wv, gg, bk, Xg[l]) <= 1e-10, (k, l)
    # a warm-started graph: x0 = what X holds when it is replayed
    wopts = rsr.SolveOptions(tol=1e-10, maxit=5000, init=rsr.INIT_GIVEN)
    wgraph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(wgraph):
        ctx.solve_async(g, bbuf, X, ws, stats, opts=wopts)
    torch.cuda.synchronize()
    cold = to_host(stats)[:, 0].copy()
    bbuf.copy_(to_dev(rhs[-1] * (1.0 + 1e-3)))
    wgraph.replay()
    torch.cuda.synchronize()
    S = to_host(stats)
    Xg = to_host(X)
    assert np.all(S[:, 0] < cold)
    for l, gg in enumerate(g):
        assert oracle.true_relres(pr.psf, wh, wv, gg, rhs[-1] * (1.0 + 1e-3), Xg[l]) <= 1e-10
