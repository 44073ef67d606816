"""Solves and adjoints on a caller workspace (the boundary's ownership rule:
the caller owns the scratch, the library allocates nothing during the call).

* The recycled outer loop on the 32 x 32 workload, one shift at a time and
  batched, and the 64-instance loop on small copies: the same solutions to the
  last bit and the same iteration counts as with the library's own scratch,
  and no device or pinned allocation during the workspace solves.
* A workspace of half the size rsr_workspace_size gives (less than the
  per-system vectors alone), or a misaligned one, is refused with RSR_E_ARG.
* The recycled adjoint on a workspace equals the one on library scratch.
"""
import numpy as np
import pytest

import oracle
from paper_2306_15049_amd import irn, rsr, synth
from conftest import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,mode,small", [("C1", rsr.SEQUENTIAL, None), ("C1", rsr.BATCHED, None),
                                             ("C4", rsr.BATCHED, 40)])
def test_workspace_loop_matches_library_scratch(ctx, torch_cuda, name, mode, small):
    torch = torch_cuda
    cfg = synth.config(name, small=small)
    if name == "C4":
        cfg.problems = cfg.problems[:6]
    out = {}
    for use_ws in (False, True):
        loop = irn.OuterLoop(ctx, cfg, "recycled", mode=mode, workspace=use_ws)
        recs = loop.run(cfg.outer_steps)
        out[use_ws] = ([to_host(x) for x in loop.X], [r.iters for r in recs], loop)
    for a, b in zip(out[False][0], out[True][0]):
        assert np.array_equal(a, b)
    assert out[False][1] == out[True][1]
    # one more recycled step on the workspace: no allocation inside the solve
    loop = out[True][2]
    o = loop._opts()
    M = len(cfg.gammas)
    if len(cfg.problems) == 1:
        ws = loop._workspace(cfg.gammas, None, None, o)
        n0 = ctx.allocation_count()
        rc, st = ctx.solve(cfg.gammas, loop.b[0], loop.X[0], opts=o, ws=ws)
        assert ctx.allocation_count() == n0
        assert rc == 0


def test_workspace_size_is_enforced(ctx, torch_cuda):
    torch = torch_cuda
    pr = synth.make_problem(3, 40, 56, 1.5, 7, 5)
    _, b = oracle.rhs(pr)
    ctx.set_operators([(40, 56)], [pr.psf])
    g = [1e-3, 1e-1, 1.0]
    nb = ctx.workspace_size(g)
    assert nb > 0
    X = to_dev(np.zeros((3, 40, 56)))
    short = torch.empty(nb // 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(rsr.RsrError) as e:
        ctx.solve(g, to_dev(b), X, ws=short)
    assert e.value.status == -1
    big = torch.empty(nb + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(rsr.RsrError) as e:
        ctx.solve(g, to_dev(b), X, ws=big[8:])
    assert e.value.status == -1
    n0 = ctx.allocation_count()
    rc, st = ctx.solve(g, to_dev(b), X, ws=big[:nb])
    assert rc == 0 and ctx.allocation_count() == n0
    Xh = to_host(X)
    wh, wv = oracle.unit_weights(40, 56)
    for l, gg in enumerate(g):
        assert oracle.true_relres(pr.psf, wh, wv, gg, b, Xh[l]) <= 1e-8


def test_adjoint_on_workspace_matches(ctx, torch_cuda):
    torch = torch_cuda
    cfg = synth.config("C5_small")
    pr = cfg.problems[0]
    _, b = oracle.rhs(pr)
    M = len(cfg.gammas)
    res = {}
    for use_ws in (False, True):
        ctx.set_operators([(24, 24)], [pr.psf])
        X0 = to_dev(np.zeros((M, 24, 24)))
        rc, _ = ctx.solve(cfg.gammas, to_dev(b), X0, opts=rsr.SolveOptions(tol=1e-10))
        ctx.weights_from_image(0, X0[M // 2 - 1].contiguous(), 1e-4)
        ctx.set_recycle_space(0, X0, p_max=cfg.p)
        opts = rsr.SolveOptions(tol=1e-12, init=rsr.INIT_MR, n_ritz=3, use_prev_k=True, split_I=12,
                                gamma_JL=float(cfg.gammas[11]), gamma_JR=float(cfg.gammas[15]))
        X = to_dev(np.zeros((M, 24, 24)))
        ws = None
        if use_ws:
            nb = max(ctx.workspace_size(cfg.gammas, opts=opts), ctx.workspace_size(cfg.gammas, opts=opts, adjoint=True))
            ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        rc, st = ctx.solve(cfg.gammas, to_dev(b), X, opts=opts, ws=ws)
        assert rc == 0
        G = (2.0 * (X - to_dev(np.broadcast_to(pr.x_true, (M, 24, 24)).copy()))).contiguous()
        Lam = to_dev(np.zeros((M, 24, 24)))
        n0 = ctx.allocation_count()
        rc, dg, dwh, dwv, db, sta = ctx.adjoint(cfg.gammas, X, G, Lam, opts=opts, ws=ws)
        if use_ws:
            assert ctx.allocation_count() == n0
        assert rc == 0
        res[use_ws] = (to_host(X), to_host(Lam), dg, to_host(dwh), to_host(dwv), to_host(db))
    for a, b_ in zip(res[False], res[True]):
        assert np.array_equal(a, b_)
