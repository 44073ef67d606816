"""Outer edge-preserving iteration driving the recycled shifted solver.

One outer step k (Algorithm 5, per-k solve phase) on each instance:
  1. k >= 1: new weights W_k from the previous step's selected solution
     x^(k-1, l*)  (w = ((D x)^2 + beta)^(-1/2) per difference);
  2. principal recycle space U_k from all previous solutions x^(k-1, 1..M)
     plus Ritz vectors retained from U_{k-1} (Section 5.2), stabilised by
     Algorithm 1;
  3. all shifts solved: initial guess from U_k (eq. orthupdate), local spaces
     of Ritz vectors and previous corrections (Algorithms 2-4), deflated CG.
At k = 0 there is no principal space (the first-step spike of Section 8.2).

The "plain" variant solves every shift from x0 = 0 with plain CG -- the naive
baseline of Section 8 with CG in place of MINRES; "warm" is plain CG started
from the previous outer step's solution of the same shift.

l* is fixed to the middle shift (ceil(M/2), 1-based) so that the plain and
recycled runs see identical weight sequences.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import rsr, synth


@dataclass
class StepRecord:
    k: int
    wall_ms: float
    matvec_A: int
    matvec_E: int
    iters: List[int]
    relres: List[float]
    relres_init: List[float]
    p: int = 0
    cg_kernel_ms: float = 0.0
    cg_items: int = 0
    cg_launches: int = 0
    l_star: int = -1          # shift index whose solution drives the next weights
    local_dim: List[int] = field(default_factory=list)   # local-space width used by each system


@dataclass
class RecycleParams:
    p: int
    q: int = 5
    n_ritz: int = 3
    seed_lanczos: int = 0     # k = 0, sequential: CG-Lanczos steps of the first shift that seed U (0: off)
    seed_p: int = 30          # Ritz vectors of those steps kept as the seeded U
    seed_n_ritz: int = 3      # Ritz vectors in the local spaces of the shifts after the seed
    seed_two: bool = False    # seed from two representative shifts (the first and the one at split_frac)
    correction: int = 5       # k >= 1: Krylov vectors of the correction equation added to U (0: off)
    correction_steps: int = 50    # CG steps on the correction equation
    correction_frac: float = 0.9  # the correction shift l_c = round(frac * M) (1-based)
    split_frac: float = 0.75
    beta: float = 1e-4
    cond_max: float = 1e10
    init: int = rsr.INIT_MR


def rhs_on_device(ctx: rsr.Context, inst: int, pr: synth.Problem):
    """d = K x_true + e, b = K^T d, with K applied by the library."""
    import torch
    xt = torch.from_numpy(np.ascontiguousarray(pr.x_true)).cuda()
    kx = ctx.apply(inst, rsr.OP_K, xt)
    g = torch.from_numpy(np.ascontiguousarray(pr.noise_dir)).cuda()
    e = g * (pr.noise_level * torch.linalg.vector_norm(kx) / torch.linalg.vector_norm(g))
    d = (kx + e).contiguous()
    b = ctx.apply(inst, rsr.OP_KT, d)
    return d, b


class OuterLoop:
    """Runs outer steps of one config on one context (single instance or many)."""

    def __init__(self, ctx: rsr.Context, cfg: synth.Config, method: str, rp: Optional[RecycleParams] = None,
                 tol: Optional[float] = None, tiles: Optional[Dict[int, tuple]] = None,
                 mode: Optional[int] = None, weight_rule: str = "irn", edge_p: float = 2.0,
                 lcurve: bool = False, stop_repeats: int = 3, workspace: bool = False, solver: str = "cg"):
        """weight_rule: "irn" (W = ((D x)^2 + beta)^(-1/2)) or "edge" (the cumulative edge
        rule of Sec. 2.1 with exponent edge_p).  lcurve: choose the shift that drives the
        next weights at the L-curve corner after every step; otherwise the middle shift.
        The loop reports `stopped` once that choice has repeated stop_repeats times.
        workspace: solve on a caller workspace (sized and reserved with
        rsr_workspace_size before each solve), so the solves allocate nothing.
        solver: "cg" (deflated CG) or "minres" (recycled MINRES, Sec. 2.3 and 4.2; the
        paper's inner solver) for every system of every method."""
        import torch
        if method not in ("recycled", "plain", "warm"):
            raise ValueError("method must be 'recycled', 'plain' or 'warm'")
        if weight_rule not in ("irn", "edge"):
            raise ValueError("weight_rule must be 'irn' or 'edge'")
        if solver not in ("cg", "minres"):
            raise ValueError("solver must be 'cg' or 'minres'")
        self.ctx = ctx
        self.cfg = cfg
        self.method = method
        self.rp = rp or RecycleParams(p=cfg.p, q=cfg.q)
        self.solver = rsr.SOLVER_MINRES if solver == "minres" else rsr.SOLVER_CG
        if self.solver == rsr.SOLVER_MINRES and self.rp.seed_lanczos > 0:
            raise ValueError("the principal-space seed records CG-Lanczos data: use solver='cg'")
        self.tol = cfg.tol if tol is None else tol
        self.M = len(cfg.gammas)
        self.mode = mode if mode is not None else (rsr.SEQUENTIAL if cfg.mode == "sequential" else rsr.BATCHED)
        if self.ct and (lcurve or self.rp.seed_lanczos > 0):
            raise ValueError("the L-curve choice and the seed are for deblurring instances")
        self._set_operators()
        if tiles and not self.ct:
            for i, t in tiles.items():
                ctx.set_tile(i, *t)
        self.b, self.d = [], []
        for i, pr in enumerate(cfg.problems):
            d, b = rhs_on_device(ctx, i, pr)
            self.b.append(b)
            self.d.append(d)
        self.X = [torch.zeros((self.M, p.ny, p.nx), dtype=torch.float64, device="cuda") for p in cfg.problems]
        self.k = 0
        self.weight_rule = weight_rule
        self.edge_p = float(edge_p)
        self.lcurve = lcurve
        self.stop_repeats = stop_repeats
        self.l_stars = [int(math.ceil(self.M / 2)) - 1] * len(cfg.problems)
        self.l_history: List[tuple] = []
        self.workspace = workspace
        self._ws = None

    @property
    def ct(self) -> bool:
        """Tomography instances (the second example's projector) instead of blurs."""
        return self.cfg.problems[0].ct is not None

    def _set_operators(self):
        shapes = [(p.ny, p.nx) for p in self.cfg.problems]
        if self.ct:
            self.ctx.set_ct_operators(shapes, [p.ct[0] for p in self.cfg.problems],
                                      [p.ct[1] for p in self.cfg.problems])
        else:
            self.ctx.set_operators(shapes, [p.psf for p in self.cfg.problems])

    def _workspace(self, gammas, inst, slots, o):
        """A caller workspace large enough for this solve (grown when needed)."""
        import torch
        if not self.workspace:
            return None
        nb = self.ctx.workspace_size(gammas, inst=inst, slots=slots, opts=o)
        if self._ws is None or self._ws.numel() < nb:
            self._ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
        return self._ws

    @property
    def l_star(self) -> int:
        return self.l_stars[0]

    @property
    def stopped(self) -> bool:
        """The outer stopping rule: the same choice for stop_repeats consecutive steps."""
        h = self.l_history
        return len(h) >= self.stop_repeats and len(set(h[-self.stop_repeats:])) == 1

    def reset(self):
        for i in range(len(self.cfg.problems)):
            self.X[i].zero_()
        if self.ct:
            self._set_operators()
        else:
            tiles = [self.ctx.tile(i) for i in range(len(self.cfg.problems))]
            self._set_operators()
            for i, t in enumerate(tiles):
                self.ctx.set_tile(i, *t)
        self.k = 0
        self.l_stars = [int(math.ceil(self.M / 2)) - 1] * len(self.cfg.problems)
        self.l_history = []

    def _opts(self) -> rsr.SolveOptions:
        M = self.M
        g = self.cfg.gammas
        if self.method == "plain":
            return rsr.SolveOptions(tol=self.tol, mode=self.mode, init=rsr.INIT_ZERO, solver=self.solver)
        if self.method == "warm":
            return rsr.SolveOptions(tol=self.tol, mode=self.mode,
                                    init=rsr.INIT_GIVEN if self.k > 0 else rsr.INIT_ZERO, solver=self.solver)
        split = int(math.ceil(self.rp.split_frac * M))
        jl = max(1, min(split, M)) - 1            # J_L = split (1-based)
        jr = max(split, M - 2)                    # J_R = M - 1 (1-based)
        seq = self.mode == rsr.SEQUENTIAL
        seed = seq and self.k == 0 and self.rp.seed_lanczos > 0
        return rsr.SolveOptions(tol=self.tol, mode=self.mode, init=self.rp.init if self.k > 0 else rsr.INIT_ZERO,
                                n_ritz=self.rp.n_ritz if self.k > 0 else 0, use_prev_k=self.k > 0,
                                use_prev_shift=seq, split_I=split, gamma_JL=float(g[jl]),
                                gamma_JR=float(g[min(jr, M - 1)]),
                                seed_lanczos=self.rp.seed_lanczos if seed else 0,
                                seed_p=min(self.rp.seed_p, self.rp.p) if seed else 0,
                                seed_n_ritz=self.rp.seed_n_ritz if seed else 0,
                                seed_second=(split - 1) if (seed and self.rp.seed_two and split > 1) else 0,
                                solver=self.solver)

    def step(self) -> StepRecord:
        import torch
        ctx = self.ctx
        torch.cuda.synchronize()
        a0, e0 = ctx.counters()
        t0 = time.perf_counter()
        n_inst = len(self.cfg.problems)
        p_dim = 0
        if self.k > 0:
            for i in range(n_inst):
                recycled = self.method == "recycled"
                # the correction space runs the persistent kernel: deblurring instances only
                corr = recycled and self.rp.correction > 0 and not self.ct
                if corr:
                    wold = ctx.get_weights(i)   # W_{k-1}, for the correction equation
                if self.weight_rule == "edge":
                    ctx.weights_edge_rule(i, self.X[i][self.l_stars[i]], self.edge_p)
                else:
                    ctx.weights_from_image(i, self.X[i][self.l_stars[i]], self.rp.beta)
                if recycled:
                    cand, n_extra = self.X[i], 0
                    if corr:
                        # [dx, Krylov vectors] of eq. delta at the shift l_c join the candidates
                        lc = min(self.M - 1, max(0, int(round(self.rp.correction_frac * self.M)) - 1))
                        V, nv = ctx.correction_space(i, self.X[i][lc], wold[0], wold[1], float(self.cfg.gammas[lc]),
                                                     self.rp.correction_steps, self.rp.correction)
                        cand = torch.cat([self.X[i], V[:nv]])
                        n_extra = nv
                    n_retain = max(0, self.rp.p - self.M - n_extra)
                    p_dim = ctx.set_recycle_space(i, cand, n_retain=n_retain,
                                                  gamma_retain=float(self.cfg.gammas[0]), p_max=self.rp.p,
                                                  cond_max=self.rp.cond_max)
        o = self._opts()
        iters, rel, rel0, qd = [], [], [], []
        if n_inst == 1:
            ws = self._workspace(self.cfg.gammas, None, None, o)
            rc, st = ctx.solve(self.cfg.gammas, self.b[0], self.X[0], opts=o, ws=ws)
            stats = [st]
        else:
            stats = self._solve_instances(o)
        if self.k == 0 and self.method == "recycled" and n_inst == 1:
            p_dim = ctx.recycle_info(0)[0]   # a principal space seeded during the solve
        cg_ms, launches, items = ctx.last_timing()
        if self.lcurve:
            for i in range(n_inst):
                c = ctx.lcurve(self.cfg.gammas, self.X[i], self.d[i], inst=i)[3]
                if c >= 0:
                    self.l_stars[i] = c
            self.l_history.append(tuple(self.l_stars))
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        a1, e1 = ctx.counters()
        for st in stats:
            iters += [s["iters"] for s in st]
            rel += [s["relres_true"] for s in st]
            rel0 += [s["relres_init"] for s in st]
            qd += [s["local_dim"] for s in st]
        rec = StepRecord(self.k, wall, a1 - a0, e1 - e0, iters, rel, rel0, p_dim, cg_ms, items, launches,
                         self.l_stars[0], qd)
        self.k += 1
        return rec

    def _solve_instances(self, o: rsr.SolveOptions):
        """All instances and shifts in one batched call (uneven sizes in one launch)."""
        import torch
        M = self.M
        n_inst = len(self.cfg.problems)
        inst = [i for i in range(n_inst) for _ in range(M)]
        gam = [float(g) for _ in range(n_inst) for g in self.cfg.gammas]
        slots = [l for _ in range(n_inst) for l in range(M)]
        # pack right-hand sides and solutions with a common stride
        nmax = max(p.ny * p.nx for p in self.cfg.problems)
        if not hasattr(self, "_Bp"):
            self._Bp = torch.zeros((n_inst * M, nmax), dtype=torch.float64, device="cuda")
            self._Xp = torch.zeros((n_inst * M, nmax), dtype=torch.float64, device="cuda")
            for i in range(n_inst):
                for l in range(M):
                    self._Bp[i * M + l, : self.b[i].numel()] = self.b[i].reshape(-1)
        for i in range(n_inst):
            n = self.X[i][0].numel()
            self._Xp[i * M:(i + 1) * M, :n] = self.X[i].reshape(M, -1)
        ws = self._workspace(gam, inst, slots, o)
        rc, st = self.ctx.solve(gam, self._Bp, self._Xp, inst=inst, slots=slots, opts=o, shared_b=False, ws=ws)
        for i in range(n_inst):
            n = self.X[i][0].numel()
            self.X[i].copy_(self._Xp[i * M:(i + 1) * M, :n].reshape(self.X[i].shape))
        return [st[i * M:(i + 1) * M] for i in range(n_inst)]

    def run(self, steps: int, log=None) -> List[StepRecord]:
        out = []
        for _ in range(steps):
            r = self.step()
            if log is not None:
                print(f"[{self.method}] k={r.k} wall={r.wall_ms:.2f} ms cg={r.cg_kernel_ms:.2f} ms A={r.matvec_A} "
                      f"p={r.p} iters={r.iters} relres0={[f'{v:.1e}' for v in r.relres_init]}", file=log, flush=True)
            out.append(r)
        return out
