"""Differentiable shifted solves: X = RecycledShiftSolve.apply(...).

Forward solves (A + gamma_l E(w)) x_l = b for every shift with the recycled
solver; backward returns dL/dgamma, dL/dw_h, dL/dw_v and dL/db by the adjoint
of the exact solution map (implicit differentiation): the systems are
symmetric, so one recycled solve B_l lambda_l = dL/dx_l per shift gives
  dL/dgamma_l = -lambda_l^T E x_l,
  dL/dw       = -sum_l gamma_l (D lambda_l) .* (D x_l)   (per difference plane),
  dL/db       = sum_l lambda_l.
There is no backpropagation through CG iterations.  Every numeric step runs
in the HIP library (rsr_solve_shift_set, rsr_adjoint); torch supplies memory.

With recycling options (a principal space set for the current weights, the
minimum-residual guess, Ritz vectors, previous corrections) both the forward
and the adjoint solves are recycled: the adjoint systems share the forward's
principal space and Ritz blocks (same matrices B_l), and their local spaces
take the forward correction of the same shift.  The weights are passed to the
library only when they differ from its current ones, since new weights
invalidate the principal space's products A U, E U.
"""
from __future__ import annotations

import torch

from . import rsr


def _set_weights(context: rsr.Context, inst: int, w_h: torch.Tensor, w_v: torch.Tensor):
    """Upload W unless the library already holds it (entries that weigh no difference are ignored)."""
    cur_h, cur_v = context.get_weights(inst)
    if torch.equal(cur_h[:, :-1], w_h[:, :-1]) and torch.equal(cur_v[:-1, :], w_v[:-1, :]):
        return
    context.update_weights(inst, w_h.detach().contiguous(), w_v.detach().contiguous())


class RecycledShiftSolve(torch.autograd.Function):
    """apply(context, gammas[M] (CPU float64), w_h, w_v, b, inst=0, opts=None) -> X [M, ny, nx]."""

    @staticmethod
    def forward(fctx, context: rsr.Context, gammas: torch.Tensor, w_h: torch.Tensor, w_v: torch.Tensor,
                b: torch.Tensor, inst: int = 0, opts: rsr.SolveOptions = None):
        opts = opts or rsr.SolveOptions(tol=1e-12)
        g = [float(v) for v in gammas.detach().cpu().tolist()]
        _set_weights(context, inst, w_h.detach(), w_v.detach())
        ny, nx = context.shapes[inst]
        X = torch.zeros((len(g), ny, nx), dtype=torch.float64, device=b.device)
        rc, st = context.solve(g, b.detach().contiguous(), X, inst=[inst] * len(g), opts=opts)
        if rc != 0:
            raise rsr.RsrError(rc, "forward solve did not converge")
        fctx.context, fctx.inst, fctx.opts, fctx.g = context, inst, opts, g
        fctx.gamma_device = gammas.device
        fctx.save_for_backward(X, w_h, w_v)
        return X

    @staticmethod
    def backward(fctx, gX: torch.Tensor):
        X, w_h, w_v = fctx.saved_tensors
        context = fctx.context
        _set_weights(context, fctx.inst, w_h.detach(), w_v.detach())
        Lam = torch.zeros_like(X)
        rc, dg, dwh, dwv, db, st = context.adjoint(fctx.g, X, gX.contiguous(), Lam, inst=fctx.inst,
                                                  opts=fctx.opts)
        if rc != 0:
            raise rsr.RsrError(rc, "adjoint solve did not converge")
        dgamma = torch.from_numpy(dg).to(fctx.gamma_device)
        return None, dgamma, dwh, dwv, db, None, None
