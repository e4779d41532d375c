"""Differentiable smooth objective of the CONCORD / PseudoNet estimator.

    f(Omega; X) = -sum_i log omega_ii + ||Omega X^T||_F^2 / (2n) + lam2/2 ||Omega||_F^2

(the smooth part of the objective in the Obs form, Section 3, with the
half-scaled reading of eq. (1)).  Forward and backward both run in the HIP
library (concord_smooth_value / concord_gradient); Y = Omega X^T is not kept
between them but recomputed in the backward pass.

Gradients returned:
  d/d values : G_ij on the stored entries of Omega, where G is the gradient
               over symmetric matrices (Algorithm 1's gradient step).  Moving
               a symmetric pair (i,j),(j,i) together by h changes f by
               2 h G_ij, and a diagonal entry by h G_ii.
  d/d X      : (Omega Y)^T / n.
"""
from __future__ import annotations

import torch

from ._lib import Solver


class ConcordSmooth(torch.autograd.Function):
    @staticmethod
    def forward(ctx, values, X, rowptr, col, lam2: float, solver: Solver):
        solver.set_data(X.detach())
        solver.set_omega(rowptr, col, values.detach())
        f = solver.smooth_value(lam2)
        ctx.solver = solver
        ctx.lam2 = lam2
        ctx.vdtype = values.dtype
        ctx.xdtype = X.dtype
        ctx.inputs = (values.detach(), X.detach(), rowptr, col)
        token = object()
        solver._autograd_token = token
        ctx.token = token
        return torch.tensor(f, dtype=torch.float64, device=values.device)

    @staticmethod
    def backward(ctx, grad_f):
        solver = ctx.solver
        if getattr(solver, "_autograd_token", None) is not ctx.token:
            # another forward used the handle since: reload this call's inputs
            values, X, rowptr, col = ctx.inputs
            solver.set_data(X)
            solver.set_omega(rowptr, col, values)
            solver._autograd_token = ctx.token
        want_v, want_x = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        dtype = torch.float64 if torch.float64 in (ctx.vdtype, ctx.xdtype) else torch.float32
        dv, dX = ctx.solver.gradient(ctx.lam2, mode="masked", want_omega=want_v, want_x=want_x,
                                     dtype=dtype)
        # the usual incoming gradient is 1: then the library's outputs are returned as
        # they are, without another pass over the n x p d f / d X
        unit = float(grad_f) == 1.0
        g = grad_f.to(dtype)
        gv = gx = None
        if dv is not None:
            gv = (dv if unit else g * dv).to(ctx.vdtype)
        if dX is not None:
            gx = (dX if unit else g * dX).to(ctx.xdtype)
        return gv, gx, None, None, None, None


def concord_smooth(values, X, rowptr, col, lam2: float, solver: Solver):
    """f(Omega; X) with Omega given as CSR (rowptr, col, values); differentiable
    in ``values`` and ``X``.  ``solver`` is an Obs handle of matching p, n."""
    return ConcordSmooth.apply(values, X, rowptr, col, lam2, solver)
