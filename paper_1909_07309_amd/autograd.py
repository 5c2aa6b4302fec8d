"""Differentiable space-time heat solve: u = A^{-1} (f - A_{I,0} c0).

Forward: GMRES (right-preconditioned by the fast-diagonalization A-hat^{-1}) on
the kept unknowns, with the initial datum c0 entering through the discrete
lifting of the removed first time function (Section 3.1, non-homogeneous
initial condition).  Backward (adjoint): lambda = A^{-T} g by GMRES with A^T and
A-hat^{-T} (same spatial eigenvectors, transposed time pencil), then
    dL/df = lambda,     dL/dc0 = -A_{I,0}^T lambda.
Every step runs in libstig; PyTorch only carries the tensors and the graph.
"""
from __future__ import annotations

import torch

from .api import Plan


class STIGSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, c0, plan: Plan, a_col, b_col, opts):
        """f: [rhs][t][x_d]..[x_1] float64 (HIP); c0: [rhs][x_d]..[x_1] or None."""
        rhs = f.contiguous()
        if c0 is not None:
            # f - A_{I,0} c0 in one library call
            rhs = plan.lift_apply(a_col, b_col, c0.contiguous(), f=rhs).view_as(rhs)
        u, info = plan.gmres_solve(rhs, **opts)
        ctx.plan, ctx.a_col, ctx.b_col, ctx.opts = plan, a_col, b_col, opts
        ctx.has_c0 = c0 is not None
        ctx.info = info
        return u

    @staticmethod
    def backward(ctx, grad_u):
        plan = ctx.plan
        lam, _ = plan.gmres_solve(grad_u.contiguous(), transpose=True, **ctx.opts)
        grad_c0 = None
        if ctx.has_c0:
            grad_c0 = plan.lift_adjoint(ctx.a_col, ctx.b_col, lam)
        return lam.view_as(grad_u), grad_c0, None, None, None, None


def solve(plan: Plan, f, c0=None, lift_cols=None, **opts):
    """u(f, c0) with gradients w.r.t. f and c0.  lift_cols = (a_col, b_col) as in
    Plan.lift_apply (the removed first time function's columns of W_t and M_t)."""
    a_col, b_col = lift_cols if lift_cols is not None else (None, None)
    if c0 is not None and lift_cols is None:
        raise ValueError("an initial datum needs the lifting columns")
    return STIGSolve.apply(f, c0, plan, a_col, b_col, opts)
