"""Differentiable contact solve: torch.autograd.Function around fgmres_solve.

Forward: x = A(K)^-1 b with the block-AMG preconditioned FGMRES.
Backward (hand-written adjoint): A^T lam = dL/dx solved by FGMRES with the
transposed V-cycle on the same hierarchy; dL/db = lam and
dL/dK_ij = -lam_i x_j on K's stored entries (amg_grad_K).  Both solves and
the gradient sampling run in the HIP library.

The solver holds one set of level-0 values at a time, so backward first
writes the forward's K values back: another forward (or a no-grad solve with
other values) between a forward and its backward then cannot change the
operator the adjoint solves with.
"""
from __future__ import annotations

import torch

from .camg import AMGSolver


class ContactSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver: AMGSolver, K_val: torch.Tensor, b: torch.Tensor, rtol: float = 1e-10, m: int = 50):
        if K_val is not None:
            solver.update_fine_values(K_val=K_val.detach())
        x, info = solver.solve(b.detach(), rtol=rtol, m=m)
        if not info["converged"]:
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.solver = solver
        ctx.rtol = rtol
        ctx.m = m
        ctx.has_K = K_val is not None
        if K_val is not None:
            ctx.save_for_backward(x, K_val)
        else:
            ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx: torch.Tensor):
        saved = ctx.saved_tensors
        x = saved[0]
        solver = ctx.solver
        if ctx.has_K:
            # the operator of this forward, whatever values later calls loaded
            solver.update_fine_values(K_val=saved[1].detach())
        lam, info = solver.solve(gx.contiguous(), transpose=True, rtol=ctx.rtol, m=ctx.m)
        if not info["converged"]:
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        grad_K = solver.grad_K(lam, x) if ctx.needs_input_grad[1] else None
        grad_b = lam if ctx.needs_input_grad[2] else None
        return None, grad_K, grad_b, None, None


def contact_solve(solver: AMGSolver, K_val: torch.Tensor, b: torch.Tensor, rtol: float = 1e-10, m: int = 50):
    return ContactSolve.apply(solver, K_val, b, rtol, m)
