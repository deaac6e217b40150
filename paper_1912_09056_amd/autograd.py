"""Differentiable contact solve: torch.autograd.Function around fgmres_solve.

Forward: x = A^-1 b, A = [[K, G], [B, C]] with the given stored values, by
the block-AMG preconditioned FGMRES.
Backward (hand-written adjoint): A^T lam = dL/dx solved by FGMRES with the
transposed V-cycle on the same hierarchy; dL/db = lam and dL/dA_ij =
-lam_i x_j on the stored entries of each block whose values were passed
(amg_grad_A).  Both solves and the gradient sampling run in the HIP library.

The solver holds one set of level-0 values at a time, so backward first
writes the forward's values back: another forward (or a no-grad solve with
other values) between a forward and its backward then cannot change the
operator the adjoint solves with.
"""
from __future__ import annotations

import torch

from .camg import AMGSolver

_BLOCKS = ("K", "G", "B", "C")


def _load(solver: AMGSolver, vals):
    if any(v is not None for v in vals):
        solver.update_fine_values(*[None if v is None else v.detach() for v in vals])


class ContactSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver: AMGSolver, K_val, b, rtol=1e-10, m=50, G_val=None, B_val=None, C_val=None):
        vals = (K_val, G_val, B_val, C_val)
        _load(solver, vals)
        x, info = solver.solve(b.detach(), rtol=rtol, m=m)
        if not info["converged"]:
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.solver = solver
        ctx.rtol = rtol
        ctx.m = m
        ctx.given = tuple(v is not None for v in vals)
        ctx.save_for_backward(x, *[v for v in vals if v is not None])
        return x

    @staticmethod
    def backward(ctx, gx: torch.Tensor):
        x, *saved = ctx.saved_tensors
        it = iter(saved)
        vals = [next(it) if g else None for g in ctx.given]
        solver = ctx.solver
        # the operator of this forward, whatever values later calls loaded
        _load(solver, vals)
        lam, info = solver.solve(gx.contiguous(), transpose=True, rtol=ctx.rtol, m=ctx.m)
        if not info["converged"]:
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        # input positions of K, G, B, C in forward's signature
        pos = dict(K=1, G=5, B=6, C=7)
        want = [name for name, g in zip(_BLOCKS, ctx.given) if g and ctx.needs_input_grad[pos[name]]]
        grads = solver.grad_A(lam, x, blocks=want) if want else {}
        grad_b = lam if ctx.needs_input_grad[2] else None
        return None, grads.get("K"), grad_b, None, None, grads.get("G"), grads.get("B"), grads.get("C")


def contact_solve(solver: AMGSolver, K_val: torch.Tensor, b: torch.Tensor, rtol: float = 1e-10, m: int = 50,
                  G_val: torch.Tensor = None, B_val: torch.Tensor = None, C_val: torch.Tensor = None):
    """x = A^-1 b, differentiable in b and in the stored values of every block
    passed (K_val may be None to keep the setup values)."""
    return ContactSolve.apply(solver, K_val, b, rtol, m, G_val, B_val, C_val)
