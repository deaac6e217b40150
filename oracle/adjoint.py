"""Oracle: forward solve, adjoint solve and gradients (FP64, CPU).

Test infrastructure only (see the package docstring).

For x = A^-1 b and a scalar loss L(x) with g = dL/dx, the adjoint solve
A^T lam = g gives dL/db = lam and dL/dA_ij = -lam_i x_j; restricted to the
stored entries of K this is the gradient with respect to K's nonzeros.  The
adjoint system is solved with FGMRES preconditioned by the transposed
V-cycle on the same hierarchy.
"""
from __future__ import annotations

import numpy as np

from .fgmres import fgmres
from .vcycle import vcycle, _apply_A


def solve(levels, opts, b, transpose=False, x0=None, m=50, rtol=1e-8, max_iters=1000, fixed_iters=None):
    L0 = levels[0]
    return fgmres(
        lambda v: _apply_A(L0, v, transpose),
        lambda v: vcycle(levels, v, opts, 0, transpose),
        b,
        x0=x0,
        m=m,
        rtol=rtol,
        max_iters=max_iters,
        fixed_iters=fixed_iters,
    )


def grad_K_values(K, lam_u, x_u):
    """-lam_i x_j for every stored entry (i, j) of K, in K's storage order."""
    rows = np.repeat(np.arange(K.shape[0]), np.diff(K.indptr))
    return -lam_u[rows] * x_u[K.indices]


def solve_with_adjoint(levels, opts, b, dLdx_fn, rtol=1e-10, m=50):
    """Returns (x, lam, grad_b, grad_Kvals)."""
    fwd = solve(levels, opts, b, rtol=rtol, m=m)
    g = dLdx_fn(fwd.x)
    adj = solve(levels, opts, g, transpose=True, rtol=rtol, m=m)
    n_u = levels[0].n_u
    return fwd.x, adj.x, adj.x, grad_K_values(levels[0].K, adj.x[:n_u], fwd.x[:n_u])
