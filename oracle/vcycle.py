"""Oracle: recursive V-cycle and its transpose (FP64, CPU).

Test infrastructure only (see the package docstring).

Follows the recursive multigrid algorithm of Sec. 3.1.1 (Fig. 2a), started
from z = 0 as a preconditioner: nu_pre smoothing sweeps, residual,
restriction with R = P^T, recursion (or the direct solve on the coarsest
level), prolongation of the correction, nu_post sweeps.

The transposed cycle applies exactly M^-T for the forward cycle's M^-1: the
same recursion on A^T with the adjoint sweep, the pre/post sweep counts
swapped, restriction P^T and prolongation R^T (identical to the forward
transfers because R = P^T), and A_c^-T on the coarsest level.

With the CheapSIMPLE coarse solver (the weak-scaling study's second
variant) the coarsest level runs `coarse_sweeps` sweeps from zero instead of
the direct solve.  k sweeps from zero give I - M_k A = (I - Q^-1 A)^k, whose
transpose is k adjoint sweeps from zero, so the transposed cycle stays exact.
"""
from __future__ import annotations

import numpy as np

from .smoother import (braess_sarazin_sweep, braess_sarazin_sweep_adjoint, cheap_simple_sweep,
                       cheap_simple_sweep_adjoint, cheap_uzawa_sweep, cheap_uzawa_sweep_adjoint)


def _apply_A(L, z, transpose):
    n_u = L.n_u
    zu, zl = z[:n_u], z[n_u:]
    if not transpose:
        return np.concatenate([L.K @ zu + L.G @ zl, L.B @ zu + L.C @ zl])
    return np.concatenate([L.K.T @ zu + L.B.T @ zl, L.G.T @ zu + L.C.T @ zl])


def vcycle(levels, b, opts, level=0, transpose=False):
    """z = M^-1 b (or M^-T b) for the hierarchy starting at `level`."""
    L = levels[level]
    coarsest = level == len(levels) - 1
    if coarsest and opts.coarse_solver != "simple":
        return (L.A_inv.T if transpose else L.A_inv) @ b
    if transpose:
        n_pre, n_post = opts.nu_post, opts.nu_pre
        KT = L.K.T.tocsr()

        def sweep(bb, zz):
            if opts.smoother == "uzawa":
                return cheap_uzawa_sweep_adjoint(L, bb, zz, opts.jacobi_omega, opts.simple_alpha, opts.jacobi_sweeps,
                                                 KT, schur_sweeps=opts.schur_sweeps)
            if opts.smoother == "braess_sarazin":
                return braess_sarazin_sweep_adjoint(L, bb, zz, opts.simple_alpha, opts.schur_sweeps, KT)
            return cheap_simple_sweep_adjoint(L, bb, zz, opts.jacobi_omega, opts.simple_alpha, opts.jacobi_sweeps, KT,
                                              schur_sweeps=opts.schur_sweeps)
    else:
        n_pre, n_post = opts.nu_pre, opts.nu_post

        def sweep(bb, zz):
            if opts.smoother == "uzawa":
                return cheap_uzawa_sweep(L, bb, zz, opts.jacobi_omega, opts.simple_alpha, opts.jacobi_sweeps,
                                         schur_sweeps=opts.schur_sweeps)
            if opts.smoother == "braess_sarazin":
                return braess_sarazin_sweep(L, bb, zz, opts.simple_alpha, opts.schur_sweeps)
            return cheap_simple_sweep(L, bb, zz, opts.jacobi_omega, opts.simple_alpha, opts.jacobi_sweeps,
                                      schur_sweeps=opts.schur_sweeps)

    n_u = L.n_u
    z = np.zeros_like(b)
    if coarsest:
        for _ in range(opts.coarse_sweeps):
            z = sweep(b, z)
        return z
    for _ in range(n_pre):
        z = sweep(b, z)
    r = b - _apply_A(L, z, transpose)
    bc = np.concatenate([L.P_u.T @ r[:n_u], L.P_l.T @ r[n_u:]])
    zc = vcycle(levels, bc, opts, level + 1, transpose)
    nc_u = L.P_u.shape[1]
    z = z + np.concatenate([L.P_u @ zc[:nc_u], L.P_l @ zc[nc_u:]])
    for _ in range(n_post):
        z = sweep(b, z)
    return z
