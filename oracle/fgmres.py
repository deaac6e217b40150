"""Oracle: right-preconditioned flexible GMRES(m) with CGS2 (FP64, CPU).

Test infrastructure only (see the package docstring).

The paper solves with preconditioned GMRES, one V-cycle per iteration, and
stops when the full residual has dropped by 1e-8 relative to the initial one
(Sec. 3 introduction; stopping criterion of the numerical examples).  Its
GMRES variant is not stated; this oracle takes the flexible right-
preconditioned form (the preconditioned directions z_j are kept), classical
Gram-Schmidt with one full re-orthogonalisation pass, Givens rotations on
the Hessenberg matrix, and restarts every m iterations.  The estimate
|g_{j+1}| drives the inner stop; convergence is only reported once the true
residual ||b - A x|| passes as well.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class FGMRESResult:
    x: np.ndarray
    iters: int
    restarts: int
    converged: bool
    rel_res_est: float
    rel_res_true: float
    history: list


def _givens(a, b):
    d = np.hypot(a, b)
    if d == 0.0:
        return 1.0, 0.0, 0.0
    return a / d, b / d, d


def fgmres(apply_A, apply_M, b, x0=None, m=50, rtol=1e-8, max_iters=1000, fixed_iters=None):
    """Solve A x = b.

    apply_A / apply_M: callables (vector -> vector).
    fixed_iters: if given, run exactly that many iterations (no tolerance
        stop, restarts every m) -- used to compare two implementations.
    Returns FGMRESResult.
    """
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=float)
    r = b - apply_A(x)
    r0 = np.linalg.norm(r)
    history = [1.0]
    total = 0
    restarts = 0
    est = 1.0
    limit = fixed_iters if fixed_iters is not None else max_iters
    if r0 == 0.0:
        return FGMRESResult(x, 0, 0, True, 0.0, 0.0, history)
    while True:
        beta = np.linalg.norm(r)
        if fixed_iters is None and beta <= rtol * r0:
            break
        if total >= limit:
            break
        V = np.zeros((n, m + 1))
        Z = np.zeros((n, m))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[:, 0] = r / beta
        k = 0
        for j in range(m):
            Z[:, j] = apply_M(V[:, j])
            w = apply_A(Z[:, j])
            h = V[:, : j + 1].T @ w
            w = w - V[:, : j + 1] @ h
            h2 = V[:, : j + 1].T @ w
            w = w - V[:, : j + 1] @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            H[: j + 1, j] = h
            H[j + 1, j] = hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j], H[j, j] = _givens(H[j, j], H[j + 1, j])
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            k = j + 1
            est = abs(g[j + 1]) / r0
            history.append(est)
            if hn == 0.0:
                break
            V[:, j + 1] = w / hn
            if fixed_iters is None and abs(g[j + 1]) <= rtol * r0:
                break
            if total >= limit:
                break
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:, :k] @ y
        r = b - apply_A(x)
        if total >= limit:
            break
        restarts += 1
    true = np.linalg.norm(r) / r0
    converged = true <= rtol if fixed_iters is None else False
    return FGMRESResult(x, total, restarts, converged, est, true, history)
