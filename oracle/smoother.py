"""Oracle: CheapSIMPLE block smoother and its adjoint (FP64, CPU).

Test infrastructure only (see the package docstring).

One sweep follows the SIMPLE predictor-corrector (Sec. 5.1.3, Alg. 3) in
increment form z <- z + Q^-1 (b - A z) (Sec. 5.1, the common block
relaxation), with the cheap inverses of Sec. 5.2:

  r      = b - A z
  w      = J(r_u)           prediction: damped Jacobi sweeps on K w = r_u
                            from zero
  rt     = r_l - B w        constraint residual after the prediction
  delta  = -rt / S_d        correction with the diagonal Schur approximation
                            S_d = diag(B Atilde^-1 G - C); optionally k
                            undamped Jacobi sweeps on S delta = -rt with
                            that diagonal (from zero) instead
  z_l   += alpha delta
  z_u   += w - alpha Atilde^-1 G delta

Reading of the damping: alpha multiplies the multiplier update and the
back-substitution exactly as Alg. 3 writes them and S is left unscaled (with
the paper's "default" alpha-scaled Schur choice the sweep would not depend on
alpha at all).  With exact inverses and alpha = 1 the constraint rows are
satisfied after one sweep, as the SIMPLE error-matrix discussion states.

The adjoint sweep applies Q^-T for the transposed operator
A^T = [[K^T, B^T], [G^T, C^T]]:

  s      = b - A^T z
  delta  = -(s_l - G^T Atilde^-1 s_u) / S_d
  z_l   += alpha delta
  z_u   += J^T(s_u - alpha B^T delta)

J^T is the same Jacobi polynomial taken with K^T; with Schur sweeps the
division by S_d becomes the same number of Jacobi sweeps on S^T (the
transpose of sum_i (I - D^-1 S)^i D^-1 is sum_i (I - D^-1 S^T)^i D^-1).
"""
from __future__ import annotations

import numpy as np


def jacobi(K, dinv, r, omega, sweeps):
    """sweeps damped-Jacobi steps on K w = r from w = 0."""
    w = np.zeros_like(r)
    for _ in range(sweeps):
        w = w + omega * dinv * (r - K @ w)
    return w


def schur_apply(L, rt, sweeps, transpose=False):
    """Approximate solve of S delta = rt: division by the stored diagonal
    (one sweep) or `sweeps` undamped Jacobi sweeps from zero on S (S^T)."""
    if sweeps <= 1:
        return rt * L.sd_inv
    if transpose:
        if "ST" not in L.extra:
            L.extra["ST"] = L.S.T.tocsr()
        S = L.extra["ST"]
    else:
        S = L.S
    return jacobi(S, L.sd_inv, rt, 1.0, sweeps)


def cheap_simple_sweep(L, b, z, omega, alpha, jac_sweeps=1, predict=None, schur_solve=None, schur_sweeps=1):
    """One sweep.  predict(r_u) and schur_solve(rt) replace the cheap inner
    inverses (Jacobi prediction, diagonal Schur) when given, e.g. by exact
    solves to check the paper's statements about exact SIMPLE."""
    n_u = L.n_u
    zu, zl = z[:n_u], z[n_u:]
    ru = b[:n_u] - (L.K @ zu + L.G @ zl)
    rl = b[n_u:] - (L.B @ zu + L.C @ zl)
    w = jacobi(L.K, L.dinv, ru, omega, jac_sweeps) if predict is None else predict(ru)
    rt = rl - L.B @ w
    delta = -schur_apply(L, rt, schur_sweeps) if schur_solve is None else -schur_solve(rt)
    out = np.empty_like(z)
    out[n_u:] = zl + alpha * delta
    out[:n_u] = zu + w - alpha * L.atilde_inv * (L.G @ delta)
    return out


def cheap_simple_sweep_adjoint(L, b, z, omega, alpha, jac_sweeps=1, KT=None, schur_sweeps=1):
    n_u = L.n_u
    KT = L.K.T.tocsr() if KT is None else KT
    zu, zl = z[:n_u], z[n_u:]
    su = b[:n_u] - (KT @ zu + L.B.T @ zl)
    sl = b[n_u:] - (L.G.T @ zu + L.C.T @ zl)
    delta = -schur_apply(L, sl - L.G.T @ (L.atilde_inv * su), schur_sweeps, transpose=True)
    out = np.empty_like(z)
    out[n_u:] = zl + alpha * delta
    out[:n_u] = zu + jacobi(KT, L.dinv, su - alpha * (L.B.T @ delta), omega, jac_sweeps)
    return out
