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
transpose of sum_i (I - D^-1 S)^i D^-1 is sum_i (I - D^-T S^T)^i D^-T).

Block option: D is the block diagonal of S over multiplier nodes (the d
Cartesian components of one slave node, or of one coarse multiplier
aggregate), so the correction solves a small dense system per node instead
of dividing per row; the transposed sweep relaxes S^T with the transposed
blocks.
"""
from __future__ import annotations

import numpy as np


def jacobi(K, dinv, r, omega, sweeps, transpose=False):
    """sweeps damped-Jacobi steps on K w = r from w = 0; dinv is the inverse
    relaxation diagonal, or a (nb, bs, bs) stack of inverse nodal blocks
    (block Jacobi; applied transposed with transpose, for K^T)."""
    w = np.zeros_like(r)
    for _ in range(sweeps):
        if np.ndim(dinv) == 1:
            w = w + omega * dinv * (r - K @ w)
        else:
            w = w + omega * node_block_solve(dinv, r - K @ w, transpose)
    return w


def lumped(L, v, scale=1.0, transpose=False):
    """scale * Atilde^-1 v with the level's lumping: the diagonal, or the
    nodal blocks (transposed with transpose)."""
    if np.ndim(L.atilde_inv) == 1:
        return scale * L.atilde_inv * v
    return scale * node_block_solve(L.atilde_inv, v, transpose)


def node_block_solve(blk_inv, r, transpose=False):
    """Per multiplier node j (bs consecutive dofs): blk_inv[j] @ r_j, or
    blk_inv[j]^T @ r_j with transpose (the inverse of the transposed block)."""
    nb, bs, _ = blk_inv.shape
    R = np.asarray(r).reshape(nb, bs)
    # out_j[a] = sum_b M_j[a, b] r_j[b]   (M_j[b, a] with transpose)
    return np.einsum("nba,nb->na" if transpose else "nab,nb->na", blk_inv, R).reshape(-1)


def _schur_relax(S_of, d_inv, blk_inv, rt, sweeps, transpose):
    """`sweeps` undamped Jacobi sweeps from zero on S delta = rt (S^T with
    transpose), relaxing with the diagonal d_inv or, when blk_inv is given,
    with the nodal diagonal blocks (block Jacobi); one sweep is the division
    (block solve) alone."""
    if blk_inv is not None:
        relax = lambda v: node_block_solve(blk_inv, v, transpose)  # noqa: E731
    else:
        relax = lambda v: v * d_inv  # noqa: E731
    if sweeps <= 1:
        return relax(rt)
    S = S_of()
    x = np.zeros_like(rt)
    for _ in range(sweeps):
        x = x + relax(rt - S @ x)
    return x


def schur_apply(L, rt, sweeps, transpose=False):
    """Approximate solve of S delta = rt: division by the stored diagonal
    (by the nodal blocks with the block option) for one sweep, else `sweeps`
    undamped (block) Jacobi sweeps from zero on S (S^T)."""

    def S_of():
        if not transpose:
            return L.S
        if "ST" not in L.extra:
            L.extra["ST"] = L.S.T.tocsr()
        return L.extra["ST"]

    return _schur_relax(S_of, L.sd_inv, L.extra.get("sb_inv"), rt, sweeps, transpose)


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
    out[:n_u] = zu + w - lumped(L, L.G @ delta, alpha)
    return out


def cheap_uzawa_sweep(L, b, z, omega, alpha, jac_sweeps=1, schur_sweeps=1, predict=None, schur_solve=None):
    """One inexact Uzawa sweep (Sec. 5.1.1, Alg. 2) with the cheap inverses:
    prediction w = J(r_u) (Jacobi sweeps on K), multiplier increment
    delta = -S^-1 (r_l - B w) with the SIMPLE Schur approximation
    S = B Atilde^-1 G - C, both updates damped by alpha and no
    back-substitution into the displacements (the one-way coupling of the
    Uzawa matrix).  predict / schur_solve replace the cheap inverses when
    given (exact solves for the paper's error-matrix statement)."""
    n_u = L.n_u
    zu, zl = z[:n_u], z[n_u:]
    ru = b[:n_u] - (L.K @ zu + L.G @ zl)
    rl = b[n_u:] - (L.B @ zu + L.C @ zl)
    w = jacobi(L.K, L.dinv, ru, omega, jac_sweeps) if predict is None else predict(ru)
    rt = rl - L.B @ w
    delta = -schur_apply(L, rt, schur_sweeps) if schur_solve is None else -schur_solve(rt)
    out = np.empty_like(z)
    out[:n_u] = zu + alpha * w
    out[n_u:] = zl + alpha * delta
    return out


def cheap_uzawa_sweep_adjoint(L, b, z, omega, alpha, jac_sweeps=1, KT=None, schur_sweeps=1):
    """Transpose of the Uzawa sweep map: delta = -S^-T s_l,
    z_l += alpha delta, z_u += alpha J^T (s_u - B^T delta)."""
    n_u = L.n_u
    KT = L.K.T.tocsr() if KT is None else KT
    zu, zl = z[:n_u], z[n_u:]
    su = b[:n_u] - (KT @ zu + L.B.T @ zl)
    sl = b[n_u:] - (L.G.T @ zu + L.C.T @ zl)
    delta = -schur_apply(L, sl, schur_sweeps, transpose=True)
    out = np.empty_like(z)
    out[n_u:] = zl + alpha * delta
    out[:n_u] = zu + alpha * jacobi(KT, L.dinv, su - L.B.T @ delta, omega, jac_sweeps, transpose=True)
    return out


def braess_sarazin_sweep(L, b, z, alpha, schur_sweeps=1, schur_solve=None):
    """One cheap Braess-Sarazin sweep (Sec. 5.1.2, Alg. 3) with the damping
    alpha and the easy-to-invert Ahat = Atilde:
      u_half = u + Ahat^-1 r_u / alpha
      delta  = -S_a^-1 (b_l - B u_half - C lam),  S_a = B Ahat^-1 G / alpha - C
      lam   += delta,  u = u_half - Ahat^-1 G delta / alpha.
    S_a's data (diagonal, optional matrix) is kept in L.extra; schur_solve
    replaces the cheap Schur inverse when given."""
    n_u = L.n_u
    zu, zl = z[:n_u], z[n_u:]
    ru = b[:n_u] - (L.K @ zu + L.G @ zl)
    u_half = zu + lumped(L, ru) / alpha
    rt = b[n_u:] - (L.B @ u_half + L.C @ zl)
    delta = -_bs_schur(L, rt, schur_sweeps, False) if schur_solve is None else -schur_solve(rt)
    out = np.empty_like(z)
    out[n_u:] = zl + delta
    out[:n_u] = u_half - lumped(L, L.G @ delta) / alpha
    return out


def braess_sarazin_sweep_adjoint(L, b, z, alpha, schur_sweeps=1, KT=None):
    """Transpose of the Braess-Sarazin sweep map:
    delta = -S_a^-T (s_l - G^T Ahat^-1 s_u / alpha), lam += delta,
    u += Ahat^-1 (s_u - B^T delta) / alpha."""
    n_u = L.n_u
    KT = L.K.T.tocsr() if KT is None else KT
    zu, zl = z[:n_u], z[n_u:]
    su = b[:n_u] - (KT @ zu + L.B.T @ zl)
    sl = b[n_u:] - (L.G.T @ zu + L.C.T @ zl)
    delta = -_bs_schur(L, sl - L.G.T @ lumped(L, su, transpose=True) / alpha, schur_sweeps, True)
    out = np.empty_like(z)
    out[n_u:] = zl + delta
    out[:n_u] = zu + lumped(L, su - L.B.T @ delta, transpose=True) / alpha
    return out


def _bs_schur(L, rt, sweeps, transpose):
    def S_of():
        if not transpose:
            return L.extra["bs_S"]
        if "bs_ST" not in L.extra:
            L.extra["bs_ST"] = L.extra["bs_S"].T.tocsr()
        return L.extra["bs_ST"]

    return _schur_relax(S_of, L.extra.get("bs_sd_inv"), L.extra.get("bs_sb_inv"), rt, sweeps, transpose)


def cheap_simple_sweep_adjoint(L, b, z, omega, alpha, jac_sweeps=1, KT=None, schur_sweeps=1):
    n_u = L.n_u
    KT = L.K.T.tocsr() if KT is None else KT
    zu, zl = z[:n_u], z[n_u:]
    su = b[:n_u] - (KT @ zu + L.B.T @ zl)
    sl = b[n_u:] - (L.G.T @ zu + L.C.T @ zl)
    delta = -schur_apply(L, sl - L.G.T @ lumped(L, su, transpose=True), schur_sweeps, transpose=True)
    out = np.empty_like(z)
    out[n_u:] = zl + alpha * delta
    out[:n_u] = zu + jacobi(KT, L.dinv, su - alpha * (L.B.T @ delta), omega, jac_sweeps, transpose=True)
    return out
