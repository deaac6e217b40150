"""Mortar matrices D and M for structured interfaces (dual or standard basis).

Input generation only.  The paper fixes the properties used here: with a dual
Lagrange-multiplier basis the biorthogonality condition makes the slave mortar
matrix D diagonal (Sec. 2.2; Sec. 2.3 remark on dual shape functions).  The
formulas for D and M themselves are deferred by the paper to its references,
so the construction below is derived from the definitions:

* slave shape functions N_j, master shape functions N_k^m, dual functions
  psi_j chosen element-wise so that  int psi_j N_k = delta_jk int N_k;
* D_jk = int psi_j N_k  (diagonal, D_jj = int N_j),
* M_jk = int psi_j N_k^m  (segment integration over the union of both
  meshes' break points, two Gauss points per segment: the integrand is
  piecewise quadratic, so this is exact).

For a linear 1D slave element with shape functions N1, N2 the dual pair is
psi1 = 2 N1 - N2, psi2 = 2 N2 - N1.  On a flat, tensor-product 2D face both
psi and N factor over the axes, so the face matrices are Kronecker products
of the 1D ones.

With the standard basis (the weak-scaling study discretises the multipliers
with linear Lagrange polynomials, Sec. 6.2 setup) the multiplier functions
are the slave shape functions themselves: D_jk = int N_j N_k is the
interface mass matrix (not diagonal) and M_jk = int N_j N_k^m.
"""
from __future__ import annotations

import numpy as np

_GP = np.array([-1.0, 1.0]) / np.sqrt(3.0)


def _locate(x_nodes: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Element index e with x_nodes[e] <= x <= x_nodes[e+1]."""
    e = np.searchsorted(x_nodes, x, side="right") - 1
    return np.clip(e, 0, len(x_nodes) - 2)


def mortar_1d(xs: np.ndarray, xm: np.ndarray, weight=None, basis: str = "dual"):
    """1D mortar matrices on a line.

    xs, xm: sorted slave / master node coordinates.
    weight: optional callable w(x) multiplying the integrand (surface
        Jacobian for a curved interface parametrised by x).
    basis: "dual" (psi) or "standard" (N) multiplier functions.
    Returns (D, M (ns, nm)) with D the diagonal (ns,) for the dual basis and
    the full (ns, ns) matrix for the standard basis.
    """
    if basis not in ("dual", "standard"):
        raise ValueError(basis)
    xs = np.asarray(xs, float)
    xm = np.asarray(xm, float)
    lo = max(xs[0], xm[0])
    hi = min(xs[-1], xm[-1])
    brk = np.unique(np.concatenate([xs, xm]))
    brk = brk[(brk >= lo) & (brk <= hi)]
    ns, nm = len(xs), len(xm)
    D = np.zeros(ns) if basis == "dual" else np.zeros((ns, ns))
    M = np.zeros((ns, nm))
    for p, q in zip(brk[:-1], brk[1:]):
        if q <= p:
            continue
        half = 0.5 * (q - p)
        mid = 0.5 * (q + p)
        for g in _GP:
            x = mid + half * g
            w = half * (1.0 if weight is None else float(weight(x)))
            es = int(_locate(xs, np.array([x]))[0])
            t = (x - xs[es]) / (xs[es + 1] - xs[es])
            N1, N2 = 1.0 - t, t
            em = int(_locate(xm, np.array([x]))[0])
            tm = (x - xm[em]) / (xm[em + 1] - xm[em])
            Nm1, Nm2 = 1.0 - tm, tm
            if basis == "dual":
                psi1, psi2 = 2.0 * N1 - N2, 2.0 * N2 - N1
                D[es] += w * psi1 * N1
                D[es + 1] += w * psi2 * N2
            else:
                psi1, psi2 = N1, N2
                D[es, es] += w * N1 * N1
                D[es, es + 1] += w * N1 * N2
                D[es + 1, es] += w * N2 * N1
                D[es + 1, es + 1] += w * N2 * N2
            M[es, em] += w * psi1 * Nm1
            M[es, em + 1] += w * psi1 * Nm2
            M[es + 1, em] += w * psi2 * Nm1
            M[es + 1, em + 1] += w * psi2 * Nm2
    return D, M


def mortar_face(axes_slave, axes_master, weights=None, basis: str = "dual"):
    """Tensor-product face matrices.

    axes_slave / axes_master: list of 1D node-coordinate arrays, x first.
    weights: optional list of per-axis weight callables.
    Face node order is x fastest, so the Kronecker factors run from the last
    axis to the first.
    Returns (D, M) with M dense (n_slave_face, n_master_face) and D the
    diagonal vector (dual basis) or the dense matrix (standard basis).
    """
    Ds, Ms = [], []
    for a, (xs, xm) in enumerate(zip(axes_slave, axes_master)):
        w = None if weights is None else weights[a]
        D1, M1 = mortar_1d(xs, xm, w, basis)
        Ds.append(D1)
        Ms.append(M1)
    D = Ds[-1]
    M = Ms[-1]
    for a in range(len(Ds) - 2, -1, -1):
        D = np.kron(D, Ds[a])
        M = np.kron(M, Ms[a])
    return D, M
