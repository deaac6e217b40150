"""Linear-elastic element matrices for the synthetic two-body contact inputs.

Input generation only: nothing here is part of the multigrid method.  The
paper discretises each body with first-order Lagrange elements (Sec. 2.2,
"Finite element discretization"); the linear, small-strain version used for
the synthetic workloads is the textbook isoparametric Q1 (2D, plane strain)
and hex8 (3D) element with full Gauss quadrature.

Every element matrix is returned split by Lame parameter,
``K_e = lam * K_lam + mu * K_mu``, so per-element material values can be
applied without recomputing shape-function derivatives.

Local node order: bit k of the local index is the offset along axis k
(x fastest), i.e. (0,0,0), (1,0,0), (0,1,0), (1,1,0), (0,0,1), ...
"""
from __future__ import annotations

import itertools

import numpy as np

_GAUSS2 = (np.array([-1.0, 1.0]) / np.sqrt(3.0), np.array([1.0, 1.0]))


def local_offsets(dim: int) -> np.ndarray:
    """(2**dim, dim) array of local node offsets in {0,1}, x fastest."""
    return np.array([[(l >> k) & 1 for k in range(dim)] for l in range(2 ** dim)], dtype=np.int64)


def _shape_grad_ref(xi: np.ndarray) -> np.ndarray:
    """Gradients of the multilinear shape functions on [-1,1]^dim at xi.

    Returns (n_local, dim).
    """
    dim = xi.shape[0]
    offs = local_offsets(dim)
    s = 2.0 * offs - 1.0  # node sign per axis
    g = np.empty((2 ** dim, dim))
    for a in range(dim):
        val = np.full(2 ** dim, 0.5 * s[:, a])
        for b in range(dim):
            if b != a:
                val = val * 0.5 * (1.0 + s[:, b] * xi[b])
        g[:, a] = val
    return g


def _strain_operator(dN: np.ndarray) -> np.ndarray:
    """Voigt strain-displacement matrix from physical shape gradients (n, dim).

    2D rows: exx, eyy, gxy.  3D rows: exx, eyy, ezz, gyz, gxz, gxy.
    Columns follow node-major dof order (node*dim + component).
    """
    n, dim = dN.shape
    if dim == 2:
        Bm = np.zeros((3, 2 * n))
        Bm[0, 0::2] = dN[:, 0]
        Bm[1, 1::2] = dN[:, 1]
        Bm[2, 0::2] = dN[:, 1]
        Bm[2, 1::2] = dN[:, 0]
        return Bm
    Bm = np.zeros((6, 3 * n))
    Bm[0, 0::3] = dN[:, 0]
    Bm[1, 1::3] = dN[:, 1]
    Bm[2, 2::3] = dN[:, 2]
    Bm[3, 1::3] = dN[:, 2]
    Bm[3, 2::3] = dN[:, 1]
    Bm[4, 0::3] = dN[:, 2]
    Bm[4, 2::3] = dN[:, 0]
    Bm[5, 0::3] = dN[:, 1]
    Bm[5, 1::3] = dN[:, 0]
    return Bm


def lame_split_material(dim: int):
    """Voigt material matrices (D_lam, D_mu) with D = lam*D_lam + mu*D_mu.

    2D is plane strain, so the out-of-plane strain is zero and the in-plane
    block of the 3D law applies unchanged.
    """
    if dim == 2:
        m = np.array([1.0, 1.0, 0.0])
        return np.outer(m, m), np.diag([2.0, 2.0, 1.0])
    m = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])
    return np.outer(m, m), np.diag([2.0, 2.0, 2.0, 1.0, 1.0, 1.0])


def element_stiffness_split(coords: np.ndarray):
    """Return (K_lam, K_mu) for one element with nodal coordinates (2**dim, dim)."""
    dim = coords.shape[1]
    D_lam, D_mu = lame_split_material(dim)
    nd = dim * 2 ** dim
    K_lam = np.zeros((nd, nd))
    K_mu = np.zeros((nd, nd))
    pts, wts = _GAUSS2
    for idx in itertools.product(range(2), repeat=dim):
        xi = np.array([pts[i] for i in idx])
        w = np.prod([wts[i] for i in idx])
        g_ref = _shape_grad_ref(xi)
        J = g_ref.T @ coords  # J[a, b] = d x_b / d xi_a
        detJ = np.linalg.det(J)
        if detJ <= 0.0:
            raise ValueError("inverted element")
        dN = np.linalg.solve(J, g_ref.T).T  # physical gradients (n, dim)
        Bm = _strain_operator(dN)
        K_lam += w * detJ * Bm.T @ D_lam @ Bm
        K_mu += w * detJ * Bm.T @ D_mu @ Bm
    return K_lam, K_mu


def box_element_coords(h) -> np.ndarray:
    """Nodal coordinates of an axis-aligned box element with edge lengths h."""
    h = np.asarray(h, dtype=float)
    return local_offsets(len(h)) * h[None, :]


def lame_from_E_nu(E, nu):
    E = np.asarray(E, dtype=float)
    nu = np.asarray(nu, dtype=float)
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu
