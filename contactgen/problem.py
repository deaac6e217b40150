"""Seeded synthetic two-body mortar-contact problems.

Input generation only: this module builds the linear system the solver is
given and holds none of the multigrid method's arithmetic.  It is shared by
the CPU oracle (tests) and by the GPU library's callers (tests, bench).

The system is the paper's compact saddle-point form (Sec. 2.3, the 2x2
dashed block system and its short notation)

    [ K   G ] [u]   [f]
    [ B   C ] [l] = [g]

with G = C1^T (upper-right coupling), B = C2 (constraint rows) and C = -Z.
The synthetic instance is linear elasticity of two structured blocks glued by
frictionless contact in which every slave node is active:

* slave body on top, master body below, flat (or smoothly curved) interface;
* dual mortar basis, so D is diagonal (Sec. 2.2), or optionally the standard
  basis of the weak-scaling study (D the interface mass matrix); multipliers
  are Cartesian, d per slave interface node (Sec. 2.3 remark on the
  Cartesian frame);
* G = [D; -M^T] (x) I_d on slave / master interface rows;
* constraint row of slave node j: the normal slot holds n_j^T (x) [D_j, -M_j]
  (weighted-gap linearisation); the tangential slots hold tau_a^T acting on
  lambda_j with a zero B row (frictionless sliding, identity-like rows);
* master bottom face clamped, slave top face on rollers (tangential
  components fixed) carrying a uniform normal traction.  Dirichlet dofs are
  kept as identity rows with zeroed row and column.

Node numbering: slave body first, then master; each body lexicographic with x
fastest; d dofs per node contiguous.  Multiplier pseudo-node j belongs to the
j-th slave interface node in the same lexicographic order.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

from .fe import box_element_coords, element_stiffness_split, lame_from_E_nu, local_offsets
from .mortar import mortar_face


@dataclass
class ContactProblem:
    dim: int
    K: sp.csr_matrix
    G: sp.csr_matrix
    B: sp.csr_matrix
    C: sp.csr_matrix
    b: np.ndarray
    slave_dofs: np.ndarray
    master_dofs: np.ndarray
    lm_node: np.ndarray
    nullspace: np.ndarray
    coords: np.ndarray
    dirichlet: np.ndarray
    top_dofs: np.ndarray
    info: dict = field(default_factory=dict)

    @property
    def n_u(self) -> int:
        return self.K.shape[0]

    @property
    def n_lam(self) -> int:
        return self.C.shape[0]

    @property
    def n(self) -> int:
        return self.n_u + self.n_lam

    def full_matrix(self) -> sp.csr_matrix:
        return sp.bmat([[self.K, self.G], [self.B, self.C]], format="csr")


# ----------------------------------------------------------------------------
# structured body assembly


def _grid_coords(nelem, origin, length):
    """Per-axis node coordinates of a uniform structured grid."""
    return [origin[a] + length[a] * np.arange(nelem[a] + 1) / nelem[a] for a in range(len(nelem))]


def _assemble_body(nelem, axes, lam_e, mu_e, Klam, Kmu):
    """CSR stiffness of one structured body, rows/cols sorted.

    nelem: elements per axis (x first).  lam_e / mu_e: per-element Lame
    parameters, shape reversed-axis (z, y, x) grid.  Klam / Kmu: element
    matrices, broadcastable to (..., nd, nd) over the reversed element grid.
    """
    dim = len(nelem)
    nn = [n + 1 for n in nelem]
    offs = local_offsets(dim)
    n_nodes = int(np.prod(nn))
    n_off = 3 ** dim
    blocks = np.zeros(tuple(reversed(nn)) + (n_off, dim, dim))
    for li in range(2 ** dim):
        for lj in range(2 ** dim):
            d = offs[lj] - offs[li]
            o = int(sum((d[k] + 1) * 3 ** k for k in range(dim)))
            kl = Klam[..., li * dim:(li + 1) * dim, lj * dim:(lj + 1) * dim]
            km = Kmu[..., li * dim:(li + 1) * dim, lj * dim:(lj + 1) * dim]
            contrib = lam_e[..., None, None] * kl + mu_e[..., None, None] * km
            sl = tuple(slice(offs[li][k], offs[li][k] + nelem[k]) for k in reversed(range(dim)))
            blocks[sl + (o,)] += contrib
    blocks = blocks.reshape(n_nodes, n_off, dim, dim)
    # neighbour validity and linear index for each offset
    idx = np.indices(tuple(reversed(nn))).reshape(dim, -1)[::-1]  # idx[k] = coordinate along axis k
    valid = np.ones((n_nodes, n_off), dtype=bool)
    nbr = np.zeros((n_nodes, n_off), dtype=np.int64)
    stride = [int(np.prod(nn[:k])) for k in range(dim)]
    for o in range(n_off):
        dvec = [(o // 3 ** k) % 3 - 1 for k in range(dim)]
        lin = np.arange(n_nodes, dtype=np.int64)
        for k in range(dim):
            c = idx[k] + dvec[k]
            valid[:, o] &= (c >= 0) & (c < nn[k])
            lin = lin + dvec[k] * stride[k]
        nbr[:, o] = lin
    # exact symmetry: the loop above reaches block (i, j) and block (j, i)^T
    # through different element orders, so they differ by rounding; both
    # become their mean (offset o and n_off - 1 - o are mirrors)
    sym = np.empty_like(blocks)
    for o in range(n_off):
        v = valid[:, o]
        mirror = np.swapaxes(blocks[nbr[v, o], n_off - 1 - o], -1, -2)
        sym[v, o] = (blocks[v, o] + mirror) * 0.5
        sym[~v, o] = 0.0
    blocks = sym
    del sym
    # row (node, a) holds, for each valid offset o (increasing column), d columns
    vals = np.transpose(blocks, (0, 2, 1, 3))  # node, a, o, b
    mask = np.broadcast_to(valid[:, None, :, None], vals.shape)
    cols = nbr[:, None, :, None] * dim + np.arange(dim)[None, None, None, :]
    cols = np.broadcast_to(cols, vals.shape)
    data = vals[mask]
    indices = cols[mask]
    counts = np.repeat(valid.sum(axis=1) * dim, dim)
    indptr = np.zeros(n_nodes * dim + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    return sp.csr_matrix((data, indices, indptr), shape=(n_nodes * dim, n_nodes * dim))


def exact_symmetric(K: sp.csr_matrix) -> sp.csr_matrix:
    """(K + K^T) / 2, which equals its transpose bit for bit.

    The stiffness matrix is symmetric, but the floating-point sums of the
    element contributions reach K_ij and K_ji in different orders: mirrored
    entries differ by a few units in the last place, and a coupling that
    cancels may come out as an exact zero on one side only.  K_ij + K_ji is
    the same sum for both entries and the halving is exact, so the mean is
    symmetric in value and pattern (entries that are exact zeros dropped,
    indices sorted)."""
    K = sp.csr_matrix(K)
    S = (K + K.T.tocsr()).tocsr()
    S.data *= 0.5
    S.eliminate_zeros()
    S.sort_indices()
    return S


def _element_shapes(nelem, axes, shift):
    """Element matrices (Klam, Kmu) for every distinct element shape.

    Without a shift every element is the same box.  With a curved shift
    z += shift(x, z) the shape varies with the x and z element indices only.
    """
    dim = len(nelem)
    if shift is None:
        h = [axes[a][1] - axes[a][0] for a in range(dim)]
        Kl, Km = element_stiffness_split(box_element_coords(h))
        shp = (1,) * dim + Kl.shape
        return Kl.reshape(shp), Km.reshape(shp)
    assert dim == 3
    nex, ney, nez = nelem
    nd = 24
    Kl = np.zeros((nez, 1, nex, nd, nd))
    Km = np.zeros((nez, 1, nex, nd, nd))
    offs = local_offsets(3)
    for ez in range(nez):
        for ex in range(nex):
            xc = axes[0][ex + offs[:, 0]]
            yc = axes[1][offs[:, 1]]
            zc = axes[2][ez + offs[:, 2]]
            zc = zc + shift(xc, zc)
            kl, km = element_stiffness_split(np.stack([xc, yc, zc], axis=1))
            Kl[ez, 0, ex] = kl
            Km[ez, 0, ex] = km
    return Kl, Km


def _face_weights(axes_face):
    """Trapezoid weights int N_j over a flat structured face, x fastest."""
    w = None
    for xs in axes_face:
        h = np.diff(xs)
        w1 = np.zeros(len(xs))
        w1[:-1] += 0.5 * h
        w1[1:] += 0.5 * h
        w = w1 if w is None else np.kron(w1, w)
    return w


# ----------------------------------------------------------------------------
# problem builder


def make_contact_problem(
    dim: int,
    slave_elems,
    master_elems,
    slave_box=None,
    master_box=None,
    E_sigma: float = 0.0,
    nu=0.3,
    traction: float = -0.01,
    curve_amp: float = 0.0,
    top_bc: str = "roller",
    seed: int = 0,
    rhs: str = "load",
    lm_basis: str = "dual",
    E: float = 1.0,
    penetration: float = 0.0,
) -> ContactProblem:
    """Build a two-block contact problem (see module docstring).

    slave_box / master_box: (origin, lengths); defaults are the unit box
    [0,1]^dim for the slave and the unit box shifted by -1 along the last
    axis for the master, meeting at the plane x_dim = 0.
    E_sigma: sigma of a lognormal(0, sigma) per-element Young's modulus
        (0 means E = 1 everywhere).
    nu: Poisson ratio, or (lo, hi) for a per-element uniform draw.
    curve_amp: amplitude a of a curved interface x_dim = a sin(2 pi x)
        (3D only); the shift blends linearly to zero at the far faces.
    top_bc: slave top face condition: "roller" fixes the tangential
        components, "clamped" all components (then K alone is nonsingular),
        "free" none (the slave body can slide and the operator is singular).
    rhs: "load" (consistent traction forces), "random" (seeded U(-1,1)) or
        "gap": no load; the blocks overlap by `penetration` along the
        interface normal, so each normal constraint row asks
        n_j . (D u_s - M u_m)_j = penetration * sum_k D_jk (the weighted gap
        g~_j = int N_j g0 with g0 = -penetration, moved to the right-hand
        side: the slave moves away from the master by the overlap).
    lm_basis: "dual" (diagonal D) or "standard" (D = interface mass matrix).
    E: Young's modulus scale (times the lognormal factor when E_sigma > 0).
    """
    slave_elems = list(slave_elems)
    master_elems = list(master_elems)
    assert len(slave_elems) == dim and len(master_elems) == dim
    if slave_box is None:
        slave_box = ([0.0] * dim, [1.0] * dim)
    if master_box is None:
        master_box = ([0.0] * (dim - 1) + [-1.0], [1.0] * dim)
    rng = np.random.default_rng(seed)
    n_el_s = int(np.prod(slave_elems))
    n_el_m = int(np.prod(master_elems))
    if E_sigma > 0.0:
        Ee = E * rng.lognormal(0.0, E_sigma, n_el_s + n_el_m)
    else:
        Ee = np.full(n_el_s + n_el_m, float(E))
    if isinstance(nu, (tuple, list)):
        nus = rng.uniform(nu[0], nu[1], n_el_s + n_el_m)
    else:
        nus = np.full(n_el_s + n_el_m, float(nu))
    lam, mu = lame_from_E_nu(Ee, nus)

    axes_s = _grid_coords(slave_elems, *slave_box)
    axes_m = _grid_coords(master_elems, *master_box)
    if curve_amp != 0.0:
        assert dim == 3
        z_top = slave_box[0][2] + slave_box[1][2]
        z_bot = master_box[0][2]

        def f(x):
            return curve_amp * np.sin(2.0 * np.pi * x)

        def fprime(x):
            return curve_amp * 2.0 * np.pi * np.cos(2.0 * np.pi * x)

        def shift_s(x, z):
            return f(x) * (z_top - z) / z_top

        def shift_m(x, z):
            return f(x) * (z - z_bot) / (-z_bot)
    else:
        f = fprime = shift_s = shift_m = None

    Ks = []
    for nel, axes, sl, shift in (
        (slave_elems, axes_s, slice(0, n_el_s), shift_s),
        (master_elems, axes_m, slice(n_el_s, n_el_s + n_el_m), shift_m),
    ):
        Kl, Km = _element_shapes(nel, axes, shift)
        grid = tuple(reversed(nel))
        Ks.append(_assemble_body(nel, axes, lam[sl].reshape(grid), mu[sl].reshape(grid), Kl, Km))
    K = sp.block_diag(Ks, format="csr")

    nn_s = [n + 1 for n in slave_elems]
    nn_m = [n + 1 for n in master_elems]
    n_nodes_s = int(np.prod(nn_s))
    n_nodes_m = int(np.prod(nn_m))
    n_u = dim * (n_nodes_s + n_nodes_m)

    # node coordinates (physical)
    def body_coords(axes, shift):
        mesh = np.meshgrid(*axes, indexing="ij")
        pts = np.stack([m.transpose(tuple(reversed(range(dim)))).ravel() for m in mesh], axis=1)
        if shift is not None:
            pts[:, 2] = pts[:, 2] + shift(pts[:, 0], pts[:, 2])
        return pts

    coords = np.vstack([body_coords(axes_s, shift_s), body_coords(axes_m, shift_m)])

    def layer(nn, k_axis, k_val, offset):
        idx = np.indices(tuple(reversed(nn))).reshape(dim, -1)[::-1]
        return offset + np.nonzero(idx[k_axis] == k_val)[0]

    last = dim - 1
    slave_iface_nodes = layer(nn_s, last, 0, 0)
    slave_top_nodes = layer(nn_s, last, nn_s[last] - 1, 0)
    master_iface_nodes = layer(nn_m, last, nn_m[last] - 1, n_nodes_s)
    master_bottom_nodes = layer(nn_m, last, 0, n_nodes_s)

    dirichlet = np.zeros(n_u, dtype=bool)
    for c in range(dim):
        dirichlet[master_bottom_nodes * dim + c] = True
    if top_bc not in ("roller", "clamped", "free"):
        raise ValueError(top_bc)
    n_fix = {"roller": dim - 1, "clamped": dim, "free": 0}[top_bc]
    for c in range(n_fix):
        dirichlet[slave_top_nodes * dim + c] = True

    # mortar matrices on the interface (parameter plane of the first dim-1 axes)
    face_s = [axes_s[a] for a in range(dim - 1)]
    face_m = [axes_m[a] for a in range(dim - 1)]
    weights = None
    if fprime is not None:
        weights = [lambda x: np.sqrt(1.0 + fprime(x) ** 2), None]
    Dm, Mf = mortar_face(face_s, face_m, weights, lm_basis)
    ns = len(slave_iface_nodes)
    nm = len(master_iface_nodes)
    Dsp = sp.diags(Dm).tocsr() if Dm.ndim == 1 else sp.csr_matrix(Dm)
    Dsp.eliminate_zeros()
    Dcoo = Dsp.tocoo()
    D_rowsum = np.asarray(Dsp.sum(axis=1)).ravel()
    assert Dsp.shape == (ns, ns) and Mf.shape == (ns, nm)
    n_lam = dim * ns

    # normals / tangents per slave interface node (the +x_dim-facing normal)
    if fprime is None:
        normals = np.zeros((ns, dim))
        normals[:, last] = 1.0
        tangents = [np.zeros((ns, dim)) for _ in range(dim - 1)]
        for a in range(dim - 1):
            tangents[a][:, a] = 1.0
    else:
        xj = coords[slave_iface_nodes, 0]
        fp = fprime(xj)
        s = np.sqrt(1.0 + fp ** 2)
        normals = np.stack([-fp / s, np.zeros(ns), 1.0 / s], axis=1)
        t1 = np.stack([1.0 / s, np.zeros(ns), fp / s], axis=1)
        t2 = np.tile(np.array([0.0, 1.0, 0.0]), (ns, 1))
        tangents = [t1, t2]

    Msp = sp.csr_matrix(Mf)
    Msp.eliminate_zeros()
    Mcoo = Msp.tocoo()

    # G = [D; -M^T] (x) I_d
    g_rows, g_cols, g_vals = [], [], []
    for c in range(dim):
        g_rows.append(slave_iface_nodes[Dcoo.col] * dim + c)
        g_cols.append(Dcoo.row * dim + c)
        g_vals.append(Dcoo.data)
        g_rows.append(master_iface_nodes[Mcoo.col] * dim + c)
        g_cols.append(Mcoo.row * dim + c)
        g_vals.append(-Mcoo.data)
    G = sp.csr_matrix(
        (np.concatenate(g_vals), (np.concatenate(g_rows), np.concatenate(g_cols))), shape=(n_u, n_lam)
    )

    # B: normal rows n_j^T (x) [D_j, -M_j] in slot dim-1; C: tangential rows
    b_rows, b_cols, b_vals = [], [], []
    for c in range(dim):
        nc = normals[:, c]
        b_rows.append(Dcoo.row * dim + last)
        b_cols.append(slave_iface_nodes[Dcoo.col] * dim + c)
        b_vals.append(nc[Dcoo.row] * Dcoo.data)
        b_rows.append(Mcoo.row * dim + last)
        b_cols.append(master_iface_nodes[Mcoo.col] * dim + c)
        b_vals.append(-nc[Mcoo.row] * Mcoo.data)
    Bm = sp.csr_matrix(
        (np.concatenate(b_vals), (np.concatenate(b_rows), np.concatenate(b_cols))), shape=(n_lam, n_u)
    )
    c_rows, c_cols, c_vals = [], [], []
    for a in range(dim - 1):
        for c in range(dim):
            c_rows.append(np.arange(ns) * dim + a)
            c_cols.append(np.arange(ns) * dim + c)
            c_vals.append(tangents[a][:, c])
    Cm = sp.csr_matrix(
        (np.concatenate(c_vals), (np.concatenate(c_rows), np.concatenate(c_cols))), shape=(n_lam, n_lam)
    )

    # Dirichlet: identity rows, zeroed rows and columns (K), zero G rows / B cols
    K = K.tocsr()
    rows = np.repeat(np.arange(n_u), np.diff(K.indptr))
    kill = dirichlet[rows] | dirichlet[K.indices]
    K.data[kill] = 0.0
    K = K + sp.diags(dirichlet.astype(float), format="csr")
    G = sp.diags((~dirichlet).astype(float)) @ G
    Bm = Bm @ sp.diags((~dirichlet).astype(float))
    mats = []
    for Mx in (K, G, Bm, Cm):
        Mx = sp.csr_matrix(Mx)
        Mx.eliminate_zeros()
        Mx.sort_indices()
        Mx.sum_duplicates()
        mats.append(Mx)
    K, G, Bm, Cm = mats

    # right-hand side
    top_dofs = slave_top_nodes * dim + last
    if rhs == "load":
        b = np.zeros(n_u + n_lam)
        face_top = [axes_s[a] for a in range(dim - 1)]
        b[top_dofs] = traction * _face_weights(face_top)
    elif rhs == "gap":
        b = np.zeros(n_u + n_lam)
        b[n_u + np.arange(ns) * dim + last] = penetration * D_rowsum
    elif rhs == "random":
        b = rng.uniform(-1.0, 1.0, n_u + n_lam)
    else:
        raise ValueError(rhs)
    b[:n_u][dirichlet] = 0.0

    # rigid body modes from the physical coordinates
    n_nodes = n_nodes_s + n_nodes_m
    if dim == 2:
        ns_cols = 3
        Z = np.zeros((n_u, 3))
        Z[0::2, 0] = 1.0
        Z[1::2, 1] = 1.0
        Z[0::2, 2] = -coords[:, 1]
        Z[1::2, 2] = coords[:, 0]
    else:
        ns_cols = 6
        Z = np.zeros((n_u, 6))
        x, y, z = coords[:, 0], coords[:, 1], coords[:, 2]
        Z[0::3, 0] = 1.0
        Z[1::3, 1] = 1.0
        Z[2::3, 2] = 1.0
        Z[1::3, 3] = -z
        Z[2::3, 3] = y
        Z[0::3, 4] = z
        Z[2::3, 4] = -x
        Z[0::3, 5] = -y
        Z[1::3, 5] = x

    slave_dofs = np.sort((slave_iface_nodes[:, None] * dim + np.arange(dim)).ravel()).astype(np.int32)
    master_dofs = np.sort((master_iface_nodes[:, None] * dim + np.arange(dim)).ravel()).astype(np.int32)
    lm_node = (np.arange(n_lam) // dim).astype(np.int32)
    info = dict(
        slave_elems=slave_elems,
        master_elems=master_elems,
        n_nodes=n_nodes,
        n_slave_face=ns,
        n_master_face=nm,
        E_sigma=E_sigma,
        nu=nu,
        curve_amp=curve_amp,
        seed=seed,
        rhs=rhs,
        n_ns=ns_cols,
    )
    return ContactProblem(
        dim=dim,
        K=K,
        G=G,
        B=Bm,
        C=Cm,
        b=b,
        slave_dofs=slave_dofs,
        master_dofs=master_dofs,
        lm_node=lm_node,
        nullspace=Z,
        coords=coords,
        dirichlet=dirichlet,
        top_dofs=top_dofs.astype(np.int64),
        info=info,
    )


# ----------------------------------------------------------------------------
# named workloads

WORKLOADS = {
    # 2D plane strain, 16x16 slave over 17x16 master, ~1.2k dofs
    "contact2d_16": dict(dim=2, slave_elems=(16, 16), master_elems=(17, 16)),
    # 3D hex8, 40^3 slave over 41x41x40 master, ~429k dofs
    "contact3d_40": dict(dim=3, slave_elems=(40, 40, 40), master_elems=(41, 41, 40)),
    # 3D hex8, 100^3 over 101x101x100, lognormal(0,1) Young's modulus, ~6.3M dofs
    "contact3d_100_lognormal": dict(
        dim=3, slave_elems=(100, 100, 100), master_elems=(101, 101, 100), E_sigma=1.0
    ),
    # 3D hex8, 6^3 over 7x7x6, 2520 dofs (dense-reference size)
    "contact3d_6": dict(dim=3, slave_elems=(6, 6, 6), master_elems=(7, 7, 6)),
    # 3D hex8, 150^3 over 151x151x150, lognormal(0,2) E, nu in [0.25,0.35], curved interface
    "contact3d_150_curved": dict(
        dim=3,
        slave_elems=(150, 150, 150),
        master_elems=(151, 151, 150),
        E_sigma=2.0,
        nu=(0.25, 0.35),
        curve_amp=0.05,
    ),
}


def make_workload(name: str, seed: int = 0, rhs: str = "load", **overrides) -> ContactProblem:
    params = dict(WORKLOADS[name])
    params.update(overrides)
    return make_contact_problem(seed=seed, rhs=rhs, **params)


def weak_scaling_problem(kappa: int, seed: int = 0, lm_basis: str = "standard", rhs: str = "gap") -> ContactProblem:
    """The paper's weak-scaling problem (Sec. 6.2 setup): a 0.8 x 0.8 x 0.4
    slave block on a 1.0 x 1.0 x 0.5 master block, each with 2*kappa
    elements along its long edges and kappa along the short one, the faces
    opposite the interface clamped, an initial overlap of 0.001, E = 10 and
    nu = 0.3, and multipliers in the standard (linear Lagrange) basis.  The
    paper's material is Neo-Hooke; this is its linearisation at rest."""
    return make_contact_problem(
        3,
        (2 * kappa, 2 * kappa, kappa),
        (2 * kappa, 2 * kappa, kappa),
        slave_box=([0.1, 0.1, 0.0], [0.8, 0.8, 0.4]),
        master_box=([0.0, 0.0, -0.5], [1.0, 1.0, 0.5]),
        seed=seed,
        top_bc="clamped",
        rhs=rhs,
        lm_basis=lm_basis,
        E=10.0,
        penetration=0.001,
    )


def rotate_problem(p: ContactProblem, angle_y: float, angle_z: float) -> ContactProblem:
    """The same contact problem with the whole geometry rotated by R =
    R_z(angle_z) R_y(angle_y) (radians), as in the rotation experiment of
    the two-body example (Sec. 6.1 experimental setup).  Displacements and
    the Cartesian multipliers rotate with R node by node; the constraint rows
    (normal gap, tangential slots) are scalar equations and do not:
        K' = Q K Q^T, G' = Q G Ql^T, B' = B Q^T, C' = C Ql^T,
        b' = [Q b_u; b_l],
    so the solution is [Q u; Ql l].  Dirichlet rows stay identity rows only
    where whole nodes are clamped (top_bc="clamped")."""
    cy, sy, cz, sz = np.cos(angle_y), np.sin(angle_y), np.cos(angle_z), np.sin(angle_z)
    Ry = np.array([[cy, 0.0, sy], [0.0, 1.0, 0.0], [-sy, 0.0, cy]])
    Rz = np.array([[cz, -sz, 0.0], [sz, cz, 0.0], [0.0, 0.0, 1.0]])
    R = Rz @ Ry
    d = p.dim
    assert d == 3
    d_nodes = p.dirichlet.reshape(-1, d)
    if np.any(d_nodes.any(axis=1) & ~d_nodes.all(axis=1)):
        raise ValueError("rotation needs whole nodes clamped (top_bc='clamped')")
    Q = sp.kron(sp.identity(p.n_u // d), sp.csr_matrix(R), format="csr")
    Ql = sp.kron(sp.identity(p.n_lam // d), sp.csr_matrix(R), format="csr")

    def clean(M):
        M = sp.csr_matrix(M)
        M.eliminate_zeros()
        M.sort_indices()
        return M

    # a clamped node's rows and columns of K are identity ones, and R R^T = I
    # keeps them so; write them exactly rather than with rounding residue
    K = sp.csr_matrix(Q @ p.K @ Q.T).tocoo()
    keep = ~(p.dirichlet[K.row] | p.dirichlet[K.col])
    n_dir = np.nonzero(p.dirichlet)[0]
    K = sp.csr_matrix((np.concatenate([K.data[keep], p.K.diagonal()[n_dir]]),
                       (np.concatenate([K.row[keep], n_dir]), np.concatenate([K.col[keep], n_dir]))), shape=K.shape)
    b = p.b.copy()
    b[: p.n_u] = Q @ p.b[: p.n_u]
    return ContactProblem(
        dim=d,
        K=exact_symmetric(clean(K)),
        G=clean(Q @ p.G @ Ql.T),
        B=clean(p.B @ Q.T),
        C=clean(p.C @ Ql.T),
        b=b,
        slave_dofs=p.slave_dofs,
        master_dofs=p.master_dofs,
        lm_node=p.lm_node,
        nullspace=np.asarray(Q @ p.nullspace),
        coords=p.coords @ R.T,
        dirichlet=p.dirichlet,
        top_dofs=p.top_dofs,
        info=dict(p.info, rotation=(angle_y, angle_z)),
    )
