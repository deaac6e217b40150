"""Pins for the seeded input generator (CPU).

The generator is input-side, but its properties are checked against what the
paper and the mathematics fix: printed dof counts, rigid-body invariance of
the stiffness, patch test, dual-mortar identities.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

from contactgen import make_contact_problem, make_workload, weak_scaling_problem
from contactgen.fe import box_element_coords, element_stiffness_split, lame_from_E_nu
from contactgen.mortar import mortar_1d, mortar_face
from contactgen.problem import _assemble_body, _element_shapes, _grid_coords

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_rows(name):
    rows = []
    for line in open(os.path.join(GOLDEN, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append([int(v) for v in line.split()])
    return rows


def test_table3_first_row_from_generator():
    kappa, n_u, n_l, n = _read_rows("weak_scaling_table3_sizes.txt")[0]
    p = weak_scaling_problem(kappa)
    assert (p.n_u, p.n_lam, p.n) == (n_u, n_l, n)


@pytest.mark.parametrize("kappa", [1, 2, 3])
def test_table3_counting_small(kappa):
    # node counting of the generator vs the structure of the table: two blocks of
    # (2k+1)^2 (k+1) nodes, 3 dofs each; slave face (2k+1)^2 nodes, 3 multipliers each
    p = weak_scaling_problem(kappa)
    assert p.n_u == 2 * 3 * (2 * kappa + 1) ** 2 * (kappa + 1)
    assert p.n_lam == 3 * (2 * kappa + 1) ** 2


def test_table3_all_rows_consistent():
    # every printed row obeys the generator's node counting
    for kappa, n_u, n_l, n in _read_rows("weak_scaling_table3_sizes.txt"):
        assert n_u == 6 * (2 * kappa + 1) ** 2 * (kappa + 1)
        assert n_l == 3 * (2 * kappa + 1) ** 2
        assert n == n_u + n_l


def test_two_bodies_worked_example_counts():
    (n_u, n_l), = _read_rows("two_bodies_dofs.txt")
    p = make_contact_problem(3, (9, 9, 9), (9, 9, 9))
    assert (p.n_u, p.n_lam) == (n_u, n_l)


def test_workload_sizes():
    p = make_workload("contact2d_16")
    assert (p.n_u, p.n_lam) == (1190, 34)
    p = make_workload("contact3d_6")
    assert (p.n_u, p.n_lam) == (2373, 147)


@pytest.mark.parametrize("dim", [2, 3])
def test_element_zero_energy_modes(dim):
    Kl, Km = element_stiffness_split(box_element_coords([0.3, 0.5, 0.7][:dim]))
    lam, mu = lame_from_E_nu(1.0, 0.3)
    ev = np.linalg.eigvalsh(lam * Kl + mu * Km)
    n_rbm = 3 if dim == 2 else 6
    assert np.sum(np.abs(ev) < 1e-10 * ev.max()) == n_rbm
    assert ev.min() > -1e-10 * ev.max()


def _body(dim, nel, sigma=0.0):
    axes = _grid_coords(nel, [0.0] * dim, [1.0, 0.8, 0.6][:dim])
    Kl, Km = _element_shapes(nel, axes, None)
    rng = np.random.default_rng(1)
    grid = tuple(reversed(nel))
    E = rng.lognormal(0.0, sigma, grid) if sigma else np.ones(grid)
    lam, mu = lame_from_E_nu(E, 0.3)
    K = _assemble_body(nel, axes, lam, mu, Kl, Km)
    mesh = np.meshgrid(*axes, indexing="ij")
    X = np.stack([m.transpose(tuple(reversed(range(dim)))).ravel() for m in mesh], axis=1)
    return K, X


@pytest.mark.parametrize("dim,nel", [(2, (4, 3)), (3, (3, 2, 2))])
def test_body_stiffness_symmetric_and_rigid_modes(dim, nel):
    K, X = _body(dim, nel, sigma=1.0)
    assert abs(K - K.T).max() < 1e-14 * abs(K).max()
    n = X.shape[0]
    modes = []
    for c in range(dim):
        t = np.zeros((n, dim))
        t[:, c] = 1.0
        modes.append(t.ravel())
    if dim == 2:
        modes.append(np.stack([-X[:, 1], X[:, 0]], axis=1).ravel())
    else:
        x, y, z = X.T
        modes.append(np.stack([0 * x, -z, y], axis=1).ravel())
        modes.append(np.stack([z, 0 * x, -x], axis=1).ravel())
        modes.append(np.stack([-y, x, 0 * x], axis=1).ravel())
    for m in modes:
        assert np.abs(K @ m).max() < 1e-12 * abs(K).max()


@pytest.mark.parametrize("dim,nel", [(2, (4, 4)), (3, (3, 3, 3))])
def test_patch_test_interior_balance(dim, nel):
    # a linear displacement field has constant stress: nodal forces vanish at interior nodes
    K, X = _body(dim, nel)
    rng = np.random.default_rng(0)
    F = rng.standard_normal((dim, dim))
    u = (X @ F.T).ravel()
    f = (K @ u).reshape(-1, dim)
    hi = np.array([1.0, 0.8, 0.6][:dim])
    interior = np.all((X > 1e-12) & (X < hi - 1e-12), axis=1)
    assert interior.any()
    assert np.abs(f[interior]).max() < 1e-12 * np.abs(f).max()


def test_mortar_1d_identities():
    xs = np.linspace(0.0, 1.0, 9)
    xm = np.linspace(0.0, 1.0, 12)
    D, M = mortar_1d(xs, xm)
    h = xs[1] - xs[0]
    # D_jj = int N_j: h in the interior, h/2 at the ends
    assert np.allclose(D[1:-1], h, rtol=0, atol=1e-15)
    assert np.allclose(D[[0, -1]], h / 2, rtol=0, atol=1e-15)
    # master partition of unity: rows of M sum to D_jj
    assert np.allclose(M.sum(axis=1), D, rtol=0, atol=1e-14)
    # matching meshes: M = D
    D2, M2 = mortar_1d(xs, xs)
    assert np.allclose(M2, np.diag(D2), rtol=0, atol=1e-15)


def test_mortar_1d_brute_force_quadrature():
    xs = np.linspace(0.0, 1.0, 6)
    xm = np.array([0.0, 0.13, 0.4, 0.41, 0.77, 1.0])
    D, M = mortar_1d(xs, xm)
    # midpoint rule with many points on psi_j N_k
    x = (np.arange(200000) + 0.5) / 200000
    def hat(nodes, k, x):
        return np.interp(x, nodes, np.eye(len(nodes))[k])
    es = np.clip(np.searchsorted(xs, x, side="right") - 1, 0, len(xs) - 2)
    t = (x - xs[es]) / (xs[es + 1] - xs[es])
    for j in range(len(xs)):
        psi = np.zeros_like(x)
        left = es == j      # j is the first node of its element
        psi[left] = 2 * (1 - t[left]) - t[left]
        right = es == j - 1  # j is the second node
        psi[right] = 2 * t[right] - (1 - t[right])
        for k in range(len(xm)):
            ref = np.mean(psi * hat(xm, k, x))
            assert abs(ref - M[j, k]) < 1e-8
        assert abs(np.mean(psi * hat(xs, j, x)) - D[j]) < 1e-8
        # biorthogonality against the other slave shape functions
        for k in range(len(xs)):
            if k != j:
                assert abs(np.mean(psi * hat(xs, k, x))) < 1e-8


def test_mortar_face_is_kronecker():
    ax_s = [np.linspace(0, 1, 4), np.linspace(0, 1, 5)]
    ax_m = [np.linspace(0, 1, 6), np.linspace(0, 1, 3)]
    D, M = mortar_face(ax_s, ax_m)
    Dx, Mx = mortar_1d(ax_s[0], ax_m[0])
    Dy, My = mortar_1d(ax_s[1], ax_m[1])
    # face node index = ix + nx * iy
    for iy in range(5):
        for ix in range(4):
            j = ix + 4 * iy
            assert abs(D[j] - Dx[ix] * Dy[iy]) < 1e-15
            for ky in range(3):
                for kx in range(6):
                    assert abs(M[j, kx + 6 * ky] - Mx[ix, kx] * My[iy, ky]) < 1e-15


def test_blocks_structure_flat():
    p = make_workload("contact3d_6")
    d = p.dim
    # slave interface rows of G carry D on the matching multiplier, master rows -M^T
    G = p.G.tocsr()
    sl = p.slave_dofs
    for i in sl[:30]:
        cols = G.indices[G.indptr[i]:G.indptr[i + 1]]
        assert len(cols) == 1 and cols[0] % d == i % d
    # normal constraint rows equal the matching rows of G^T; tangential rows of B empty
    GT = G.T.tocsr()
    B = p.B.tocsr()
    for j in range(p.n_lam):
        if j % d == d - 1:
            assert abs(B[j] - GT[j]).max() < 1e-15
        else:
            assert B[j].nnz == 0
            assert p.C[j, j] == 1.0
    # Dirichlet rows are identity rows with zero columns
    K = p.K.tocsr()
    for i in np.nonzero(p.dirichlet)[0][:50]:
        assert K[i].nnz == 1 and K[i, i] == 1.0
        assert K[:, i].nnz == 1


def test_curved_interface_small():
    p = make_contact_problem(3, (4, 4, 4), (5, 5, 4), curve_amp=0.05, E_sigma=2.0, nu=(0.25, 0.35), seed=3)
    K = p.K
    assert abs(K - K.T).max() < 1e-13 * abs(K).max()
    # master partition of unity still holds with the surface weight
    Dd = np.array([p.G[i, j] for i, j in zip(p.slave_dofs[::3], range(0, p.n_lam, 3))])
    assert np.all(Dd > 0)
    A = p.full_matrix().tocsc()
    x = sp.linalg.spsolve(A, p.b)
    assert np.linalg.norm(A @ x - p.b) < 1e-10 * np.linalg.norm(p.b)


# ---- standard (non-dual) multiplier basis and the weak-scaling problem ----


def test_mortar_1d_standard_basis_closed_form():
    # linear Lagrange functions: D is the 1D mass matrix h/6 [1 4 1]
    # (h/3 on the end nodes), symmetric positive definite, with row sums
    # int N_j (the dual D's diagonal); matching meshes give M = D, and full
    # master coverage gives M row sums int N_j too
    h = 0.125
    xs = np.arange(9) * h
    D, M = mortar_1d(xs, xs, basis="standard")
    ref = np.diag(np.full(9, 4.0)) + np.diag(np.ones(8), 1) + np.diag(np.ones(8), -1)
    ref[0, 0] = ref[-1, -1] = 2.0
    assert np.allclose(D, ref * h / 6, rtol=0, atol=1e-15)
    assert np.allclose(M, D, rtol=0, atol=1e-15)
    Dd, _ = mortar_1d(xs, xs)
    assert np.allclose(D.sum(axis=1), Dd, rtol=0, atol=1e-15)
    assert np.linalg.eigvalsh(D).min() > 0
    xm = np.linspace(-0.05, 1.07, 12)  # non-matching, covers the slave line
    D2, M2 = mortar_1d(xs, xm, basis="standard")
    assert np.allclose(M2.sum(axis=1), Dd, rtol=0, atol=1e-14)
    assert np.allclose(D2, D, rtol=0, atol=1e-15)


def test_standard_basis_face_and_blocks():
    p = make_contact_problem(3, (4, 4, 2), (5, 5, 2), lm_basis="standard", top_bc="clamped", rhs="gap",
                             penetration=0.001)
    q = make_contact_problem(3, (4, 4, 2), (5, 5, 2), top_bc="clamped", rhs="gap", penetration=0.001)
    # G slave rows now couple a slave dof to up to 9 multipliers of its component
    Gs = p.G[p.slave_dofs].tocsr()
    assert np.diff(Gs.indptr).max() == 9 and np.diff(q.G[q.slave_dofs].tocsr().indptr).max() == 1
    # the two bases give the same weighted gap (row sums of D are int N_j)
    assert np.allclose(p.b, q.b, rtol=0, atol=1e-15)
    d = p.dim
    normal_rows = p.n_u + np.arange(p.n_lam // d) * d + (d - 1)
    assert np.all(p.b[normal_rows] > 0) and np.count_nonzero(p.b) == normal_rows.size
    # constraint rows equal the matching rows of G^T (normal slot)
    Bn = p.B[normal_rows - p.n_u].toarray()
    GT = p.G.T.tocsr()[normal_rows - p.n_u].toarray()
    assert np.allclose(Bn, GT, rtol=0, atol=1e-15)


def test_weak_scaling_problem_closes_the_overlap():
    # direct solve of the linearised weak-scaling problem: the slave face
    # moves away from the master by the overlap (weighted), both clamped
    # blocks are compressed
    import scipy.sparse.linalg as spl

    p = weak_scaling_problem(2)
    x = spl.spsolve(p.full_matrix().tocsc(), p.b)
    u = x[: p.n_u]
    d = p.dim
    s_nodes = p.slave_dofs[d - 1::d] // d
    m_nodes = p.master_dofs[d - 1::d] // d
    assert np.all(u[s_nodes * d + d - 1] > 0) and np.all(u[m_nodes * d + d - 1] < 0)
    normal_rows = np.arange(p.n_lam // d) * d + (d - 1)
    assert np.allclose(p.B[normal_rows] @ u, p.b[p.n_u + normal_rows], rtol=1e-9, atol=0)


def test_rotated_problem_has_the_rotated_solution():
    # rotating the geometry rotates displacements and Cartesian multipliers
    # node by node and leaves the constraint equations: the direct solution
    # of the rotated system is [Q u; Ql lam]
    import scipy.sparse.linalg as spl

    from contactgen import rotate_problem

    p = make_contact_problem(3, (4, 4, 3), (5, 5, 3), top_bc="clamped", rhs="random", seed=3)
    x = spl.spsolve(p.full_matrix().tocsc(), p.b)
    ay, az = np.pi / 8, 3 * np.pi / 8
    q = rotate_problem(p, ay, az)
    xr = spl.spsolve(q.full_matrix().tocsc(), q.b)
    cy, sy, cz, sz = np.cos(ay), np.sin(ay), np.cos(az), np.sin(az)
    R = np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1.0]]) @ np.array([[cy, 0, sy], [0, 1.0, 0], [-sy, 0, cy]])
    expect = np.concatenate([(x[: p.n_u].reshape(-1, 3) @ R.T).ravel(), (x[p.n_u:].reshape(-1, 3) @ R.T).ravel()])
    assert np.linalg.norm(xr - expect) <= 1e-10 * np.linalg.norm(expect)
    # rigid-body modes of the rotated bodies are in K's kernel away from the clamps
    KZ = np.abs(q.K @ q.nullspace).max(axis=1)
    free = ~q.dirichlet
    assert np.sort(KZ[free])[free.sum() // 2] <= 1e-12 * np.abs(q.K.data).max()
    with pytest.raises(ValueError):
        rotate_problem(make_contact_problem(3, (2, 2, 2), (3, 3, 2)), 0.1, 0.2)  # roller: partial clamps


def test_exact_symmetric_mean_of_mirrors():
    """(K + K^T)/2 entry by entry: mirrored entries become the same number,
    an entry stored on one side only appears on both with half its value,
    and exact zeros are dropped."""
    from contactgen.problem import exact_symmetric

    K = sp.csr_matrix(np.array([[4.0, 1.0 + 2.0 ** -52, 0.0],
                                [1.0, 3.0, 2.0 ** -60],
                                [0.0, 0.0, 0.0]]))
    S = exact_symmetric(K).toarray()
    assert np.array_equal(S, S.T)
    assert S[0, 1] == (1.0 + 2.0 ** -52 + 1.0) / 2
    assert S[1, 2] == S[2, 1] == 2.0 ** -61
    assert exact_symmetric(K).nnz == 6


@pytest.mark.parametrize("name", ["contact2d_16", "contact3d_6", "contact3d_150_curved"])
def test_stiffness_equals_its_transpose_bit_for_bit(name):
    """The generator's K equals K^T exactly (pattern and values), also on the
    curved geometry and after a rotation of the whole problem."""
    from contactgen.problem import rotate_problem

    kw = dict(slave_elems=(4, 4, 4), master_elems=(5, 5, 4)) if name == "contact3d_150_curved" else {}
    probs = [make_workload(name, **kw)]
    if name == "contact3d_6":
        probs.append(rotate_problem(make_contact_problem(3, (4, 4, 3), (5, 5, 3), top_bc="clamped"), 0.3, 0.2))
    for p in probs:
        K = p.K.tocsr()
        Kt = K.T.tocsr()
        Kt.sort_indices()
        assert np.array_equal(K.indptr, Kt.indptr) and np.array_equal(K.indices, Kt.indices)
        assert np.array_equal(K.data, Kt.data)


@pytest.mark.parametrize("dim,nel", [(2, (4, 3)), (3, (3, 2, 2))])
def test_body_stiffness_equals_plain_element_sum(dim, nel):
    """The structured assembly (blockwise, then each mirrored block pair
    replaced by its mean) equals the element-by-element sum written out with
    a plain COO scatter, to rounding, and is symmetric bit for bit: a wrong
    mirror pairing in the symmetrisation would show as an O(1) difference."""
    K, X = _body(dim, nel, sigma=1.0)
    axes = _grid_coords(nel, [0.0] * dim, [1.0, 0.8, 0.6][:dim])
    Kl, Km = _element_shapes(nel, axes, None)
    rng = np.random.default_rng(1)
    grid = tuple(reversed(nel))
    lam, mu = lame_from_E_nu(rng.lognormal(0.0, 1.0, grid), 0.3)
    nn = [n + 1 for n in nel]
    offs = np.array([[(l >> k) & 1 for k in range(dim)] for l in range(2 ** dim)])
    rows, cols, vals = [], [], []
    for e in np.ndindex(*grid):  # e = (z, y, x) or (y, x)
        ex = tuple(reversed(e))  # element index along x first
        nodes = [sum((ex[k] + o[k]) * int(np.prod(nn[:k])) for k in range(dim)) for o in offs]
        dofs = np.array([n * dim + c for n in nodes for c in range(dim)])
        Ke = lam[e] * Kl.reshape(Kl.shape[-2:]) + mu[e] * Km.reshape(Km.shape[-2:])
        rows.append(np.repeat(dofs, dofs.size))
        cols.append(np.tile(dofs, dofs.size))
        vals.append(Ke.ravel())
    n = int(np.prod(nn)) * dim
    R = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).toarray()
    D = K.toarray()
    assert np.abs(D - R).max() <= 1e-14 * np.abs(R).max()
    assert np.array_equal(D, D.T)
