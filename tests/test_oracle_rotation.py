"""Oracle pins for the nodal block relaxation of the Schur system and the
rotation experiment of the two-body example (Sec. 6.1: the whole setup
rigidly rotated about y and z; the iteration counts should not depend on the
angles).

Cartesian multipliers with normal/tangential constraint rows: on an
axis-aligned flat interface each multiplier node's block of
S = B Atilde^-1 G - C is diagonal, so the block option must reproduce the
diagonal one there; after a rotation the block mixes the components and
transforms with the rotation while its diagonal does not.
"""
import numpy as np
import pytest

from contactgen import make_contact_problem, rotate_problem
from oracle.adjoint import solve
from oracle.hierarchy import AMGOptions, build_hierarchy
from oracle.smoother import schur_apply
from oracle.vcycle import vcycle


def _clamped(se=(4, 4, 3), me=(5, 5, 3)):
    return make_contact_problem(3, se, me, slave_box=((0.1, 0.1, 0.0), (0.8, 0.8, 0.5)),
                                master_box=((0.0, 0.0, -1.0), (1.0, 1.0, 1.0)), top_bc="clamped", rhs="gap",
                                penetration=0.01)


def _R(ay, az):
    cy, sy, cz, sz = np.cos(ay), np.sin(ay), np.cos(az), np.sin(az)
    return np.array([[cz, -sz, 0], [sz, cz, 0], [0, 0, 1.0]]) @ np.array([[cy, 0, sy], [0, 1.0, 0], [-sy, 0, cy]])


def _rot(x, R):
    return (x.reshape(-1, 3) @ R.T).ravel()


@pytest.mark.parametrize("sweeps", [1, 3])
@pytest.mark.parametrize("transpose", [False, True])
def test_block_schur_step_is_the_nodal_dense_solve(sweeps, transpose):
    """Brute force: S built densely from its definition, its nodal 3x3
    diagonal blocks solved with numpy, block Jacobi sweeps from zero written
    out with the dense block-diagonal inverse."""
    p = rotate_problem(_clamped(), np.pi / 8, np.pi / 4)
    lv = build_hierarchy(p, AMGOptions(max_levels=2, max_coarse_rows=50, schur="block", schur_sweeps=sweeps))
    L = lv[0]
    S = L.B.toarray() @ np.diag(L.atilde_inv) @ L.G.toarray() - L.C.toarray()
    if transpose:
        S = S.T
    Db = np.zeros_like(S)
    for j in range(0, S.shape[0], 3):
        Db[j:j + 3, j:j + 3] = S[j:j + 3, j:j + 3]
    assert np.abs(S - np.diag(np.diag(S))).max() > 1e-3 * np.abs(S).max()  # the blocks really mix
    Dinv = np.linalg.inv(Db)
    rt = np.random.default_rng(5).standard_normal(S.shape[0])
    x = np.zeros_like(rt)
    for _ in range(sweeps):
        x = x + Dinv @ (rt - S @ x)
    got = schur_apply(L, rt, sweeps, transpose=transpose)
    assert np.linalg.norm(got - x) <= 1e-12 * np.linalg.norm(x)


@pytest.mark.parametrize("smoother", ["simple", "uzawa", "braess_sarazin"])
def test_block_equals_diag_on_an_axis_aligned_flat_interface(smoother):
    """Two levels: the fine level's blocks are diagonal here; coarse
    multiplier aggregates couple the components (the coarse normal row picks
    up the aggregate's rotation columns), so deeper levels differ."""
    p = _clamped()
    b = np.random.default_rng(1).standard_normal(p.n)
    out = []
    for schur in ("diag", "block"):
        opts = AMGOptions(max_levels=2, max_coarse_rows=50, schur=schur, smoother=smoother, simple_alpha=0.7)
        out.append(vcycle(build_hierarchy(p, opts), b, opts))
    assert np.linalg.norm(out[1] - out[0]) <= 1e-12 * np.linalg.norm(out[0])


@pytest.mark.parametrize("smoother", ["simple", "uzawa", "braess_sarazin"])
@pytest.mark.parametrize("angles", [(np.pi / 2, 0.0), (np.pi / 2, np.pi / 2)])
def test_quarter_turns_are_exact_symmetries_with_the_block_option(smoother, angles):
    """A quarter turn maps the Cartesian axes onto each other with signs, so
    every ingredient (row sums of |K|, aggregates, QR of the null space,
    Galerkin blocks, nodal Schur blocks) transforms exactly and the V-cycle
    of the rotated problem is the rotated V-cycle: M'(Q r) = Q M r."""
    p = _clamped()
    q = rotate_problem(p, *angles)
    R = _R(*angles)
    opts = AMGOptions(max_levels=3, max_coarse_rows=50, schur="block", smoother=smoother, simple_alpha=0.7,
                      nu_pre=3, nu_post=3)
    r = np.random.default_rng(2).standard_normal(p.n)
    z = vcycle(build_hierarchy(p, opts), r, opts)
    rq = np.concatenate([_rot(r[:p.n_u], R), r[p.n_u:]])
    zq = vcycle(build_hierarchy(q, opts), rq, opts)
    expect = np.concatenate([_rot(z[:p.n_u], R), _rot(z[p.n_u:], R)])
    assert np.linalg.norm(zq - expect) <= 1e-10 * np.linalg.norm(expect)


@pytest.mark.parametrize("smoother", ["simple", "uzawa", "braess_sarazin"])
@pytest.mark.parametrize("sweeps", [1, 3])
def test_block_schur_vcycle_transpose_dot_product(smoother, sweeps):
    p = rotate_problem(_clamped(), 3 * np.pi / 8, np.pi / 8)
    opts = AMGOptions(max_levels=3, max_coarse_rows=50, schur="block", schur_sweeps=sweeps, smoother=smoother,
                      simple_alpha=0.7)
    lv = build_hierarchy(p, opts)
    rng = np.random.default_rng(3)
    u, v = rng.standard_normal(p.n), rng.standard_normal(p.n)
    a1 = v @ vcycle(lv, u, opts)
    a2 = vcycle(lv, v, opts, transpose=True) @ u
    assert abs(a1 - a2) <= 1e-11 * abs(a1)


def test_block_schur_keeps_cheap_simple_iterations_under_rotation():
    """The diagonal Schur step loses the normal constraint's pivot once the
    interface is tilted; the nodal block step keeps the counts close to the
    unrotated ones (the paper's CheapSIMPLE table varies within about 15%)."""
    p = _clamped((6, 6, 4), (7, 7, 4))
    its = {}
    for schur in ("diag", "block"):
        opts = AMGOptions(max_levels=3, max_coarse_rows=50, schur=schur, simple_alpha=0.7, jacobi_omega=0.7,
                          nu_pre=3, nu_post=3)
        for ang in [(0.0, 0.0), (np.pi / 4, np.pi / 8), (3 * np.pi / 8, np.pi / 4)]:
            q = rotate_problem(p, *ang)
            r = solve(build_hierarchy(q, opts), opts, q.b, rtol=1e-8, max_iters=150)
            its[schur, ang] = r.iters if r.converged else 10**9
    base = its["block", (0.0, 0.0)]
    assert its["diag", (0.0, 0.0)] == base
    for ang in [(np.pi / 4, np.pi / 8), (3 * np.pi / 8, np.pi / 4)]:
        assert its["block", ang] <= 1.25 * base, its
        assert its["diag", ang] > 2 * base, its


# ---- nodal lumping --------------------------------------------------------------


def test_nodal_lumping_is_the_block_plus_frobenius_sums():
    from oracle.hierarchy import nodal_lumping

    p = rotate_problem(_clamped(), np.pi / 8, np.pi / 4)
    Kd = p.K.toarray()
    got = nodal_lumping(p.K, 3)
    for i in range(p.n_u // 3):
        bi = slice(3 * i, 3 * i + 3)
        off = sum(np.sqrt((Kd[bi, 3 * j:3 * j + 3] ** 2).sum()) for j in range(p.n_u // 3) if j != i)
        assert np.allclose(got[i], Kd[bi, bi] + off * np.eye(3), rtol=0, atol=1e-14 * np.abs(Kd).max())


def test_nodal_lumping_bounds_the_spectrum():
    """x^T K x <= x^T Atilde x: the eigenvalues of Atilde^-1 K lie in (0, 1]."""
    from oracle.hierarchy import block_diag_matrix, nodal_lumping

    p = rotate_problem(_clamped(), np.pi / 3, np.pi / 5)
    A = block_diag_matrix(nodal_lumping(p.K, 3)).toarray()
    ev = np.linalg.eigvals(np.linalg.solve(A, p.K.toarray())).real
    assert ev.min() > 0 and ev.max() <= 1 + 1e-12, (ev.min(), ev.max())


NODAL = dict(max_levels=3, max_coarse_rows=50, atilde="nodal", schur="block", nu_pre=3, nu_post=3)


@pytest.mark.parametrize("smoother", ["simple", "uzawa", "braess_sarazin"])
@pytest.mark.parametrize("prolongator", ["pa", "sa"])
def test_nodal_options_are_rotation_covariant(smoother, prolongator):
    """With the nodal lumping and the nodal Schur blocks every ingredient
    transforms with the rotation at any angle, so the V-cycle of the rotated
    problem is the rotated V-cycle: M'(Q r) = Q M r (the coarse levels are the
    same matrices, the fine-level blocks are R X R^T)."""
    p = _clamped()
    angles = (0.3, 1.1)
    q = rotate_problem(p, *angles)
    R = _R(*angles)
    opts = AMGOptions(**NODAL, smoother=smoother, prolongator=prolongator, simple_alpha=0.7, schur_sweeps=2)
    r = np.random.default_rng(6).standard_normal(p.n)
    z = vcycle(build_hierarchy(p, opts), r, opts)
    rq = np.concatenate([_rot(r[:p.n_u], R), r[p.n_u:]])
    lq = build_hierarchy(q, opts)
    zq = vcycle(lq, rq, opts)
    expect = np.concatenate([_rot(z[:p.n_u], R), _rot(z[p.n_u:], R)])
    assert np.linalg.norm(zq - expect) <= 1e-10 * np.linalg.norm(expect)
    # the point lumping is not covariant
    popts = AMGOptions(**dict(NODAL, atilde="rowsum_abs"), smoother=smoother, prolongator=prolongator,
                       simple_alpha=0.7, schur_sweeps=2)
    zp = vcycle(build_hierarchy(p, popts), r, popts)
    zpq = vcycle(build_hierarchy(q, popts), rq, popts)
    ep = np.concatenate([_rot(zp[:p.n_u], R), _rot(zp[p.n_u:], R)])
    assert np.linalg.norm(zpq - ep) > 1e-6 * np.linalg.norm(ep)


@pytest.mark.parametrize("smoother", ["simple", "uzawa", "braess_sarazin"])
@pytest.mark.parametrize("sweeps", [1, 2])
def test_nodal_vcycle_transpose_with_nonsymmetric_K(smoother, sweeps):
    """A nonsymmetric perturbation of K makes the lumping blocks
    nonsymmetric, so the adjoint sweep must apply them transposed."""
    import dataclasses

    p = rotate_problem(_clamped(), 0.4, 0.9)
    K = p.K.tocoo()
    rng = np.random.default_rng(7)
    free = ~p.dirichlet[K.row] & ~p.dirichlet[K.col]
    data = K.data + np.where(free, 0.05 * np.abs(K.data).max() * rng.uniform(-1, 1, K.nnz), 0.0)
    import scipy.sparse as sp

    p2 = dataclasses.replace(p, K=sp.csr_matrix((data, (K.row, K.col)), shape=K.shape))
    opts = AMGOptions(**NODAL, smoother=smoother, simple_alpha=0.7, schur_sweeps=sweeps, jacobi_sweeps=2)
    lv = build_hierarchy(p2, opts)
    assert np.abs(lv[0].atilde_inv - lv[0].atilde_inv.transpose(0, 2, 1)).max() > 1e-8
    u, v = rng.standard_normal(p.n), rng.standard_normal(p.n)
    a1 = v @ vcycle(lv, u, opts)
    a2 = vcycle(lv, v, opts, transpose=True) @ u
    assert abs(a1 - a2) <= 1e-11 * abs(a1)


@pytest.mark.parametrize("smoother", ["simple", "uzawa", "braess_sarazin"])
def test_nodal_iterations_do_not_depend_on_the_angles(smoother):
    p = _clamped((6, 6, 4), (7, 7, 4))
    opts = AMGOptions(**NODAL, smoother=smoother, simple_alpha=1.9 if smoother == "braess_sarazin" else 0.7,
                      jacobi_omega=0.7)
    its = []
    for ang in [(0.0, 0.0), (np.pi / 8, np.pi / 4), (3 * np.pi / 8, np.pi / 8), (np.pi / 2, 3 * np.pi / 8)]:
        q = rotate_problem(p, *ang)
        r = solve(build_hierarchy(q, opts), opts, q.b, rtol=1e-8, max_iters=300)
        assert r.converged
        its.append(r.iters)
    assert max(its) - min(its) <= 1, its
