"""Pins for the oracle's V-cycle, FGMRES and adjoint (CPU)."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

from contactgen import make_contact_problem, make_workload
from oracle.adjoint import grad_K_values, solve
from oracle.fgmres import fgmres
from oracle.hierarchy import AMGOptions, SingularCoarse, build_hierarchy
from oracle.vcycle import _apply_A, vcycle


@pytest.fixture(scope="module")
def h3d():
    p = make_workload("contact3d_6")
    opts = AMGOptions(max_levels=2)
    return p, build_hierarchy(p, opts), opts


@pytest.fixture(scope="module")
def h2d():
    p = make_workload("contact2d_16")
    opts = AMGOptions(max_levels=3, max_coarse_rows=50, nu_pre=1, nu_post=1)
    return p, build_hierarchy(p, opts), opts


def test_vcycle_transpose_dot_product(h2d, h3d):
    for p, lv, opts in (h2d, h3d):
        rng = np.random.default_rng(5)
        for _ in range(3):
            x, y = rng.standard_normal(p.n), rng.standard_normal(p.n)
            a = y @ vcycle(lv, x, opts)
            b = vcycle(lv, y, opts, transpose=True) @ x
            assert abs(a - b) <= 1e-11 * (abs(a) + 1e-30) + 1e-14


def test_vcycle_linear(h2d):
    p, lv, opts = h2d
    rng = np.random.default_rng(6)
    x, y = rng.standard_normal(p.n), rng.standard_normal(p.n)
    lhs = vcycle(lv, 2.0 * x - 3.0 * y, opts)
    rhs = 2.0 * vcycle(lv, x, opts) - 3.0 * vcycle(lv, y, opts)
    assert np.abs(lhs - rhs).max() < 1e-11 * np.abs(lhs).max()


def test_two_grid_galerkin_orthogonality(h3d):
    # without smoothing a two-grid cycle is the coarse correction z = P A_c^-1 R b, and
    # the restricted residual vanishes: R (b - A z) = 0
    p, lv, opts = h3d
    o0 = AMGOptions(max_levels=2, nu_pre=0, nu_post=0)
    rng = np.random.default_rng(7)
    b = rng.standard_normal(p.n)
    z = vcycle(lv, b, o0)
    r = b - lv[0].A() @ z
    L = lv[0]
    rc = np.concatenate([L.P_u.T @ r[:L.n_u], L.P_l.T @ r[L.n_u:]])
    assert np.abs(rc).max() < 1e-10 * np.abs(b).max()


def test_single_level_is_exact_and_fgmres_one_iteration():
    p = make_workload("contact2d_16")
    opts = AMGOptions(max_levels=1)
    lv = build_hierarchy(p, opts)
    res = solve(lv, opts, p.b, rtol=1e-8)
    assert res.iters == 1 and res.converged
    x = spl.spsolve(p.full_matrix().tocsc(), p.b)
    assert np.linalg.norm(res.x - x) <= 1e-10 * np.linalg.norm(x)


def test_fgmres_exact_preconditioner_one_iteration():
    p = make_workload("contact3d_6", rhs="random", seed=2)
    A = p.full_matrix().tocsc()
    lu = spl.splu(A)
    res = fgmres(lambda v: A @ v, lu.solve, p.b, rtol=1e-8)
    assert res.iters == 1 and res.converged


def test_fgmres_minimal_residual_property():
    # unpreconditioned, every iterate minimises ||b - A x|| over the Krylov space
    rng = np.random.default_rng(3)
    n = 40
    A = rng.standard_normal((n, n)) + 8 * np.eye(n)
    b = rng.standard_normal(n)
    for k in (1, 3, 7, 12):
        res = fgmres(lambda v: A @ v, lambda v: v, b, m=50, fixed_iters=k)
        Kry = np.column_stack([np.linalg.matrix_power(A, i) @ b for i in range(k)])
        Qk, _ = np.linalg.qr(Kry)
        y, *_ = np.linalg.lstsq(A @ Qk, b, rcond=None)
        best = np.linalg.norm(b - A @ (Qk @ y))
        assert abs(np.linalg.norm(b - A @ res.x) - best) < 1e-10 * np.linalg.norm(b)
        assert np.allclose(res.x, Qk @ y, atol=1e-9)


def test_fgmres_restart_and_history_monotone(h2d):
    p, lv, opts = h2d
    L0 = lv[0]
    res = fgmres(lambda v: _apply_A(L0, v, False), lambda v: vcycle(lv, v, opts), p.b, m=5, rtol=1e-8)
    assert res.converged and res.restarts >= 1
    # within a restart cycle the least-squares residual estimate never increases
    h = np.array(res.history)
    assert np.all(np.diff(h[1:6]) <= 1e-15)


@pytest.mark.parametrize("name", ["contact2d_16", "contact3d_6"])
def test_solution_matches_sparse_lu(name):
    p = make_workload(name)
    opts = AMGOptions(max_levels=2, nu_pre=1 if p.dim == 2 else 2, nu_post=1 if p.dim == 2 else 2)
    lv = build_hierarchy(p, opts)
    res = solve(lv, opts, p.b, rtol=1e-8)
    assert res.converged
    x = spl.spsolve(p.full_matrix().tocsc(), p.b)
    assert np.linalg.norm(res.x - x) <= 1e-6 * np.linalg.norm(x)
    res2 = solve(lv, opts, p.b, rtol=1e-12)
    assert np.linalg.norm(res2.x - x) <= 1e-9 * np.linalg.norm(x)


def test_adjoint_solve_and_dense_gradient(h3d):
    p, lv, opts = h3d
    A = p.full_matrix().toarray()
    n_u = p.n_u
    x_ref = np.linalg.solve(A, p.b)
    top = p.top_dofs
    g = np.zeros(p.n)
    g[top] = x_ref[top]  # dL/dx for L = 0.5 ||u_top||^2
    lam_ref = np.linalg.solve(A.T, g)
    fwd = solve(lv, opts, p.b, rtol=1e-12)
    adj = solve(lv, opts, g, transpose=True, rtol=1e-12)
    assert np.linalg.norm(fwd.x - x_ref) <= 1e-9 * np.linalg.norm(x_ref)
    assert np.linalg.norm(adj.x - lam_ref) <= 1e-9 * np.linalg.norm(lam_ref)
    gK = grad_K_values(p.K, adj.x[:n_u], fwd.x[:n_u])
    rows = np.repeat(np.arange(n_u), np.diff(p.K.indptr))
    dense = -np.outer(lam_ref[:n_u], x_ref[:n_u])
    ref = dense[rows, p.K.indices]
    assert np.abs(gK - ref).max() <= 1e-9 * np.abs(ref).max()


def test_gradients_central_differences(h3d):
    p, lv, opts = h3d
    n_u = p.n_u
    top = p.top_dofs

    def loss(x):
        return 0.5 * np.sum(x[top] ** 2)

    fwd = solve(lv, opts, p.b, rtol=1e-13)
    g = np.zeros(p.n)
    g[top] = fwd.x[top]
    adj = solve(lv, opts, g, transpose=True, rtol=1e-13)
    gK = grad_K_values(p.K, adj.x[:n_u], fwd.x[:n_u])
    rng = np.random.default_rng(11)
    # step 1e-6; the central difference itself is only good to about 1e-7 relative on
    # stiff entries, so the bar is 1e-6 of the gradient's largest entry
    h = 1e-6
    A = p.full_matrix().tocsc()

    def exact(Am, rhs):
        lu = spl.splu(Am)
        x = lu.solve(rhs)
        return x + lu.solve(rhs - Am @ x)  # one step of iterative refinement

    # right-hand side entries
    for i in rng.choice(np.nonzero(~p.dirichlet)[0], 10, replace=False):
        vals = []
        for s in (h, -h):
            bb = p.b.copy()
            bb[i] += s
            vals.append(loss(exact(A, bb)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - adj.x[i]) <= 1e-6 * np.abs(adj.x).max()
    # stiffness nonzeros (one entry perturbed, K becomes nonsymmetric)
    K = p.K.tocsr()
    for k in rng.choice(K.nnz, 10, replace=False):
        vals = []
        for s in (h, -h):
            Kp = K.copy()
            Kp.data[k] += s
            Ap = sp.bmat([[Kp, p.G], [p.B, p.C]], format="csc")
            vals.append(loss(exact(Ap, p.b)))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - gK[k]) <= 1e-6 * np.abs(gK).max()


def test_singular_coarsest_detected():
    # a frictionless slave block without the roller keeps free sliding modes
    p = make_contact_problem(2, (6, 6), (7, 6), top_bc="free")
    with pytest.raises(SingularCoarse):
        build_hierarchy(p, AMGOptions(max_levels=1))
