"""Pins for the oracle's optional robustness settings (CPU): smoothed
aggregation for the displacement transfers (Sec. 3.1.2, prolongator
smoothing; omega = 4/3 as in the weak-scaling settings) and Jacobi sweeps on
the Schur system with the signed l1-lumped diagonal.  Each pin is a property
the mathematics fixes independently of the code under test."""
import numpy as np
import pytest

from contactgen import make_workload
from oracle.adjoint import solve
from oracle.hierarchy import AMGOptions, build_hierarchy, galerkin
from oracle.smoother import cheap_simple_sweep
from oracle.vcycle import vcycle

ROBUST = dict(prolongator="sa", schur="l1", schur_sweeps=3, jacobi_sweeps=3)


def _cases():
    return [
        ("contact2d_16", {}),
        ("contact3d_6", {}),
        # the large-contrast workload's material law and curved interface at 6^3
        ("contact3d_150_curved", dict(slave_elems=(6, 6, 6), master_elems=(7, 7, 6))),
    ]


@pytest.fixture(scope="module", params=_cases(), ids=lambda c: c[0])
def pair(request):
    name, kw = request.param
    p = make_workload(name, **kw)
    sa = build_hierarchy(p, AMGOptions(max_levels=2, **ROBUST))
    pa = build_hierarchy(p, AMGOptions(max_levels=2))
    return p, sa, pa


def test_lumped_diagonal_bounds_spectrum(pair):
    # Gershgorin: every eigenvalue of Atilde^-1 K lies in [-1, 1] for
    # Atilde = diag(sum_j |K_ij|), so omega = 4/3 never amplifies a mode
    _, sa, _ = pair
    K = sa[0].K.toarray()
    lam = np.linalg.eigvals(K / np.abs(K).sum(axis=1)[:, None]).real
    assert lam.max() <= 1.0 + 1e-12 and lam.min() >= -1e-12


def test_smoothed_prolongator_reproduces_rigid_modes(pair):
    # wherever K annihilates the rigid body modes (rows away from the
    # boundary conditions) one damped Jacobi step leaves them unchanged, so
    # P B_c = B_f there, exactly as for the tentative prolongator
    _, sa, _ = pair
    L0, L1 = sa
    Bf, Bc = L0.nullspace_u, L1.nullspace_u
    KB = np.abs(L0.K @ Bf).max(axis=1)
    free = (KB <= 1e-12 * np.abs(L0.K).max() * np.abs(Bf).max()) & ~L0.dirichlet
    assert free.sum() > L0.n_u // 2
    err = np.abs((L0.P_u @ Bc - Bf)[free]).max()
    assert err <= 1e-12 * np.abs(Bf).max()
    # and the smoothing does change the other rows
    assert np.abs((L0.P_u @ Bc - Bf)[~free & ~L0.dirichlet]).max() > 1e-6


def test_smoothed_prolongator_lowers_column_energy(pair):
    # ||(I - w Atilde^-1 K) p||_K <= ||p||_K for w = 4/3 because every
    # eigenvalue mu of Atilde^-1 K is in [0, 1]: |1 - w mu| <= 1
    _, sa, pa = pair
    K = sa[0].K
    Pt, Ps = pa[0].P_u, sa[0].P_u
    eT = np.einsum("ij,ij->j", Pt.toarray(), (K @ Pt).toarray())
    eS = np.einsum("ij,ij->j", Ps.toarray(), (K @ Ps).toarray())
    assert np.all(eS <= eT * (1 + 1e-12))
    assert np.median(eS / eT) < 0.9


def test_smoothed_galerkin_matches_dense_triple_product(pair):
    _, sa, _ = pair
    L0, L1 = sa
    P = L0.P_u.toarray()
    for blk, Pl, Pr in (("K", P, P), ("G", P, L0.P_l.toarray()), ("B", L0.P_l.toarray(), P)):
        ref = Pl.T @ getattr(L0, blk).toarray() @ Pr
        got = getattr(L1, blk).toarray()
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max()), blk
    # pattern: symbolic product, so it contains the numerically nonzero entries
    Kc = galerkin(L0.P_u.T.tocsr(), L0.K, L0.P_u)
    assert Kc.nnz == L1.K.nnz


def test_l1_schur_jacobi_is_convergent(pair):
    # signed l1 lumping: the Jacobi iteration matrix I - D^-1 S is a
    # contraction on every case
    _, sa, _ = pair
    L = sa[0]
    S = L.S.toarray()
    rho = np.abs(np.linalg.eigvals(np.eye(len(S)) - S * L.sd_inv[:, None])).max()
    assert rho < 0.95


def test_diagonal_schur_jacobi_diverges_under_contrast():
    # the reason for the l1 option: on the lognormal(0, 2) curved case the
    # exact diagonal of S gives a Jacobi iteration matrix with spectral
    # radius above one (the mortar M couplings dominate D where the master
    # side is much softer), while the l1 lumping stays a contraction
    p = make_workload("contact3d_150_curved", slave_elems=(10, 10, 10), master_elems=(11, 11, 10))
    L = build_hierarchy(p, AMGOptions(max_levels=2, schur="diag", schur_sweeps=2))[0]
    S = L.S.toarray()
    I = np.eye(len(S))
    rho_diag = np.abs(np.linalg.eigvals(I - S / np.diag(S)[:, None])).max()
    L1 = build_hierarchy(p, AMGOptions(max_levels=2, schur="l1", schur_sweeps=2))[0]
    rho_l1 = np.abs(np.linalg.eigvals(I - S * L1.sd_inv[:, None])).max()
    assert rho_diag > 1.05 and rho_l1 < 0.95


def test_many_schur_sweeps_give_exact_simple_constraints():
    # with alpha = 1 and the exact Schur complement of the lumped system the
    # constraint rows hold after one sweep whatever the prediction
    # (Sec. 5.1.3); enough l1 Jacobi sweeps on S reproduce that to rounding
    p = make_workload("contact3d_6")
    L = build_hierarchy(p, AMGOptions(max_levels=2, schur="l1", schur_sweeps=80))[0]
    rng = np.random.default_rng(5)
    b = rng.standard_normal(L.n)
    z = cheap_simple_sweep(L, b, np.zeros(L.n), 0.8, 1.0, schur_sweeps=80)
    rl = b[L.n_u:] - (L.B @ z[: L.n_u] + L.C @ z[L.n_u:])
    assert np.abs(rl).max() <= 1e-12 * np.abs(b).max()
    # one sweep (plain division) does not
    z1 = cheap_simple_sweep(L, b, np.zeros(L.n), 0.8, 1.0, schur_sweeps=1)
    rl1 = b[L.n_u:] - (L.B @ z1[: L.n_u] + L.C @ z1[L.n_u:])
    assert np.abs(rl1).max() > 1e-4 * np.abs(b).max()


def test_robust_vcycle_transpose_dot_product(pair):
    _, sa, _ = pair
    o = AMGOptions(max_levels=2, **ROBUST)
    n = sa[0].n
    rng = np.random.default_rng(11)
    x, y = rng.standard_normal(n), rng.standard_normal(n)
    a1 = y @ vcycle(sa, x, o)
    a2 = vcycle(sa, y, o, transpose=True) @ x
    assert abs(a1 - a2) <= 1e-12 * abs(a1)


def test_robust_settings_converge_under_contrast():
    # the lognormal(0, 2) curved case at 10^3: the robust settings converge in
    # fewer iterations than the plain ones (whose smoother diverges there)
    p = make_workload("contact3d_150_curved", slave_elems=(10, 10, 10), master_elems=(11, 11, 10))
    o = AMGOptions(max_levels=2, prolongator="sa", schur="l1", schur_sweeps=2, jacobi_sweeps=3)
    r = solve(build_hierarchy(p, o), o, p.b, rtol=1e-8, max_iters=400)
    base = AMGOptions(max_levels=2)
    r0 = solve(build_hierarchy(p, base), base, p.b, rtol=1e-8, max_iters=400)
    assert r.converged and r.rel_res_true <= 1e-8
    assert r.iters < r0.iters


def _simple_coarse(**kw):
    return AMGOptions(max_levels=2, coarse_solver="simple", **kw)


def test_simple_coarse_solver_is_k_stationary_steps():
    # k smoother sweeps from zero as the coarse "solve": with the one-sweep
    # matrix Q^-1 (a sweep from zero) the k-step operator has the closed form
    # M_k = (I - (I - Q^-1 A)^k) A^-1.  One-level hierarchy of the 2D workload
    # (the coarsest level is the whole system), dense check.
    p = make_workload("contact2d_16")
    o = AMGOptions(max_levels=1, coarse_solver="simple", coarse_sweeps=3)
    lv = build_hierarchy(p, o)
    assert len(lv) == 1 and lv[0].A_inv is None
    L = lv[0]
    A = L.A().toarray()
    n = A.shape[0]
    I = np.eye(n)
    Qinv = np.column_stack([cheap_simple_sweep(L, e, np.zeros(n), o.jacobi_omega, o.simple_alpha) for e in I])
    Mk = (I - np.linalg.matrix_power(I - Qinv @ A, 3)) @ np.linalg.inv(A)
    r = np.random.default_rng(2).standard_normal(n)
    z = vcycle(lv, r, o)
    assert np.linalg.norm(z - Mk @ r) <= 1e-10 * np.linalg.norm(z)
    zt = vcycle(lv, r, o, transpose=True)
    assert np.linalg.norm(zt - Mk.T @ r) <= 1e-10 * np.linalg.norm(zt)


@pytest.mark.parametrize("sweeps", [1, 2, 3])
def test_simple_coarse_solver_transpose_dot_product(sweeps):
    p = make_workload("contact3d_6")
    o = AMGOptions(max_levels=2, coarse_solver="simple", coarse_sweeps=sweeps, schur="l1", schur_sweeps=2)
    lv = build_hierarchy(p, o)
    rng = np.random.default_rng(13)
    x, y = rng.standard_normal(p.n), rng.standard_normal(p.n)
    a1 = y @ vcycle(lv, x, o)
    a2 = vcycle(lv, y, o, transpose=True) @ x
    assert abs(a1 - a2) <= 1e-12 * abs(a1)


def test_simple_coarse_solver_needs_no_factorisation():
    # the 3-level 6^3 hierarchy's merged coarsest matrix is singular, so the
    # LU variant cannot be built; the smoother variant builds (no merge, no
    # factorisation)
    from oracle.hierarchy import SingularCoarse

    p = make_workload("contact3d_6")
    with pytest.raises(SingularCoarse):
        build_hierarchy(p, AMGOptions(max_levels=3, max_coarse_rows=10))
    lv = build_hierarchy(p, AMGOptions(max_levels=3, max_coarse_rows=10, coarse_solver="simple"))
    assert len(lv) == 3 and lv[-1].A_inv is None and lv[-1].sd_inv is not None


# ---- standard (non-dual) multiplier basis: Alg. 1 with a non-diagonal D ----


@pytest.mark.parametrize("kappa", [2, 3])
def test_alg1_first_assignment_with_nondiagonal_D(kappa):
    # brute force of the rule: a multiplier pseudo-node joins the aggregate
    # d(k) of the first slave dof (ascending) that couples to it, so two
    # pseudo-nodes share a multiplier aggregate exactly when their first
    # coupled slave dofs lie in the same displacement aggregate; no
    # multiplier aggregate is empty
    from contactgen import weak_scaling_problem

    p = weak_scaling_problem(kappa)
    L = build_hierarchy(p, AMGOptions(max_levels=2, max_coarse_rows=50))[0]
    G = L.G.tocsc()
    first = {}
    for j in range(L.n_l):
        rows = G.indices[G.indptr[j]:G.indptr[j + 1]]
        assert rows.size > 1 or kappa == 0  # D is not diagonal
        pn = L.lm_node[j]
        i = rows.min()
        first[pn] = min(first.get(pn, i), i)
    key = {pn: L.agg_u[i // L.bs_u] for pn, i in first.items()}
    pns = sorted(first)
    for a in pns:
        for b in pns:
            assert (L.agg_l[a] == L.agg_l[b]) == (key[a] == key[b])
    counts = np.bincount(L.agg_l)
    assert counts.min() > 0 and counts.size == L.agg_l.max() + 1


def test_standard_basis_hierarchy_and_solve():
    from contactgen import weak_scaling_problem

    p = weak_scaling_problem(3)
    for o in (AMGOptions(max_levels=3, max_coarse_rows=100),
              AMGOptions(max_levels=3, max_coarse_rows=100, prolongator="sa", nu_pre=3, nu_post=3)):
        lv = build_hierarchy(p, o)
        assert len(lv) == 3
        rng = np.random.default_rng(17)
        x, y = rng.standard_normal(p.n), rng.standard_normal(p.n)
        a1 = y @ vcycle(lv, x, o)
        a2 = vcycle(lv, y, o, transpose=True) @ x
        assert abs(a1 - a2) <= 1e-12 * abs(a1)
        r = solve(lv, o, p.b, rtol=1e-8, max_iters=400)
        assert r.converged and r.rel_res_true <= 1e-8
