"""Pins for the oracle's CheapSIMPLE sweep (CPU) against the paper's matrix
statements for SIMPLE (Sec. 5.1.3) and the increment form of Sec. 5.1."""
import numpy as np
import pytest

from contactgen import make_contact_problem, make_workload
from oracle.hierarchy import AMGOptions, build_hierarchy
from oracle.smoother import cheap_simple_sweep, cheap_simple_sweep_adjoint


@pytest.fixture(scope="module")
def level2d():
    p = make_workload("contact2d_16")
    opts = AMGOptions(max_levels=2, nu_pre=1, nu_post=1)
    lv = build_hierarchy(p, opts)
    return p, lv[0], opts


def _sweep_matrix(L, n, fn):
    return np.column_stack([fn(e) for e in np.eye(n)])


def test_sweep_equals_inverse_of_simple_factorisation(level2d):
    # Q = [[J^-1, 0], [B, -S]] [[I, Atilde^-1 G], [0, I/alpha]] with the cheap inverses
    # J = omega D^-1 (one Jacobi sweep) and the diagonal S; one sweep from z = 0 is Q^-1 b
    p, L, opts = level2d
    om, al = opts.jacobi_omega, opts.simple_alpha
    n_u, n_l = L.n_u, L.n_l
    Jinv = np.diag(1.0 / (om * L.dinv))
    S = np.diag(1.0 / L.sd_inv)
    left = np.block([[Jinv, np.zeros((n_u, n_l))], [L.B.toarray(), -S]])
    right = np.block([[np.eye(n_u), L.atilde_inv[:, None] * L.G.toarray()], [np.zeros((n_l, n_u)), np.eye(n_l) / al]])
    Q = left @ right
    n = n_u + n_l
    M = _sweep_matrix(L, n, lambda e: cheap_simple_sweep(L, e, np.zeros(n), om, al))
    assert np.abs(M @ Q - np.eye(n)).max() < 1e-9


def test_sweep_is_increment_form(level2d):
    # z <- z + Q^-1 (b - A z)
    p, L, opts = level2d
    n = L.n
    rng = np.random.default_rng(0)
    b, z = rng.standard_normal(n), rng.standard_normal(n)
    A = L.A()
    lhs = cheap_simple_sweep(L, b, z, opts.jacobi_omega, opts.simple_alpha)
    rhs = z + cheap_simple_sweep(L, b - A @ z, np.zeros(n), opts.jacobi_omega, opts.simple_alpha)
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(lhs).max()


@pytest.fixture(scope="module")
def level2d_clamped():
    # both outer faces clamped: K alone is nonsingular, so exact predictions exist
    p = make_contact_problem(2, (10, 10), (11, 10), top_bc="clamped")
    opts = AMGOptions(max_levels=2, max_coarse_rows=10, nu_pre=1, nu_post=1)
    lv = build_hierarchy(p, opts)
    return p, lv[0], opts


def test_exact_simple_satisfies_constraints_in_one_sweep(level2d_clamped):
    # exact Schur approximation S = B Atilde^-1 G - C and alpha = 1: the constraint rows
    # hold after one sweep, for any prediction
    p, L, opts = level2d_clamped
    Sfull = (L.B.toarray() * L.atilde_inv[None, :]) @ L.G.toarray() - L.C.toarray()
    rng = np.random.default_rng(1)
    b, z = rng.standard_normal(L.n), rng.standard_normal(L.n)
    for predict in (None, lambda r: np.linalg.solve(L.K.toarray(), r)):
        out = cheap_simple_sweep(L, b, z, opts.jacobi_omega, 1.0, predict=predict,
                                 schur_solve=lambda r: np.linalg.solve(Sfull, r))
        rl = b[L.n_u:] - (L.B @ out[:L.n_u] + L.C @ out[L.n_u:])
        assert np.abs(rl).max() < 1e-10 * np.abs(b).max()


def test_exact_prediction_kills_displacement_errors(level2d_clamped):
    # with an exact prediction the SIMPLE error matrix has a zero first block column:
    # an error living only in the displacements is removed by one sweep
    p, L, opts = level2d_clamped
    A = L.A().toarray()
    rng = np.random.default_rng(2)
    x = rng.standard_normal(L.n)
    b = A @ x
    e = np.zeros(L.n)
    e[:L.n_u] = rng.standard_normal(L.n_u)
    Kd = L.K.toarray()
    out = cheap_simple_sweep(L, b, x + e, opts.jacobi_omega, opts.simple_alpha,
                             predict=lambda r: np.linalg.solve(Kd, r))
    assert np.abs(out - x).max() < 1e-8 * np.abs(x).max()


def test_adjoint_sweep_is_transpose(level2d):
    p, L, opts = level2d
    n = L.n
    om, al = opts.jacobi_omega, opts.simple_alpha
    for js in (1, 2):
        M = _sweep_matrix(L, n, lambda e: cheap_simple_sweep(L, e, np.zeros(n), om, al, js))
        MT = _sweep_matrix(L, n, lambda e: cheap_simple_sweep_adjoint(L, e, np.zeros(n), om, al, js))
        assert np.abs(M.T - MT).max() < 1e-12 * np.abs(M).max()


# ---- Uzawa and Braess-Sarazin sweeps (Sec. 5.1.1, Sec. 5.1.2) ----

from oracle.smoother import (braess_sarazin_sweep, braess_sarazin_sweep_adjoint,  # noqa: E402
                             cheap_uzawa_sweep, cheap_uzawa_sweep_adjoint)


def test_uzawa_sweep_inverts_the_uzawa_matrix(level2d):
    # one sweep from zero is Q_U^-1 b with Q_U = (1/alpha) [[J^-1, 0], [B, -S]]
    # (the Uzawa matrix with the cheap inverses: one damped Jacobi step for
    # K, the diagonal Schur approximation)
    p, L, opts = level2d
    om, al = opts.jacobi_omega, 0.7
    n_u, n_l, n = L.n_u, L.n_l, L.n
    Q = np.block([[np.diag(1.0 / (om * L.dinv)), np.zeros((n_u, n_l))], [L.B.toarray(), -np.diag(1.0 / L.sd_inv)]]) / al
    M = _sweep_matrix(L, n, lambda e: cheap_uzawa_sweep(L, e, np.zeros(n), om, al))
    assert np.abs(M @ Q - np.eye(n)).max() < 1e-9


def test_uzawa_error_matrix(level2d_clamped):
    # with alpha = 1, an exact prediction and the exact Schur approximation
    # S = B Ahat^-1 G - C the error matrix A - Q_U is [[0, G], [0, B Ahat^-1 G]]
    # (so the constraint rows keep a systematic error)
    p, L, opts = level2d_clamped
    n_u, n = L.n_u, L.n
    Kd = L.K.toarray()
    AhG = L.atilde_inv[:, None] * L.G.toarray()
    S = L.B.toarray() @ AhG - L.C.toarray()
    M = _sweep_matrix(L, n, lambda e: cheap_uzawa_sweep(L, e, np.zeros(n), opts.jacobi_omega, 1.0,
                                                         predict=lambda r: np.linalg.solve(Kd, r),
                                                         schur_solve=lambda r: np.linalg.solve(S, r)))
    E = L.A().toarray() - np.linalg.inv(M)
    ref = np.zeros((n, n))
    ref[:n_u, n_u:] = L.G.toarray()
    ref[n_u:, n_u:] = L.B.toarray() @ AhG
    assert np.abs(E - ref).max() < 1e-8 * np.abs(ref).max()


def test_braess_sarazin_sweep_inverts_its_factorisation(level2d):
    # one sweep from zero is the inverse of
    # [[alpha Ahat, 0], [B, -S_d]] [[I, Ahat^-1 G / alpha], [0, I]]
    # with S_d the diagonal of S_a = B Ahat^-1 G / alpha - C
    p, _, _ = level2d
    al = 1.9
    o = AMGOptions(max_levels=2, nu_pre=1, nu_post=1, smoother="braess_sarazin", simple_alpha=al)
    L = build_hierarchy(p, o)[0]
    n_u, n_l, n = L.n_u, L.n_l, L.n
    Ah = np.diag(1.0 / L.atilde_inv)
    left = np.block([[al * Ah, np.zeros((n_u, n_l))], [L.B.toarray(), -np.diag(1.0 / L.extra["bs_sd_inv"])]])
    right = np.block([[np.eye(n_u), (L.atilde_inv[:, None] * L.G.toarray()) / al], [np.zeros((n_l, n_u)), np.eye(n_l)]])
    M = _sweep_matrix(L, n, lambda e: braess_sarazin_sweep(L, e, np.zeros(n), al))
    assert np.abs(M @ (left @ right) - np.eye(n)).max() < 1e-9
    # the diagonal is that of S_a
    Sa = (L.B.toarray() * L.atilde_inv[None, :]) @ L.G.toarray() / al - L.C.toarray()
    assert np.allclose(1.0 / L.extra["bs_sd_inv"], np.diag(Sa), rtol=1e-13, atol=0)


def test_braess_sarazin_error_matrix(level2d):
    # with the exact S_a the error matrix is [[K - alpha Ahat, 0], [0, 0]]:
    # the constraint rows hold exactly after every sweep
    p, _, _ = level2d
    al = 1.9
    o = AMGOptions(max_levels=2, nu_pre=1, nu_post=1, smoother="braess_sarazin", simple_alpha=al)
    L = build_hierarchy(p, o)[0]
    n_u, n = L.n_u, L.n
    Sa = (L.B.toarray() * L.atilde_inv[None, :]) @ L.G.toarray() / al - L.C.toarray()
    M = _sweep_matrix(L, n, lambda e: braess_sarazin_sweep(L, e, np.zeros(n), al,
                                                           schur_solve=lambda r: np.linalg.solve(Sa, r)))
    E = L.A().toarray() - np.linalg.inv(M)
    ref = np.zeros((n, n))
    ref[:n_u, :n_u] = L.K.toarray() - al * np.diag(1.0 / L.atilde_inv)
    assert np.abs(E - ref).max() < 1e-8 * np.abs(ref).max()


@pytest.mark.parametrize("smoother,alpha", [("uzawa", 0.7), ("braess_sarazin", 1.9)])
def test_uzawa_and_braess_sarazin_adjoints_are_transposes(level2d, smoother, alpha):
    p, _, _ = level2d
    o = AMGOptions(max_levels=2, nu_pre=1, nu_post=1, smoother=smoother, simple_alpha=alpha)
    L = build_hierarchy(p, o)[0]
    n = L.n
    if smoother == "uzawa":
        fwd = lambda e: cheap_uzawa_sweep(L, e, np.zeros(n), o.jacobi_omega, alpha)
        adj = lambda e: cheap_uzawa_sweep_adjoint(L, e, np.zeros(n), o.jacobi_omega, alpha)
    else:
        fwd = lambda e: braess_sarazin_sweep(L, e, np.zeros(n), alpha)
        adj = lambda e: braess_sarazin_sweep_adjoint(L, e, np.zeros(n), alpha)
    M, MT = _sweep_matrix(L, n, fwd), _sweep_matrix(L, n, adj)
    assert np.abs(M.T - MT).max() < 1e-12 * np.abs(M).max()


@pytest.mark.parametrize("smoother,alpha,sweeps", [("uzawa", 0.7, 3), ("braess_sarazin", 1.9, 3)])
def test_uzawa_and_braess_sarazin_converge(smoother, alpha, sweeps):
    # the paper's block-smoother comparison settings (three sweeps, damping
    # 0.7 / 1.9) as preconditioners on the 3D 6^3 workload
    from oracle.adjoint import solve

    p = make_workload("contact3d_6")
    o = AMGOptions(max_levels=2, smoother=smoother, simple_alpha=alpha, nu_pre=sweeps, nu_post=sweeps)
    r = solve(build_hierarchy(p, o), o, p.b, rtol=1e-8, max_iters=400)
    assert r.converged and r.rel_res_true <= 1e-8
