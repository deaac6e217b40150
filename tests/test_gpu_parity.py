"""GPU parity of libcamg against the CPU oracle (run on an MI355X).

Every call goes through the C-ABI (ctypes binding); the oracle runs on the
CPU on the same seeded inputs.  Tolerances:
  * FP64 operator apply: 1e-14 relative (only summation order differs);
  * FP64 V-cycle: 1e-12 relative;
  * FP64 FGMRES at a fixed iteration count: 1e-10 relative;
  * mixed FP32/FP64: the solve reaches the same 1e-8 relative residual and
    the solution differs from a 1e-12 FP64 reference by < 1e-7 relative.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl
import torch

from contactgen import make_contact_problem, make_workload
from oracle.adjoint import grad_K_values, solve as oracle_solve
from oracle.hierarchy import AMGOptions as OracleOptions
from oracle.hierarchy import build_hierarchy
from oracle.vcycle import _apply_A, vcycle as oracle_vcycle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_09056_amd.camg import load_library

    load_library()  # fails loudly when the HIP library is missing


def _solver(prob, precision=0, fmt=0, **kw):
    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver

    return AMGSolver.from_problem(prob, AMGOptions(precision=precision, spmv_format=fmt, **kw))


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# robustness settings: smoothed aggregation, l1-lumped Schur sweeps, 3 Jacobi sweeps
ROBUST_ORACLE = dict(prolongator="sa", schur="l1", schur_sweeps=3, jacobi_sweeps=3)
ROBUST_LIB = dict(prolongator=1, schur=1, schur_sweeps=3, jacobi_sweeps=3)
CURVED6 = dict(slave_elems=(6, 6, 6), master_elems=(7, 7, 6))

# (workload, shared options, K storage on the device: 1 CSR, 2 sliced
#  blocked-ELL, [oracle-only options, library-only options, generator overrides])
CASES = {
    "2d-csr": ("contact2d_16", dict(max_levels=2, nu_pre=1, nu_post=1), 1),
    "2d-bell": ("contact2d_16", dict(max_levels=2, nu_pre=1, nu_post=1), 2),
    "3d6-csr": ("contact3d_6", dict(max_levels=2), 1),
    "3d6-bell": ("contact3d_6", dict(max_levels=2), 2),
    "3d6-robust-csr": ("contact3d_6", dict(max_levels=2), 1, ROBUST_ORACLE, ROBUST_LIB, {}),
    "curved6-robust-bell": ("contact3d_150_curved", dict(max_levels=2), 2, ROBUST_ORACLE, ROBUST_LIB, CURVED6),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    name, kw, fmt, *extra = CASES[request.param]
    okw, lkw, gen = extra if extra else ({}, {}, {})
    prob = make_workload(name, **gen)
    oopts = OracleOptions(**kw, **okw)
    lv = build_hierarchy(prob, oopts)
    print(f"[case] {request.param}: {name} {kw} {lkw} fmt={fmt}", flush=True)
    return prob, lv, oopts, dict(kw, fmt=fmt, **lkw)


def test_operator_apply(case):
    prob, lv, oopts, kw = case
    s = _solver(prob, **kw)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(prob.n)
    A = prob.full_matrix()
    for tr, ref in ((False, A @ x), (True, A.T @ x)):
        y = s.apply_operator(torch.from_numpy(x), transpose=tr).cpu().numpy()
        assert _rel(y, ref) < 1e-14


def test_vcycle_fp64(case):
    prob, lv, oopts, kw = case
    s = _solver(prob, **kw)
    rng = np.random.default_rng(1)
    for tr in (False, True):
        r = rng.standard_normal(prob.n)
        z = s.vcycle(torch.from_numpy(r), transpose=tr).cpu().numpy()
        ref = oracle_vcycle(lv, r, oopts, transpose=tr)
        assert _rel(z, ref) < 1e-12, tr


def test_vcycle_deterministic(case):
    prob, lv, oopts, kw = case
    s = _solver(prob, **kw)
    r = torch.from_numpy(np.random.default_rng(2).standard_normal(prob.n))
    z1 = s.vcycle(r).cpu().numpy()
    z2 = s.vcycle(r).cpu().numpy()
    assert np.array_equal(z1, z2)


def test_vcycle_mixed(case):
    prob, lv, oopts, kw = case
    s = _solver(prob, precision=1, **kw)
    rng = np.random.default_rng(3)
    for tr in (False, True):
        r = rng.standard_normal(prob.n)
        z = s.vcycle(torch.from_numpy(r), transpose=tr).cpu().numpy()
        ref = oracle_vcycle(lv, r, oopts, transpose=tr)
        assert _rel(z, ref) < 2e-5, tr


def test_fgmres_fixed_iterations_fp64(case):
    prob, lv, oopts, kw = case
    s = _solver(prob, **kw)
    for tr in (False, True):
        # (45, 50) runs the widest CGS2 kernels (up to 64 basis vectors per pass)
        for k, m in ((7, 50), (23, 10), (45, 50)):
            ref = oracle_solve(lv, oopts, prob.b, transpose=tr, m=m, fixed_iters=k)
            x, info = s.solve(torch.from_numpy(prob.b), transpose=tr, m=m, fixed_iters=k)
            assert info["iters"] == k
            assert _rel(x.cpu().numpy(), ref.x) < 1e-10, (tr, k, m)
            # the true residual at 45 steps sits near the FP64 rounding floor of
            # b - A x (about 1e-13 of ||b||), where the two codes' summation orders differ
            assert abs(info["rel_res_true"] - ref.rel_res_true) <= 1e-8 * ref.rel_res_true + 1e-13


def test_fgmres_converges_fp64_and_mixed(case):
    prob, lv, oopts, kw = case
    A = prob.full_matrix().tocsc()
    x_exact = spl.spsolve(A, prob.b)
    ref = oracle_solve(lv, oopts, prob.b, rtol=1e-8)
    for prec in (0, 1):
        s = _solver(prob, precision=prec, **kw)
        x, info = s.solve(torch.from_numpy(prob.b), rtol=1e-8)
        x = x.cpu().numpy()
        print(f"[solve] prec={prec} iters={info['iters']} oracle={ref.iters} rel={info['rel_res_true']:.2e}",
              flush=True)
        assert info["converged"] and info["rel_res_true"] <= 1e-8
        assert np.linalg.norm(prob.b - A @ x) <= 1.0001e-8 * np.linalg.norm(prob.b)
        if prec == 0:
            assert abs(info["iters"] - ref.iters) <= 1
        x12, info12 = s.solve(torch.from_numpy(prob.b), rtol=1e-12)
        assert info12["converged"]
        assert _rel(x12.cpu().numpy(), x_exact) < 1e-9


def test_mixed_solution_error(case):
    prob, lv, oopts, kw = case
    x_ref = oracle_solve(lv, oopts, prob.b, rtol=1e-12).x
    s = _solver(prob, precision=1, **kw)
    x, info = s.solve(torch.from_numpy(prob.b), rtol=1e-8)
    err = _rel(x.cpu().numpy(), x_ref)
    print(f"[mixed] iters={info['iters']} err_vs_fp64_1e-12={err:.2e}", flush=True)
    assert info["converged"] and err < 1e-7


def test_grad_K_kernel(case):
    prob, lv, oopts, kw = case
    s = _solver(prob, **kw)
    rng = np.random.default_rng(4)
    lam, x = rng.standard_normal(prob.n), rng.standard_normal(prob.n)
    dK = s.grad_K(torch.from_numpy(lam), torch.from_numpy(x)).cpu().numpy()
    ref = grad_K_values(prob.K, lam[: prob.n_u], x[: prob.n_u])
    assert np.array_equal(dK, ref)


def test_grad_A_kernel(case):
    """-lam_i x_j on the stored entries of all four blocks, against the
    oracle's outer product on each block's pattern (row part of lam, column
    part of x)."""
    prob, lv, oopts, kw = case
    s = _solver(prob, **kw)
    rng = np.random.default_rng(14)
    lam, x = rng.standard_normal(prob.n), rng.standard_normal(prob.n)
    out = s.grad_A(torch.from_numpy(lam), torch.from_numpy(x))
    nu = prob.n_u
    parts = dict(K=(prob.K, lam[:nu], x[:nu]), G=(prob.G, lam[:nu], x[nu:]), B=(prob.B, lam[nu:], x[:nu]),
                 C=(prob.C, lam[nu:], x[nu:]))
    for name, (M, lr, xc) in parts.items():
        ref = grad_K_values(M.tocsr(), lr, xc)
        assert np.array_equal(out[name].cpu().numpy(), ref), name


def _dense_block_grads(prob, x, lam):
    nu = prob.n_u
    out = {}
    for name, M, lr, xc in (("K", prob.K, lam[:nu], x[:nu]), ("G", prob.G, lam[:nu], x[nu:]),
                            ("B", prob.B, lam[nu:], x[:nu]), ("C", prob.C, lam[nu:], x[nu:])):
        M = M.tocsr()
        D = -np.outer(lr, xc)  # dense -lam x^T of this block
        rows = np.repeat(np.arange(M.shape[0]), np.diff(M.indptr))
        out[name] = D[rows, M.indices]
    return out


def test_autograd_all_blocks_dense_reference():
    """dL/dK, dL/dG, dL/dB, dL/dC and dL/db of L = 0.5 ||u_top||^2 against
    the dense outer product -lam x^T of numpy's direct solves, sampled on each
    block's pattern (6^3 workload, both precisions)."""
    from paper_1912_09056_amd import contact_solve

    prob = make_workload("contact3d_6")
    A = prob.full_matrix().toarray()
    top = prob.top_dofs
    x_ref = np.linalg.solve(A, prob.b)
    g = np.zeros(prob.n)
    g[top] = x_ref[top]
    lam_ref = np.linalg.solve(A.T, g)
    ref = _dense_block_grads(prob, x_ref, lam_ref)
    tt = torch.from_numpy(top).cuda()
    for prec in (0, 1):
        s = _solver(prob, precision=prec, fmt=2, max_levels=2)
        t = {name: torch.tensor(M.tocsr().data, dtype=torch.float64, device="cuda", requires_grad=True)
             for name, M in (("K", prob.K), ("G", prob.G), ("B", prob.B), ("C", prob.C))}
        b = torch.tensor(prob.b, dtype=torch.float64, device="cuda", requires_grad=True)
        x = contact_solve(s, t["K"], b, rtol=1e-12, G_val=t["G"], B_val=t["B"], C_val=t["C"])
        (0.5 * (x[tt] ** 2).sum()).backward()
        assert _rel(x.detach().cpu().numpy(), x_ref) < 1e-10
        assert _rel(b.grad.cpu().numpy(), lam_ref) < 1e-9
        for name in ("K", "G", "B", "C"):
            assert _rel(t[name].grad.cpu().numpy(), ref[name]) < 1e-9, (prec, name)


def test_grad_coupling_blocks_central_differences():
    """Central differences (h = 1e-6) of L = 0.5 ||u_top||^2 through the
    library's FP64 solve, for 6 seeded stored entries of each of G, B and C,
    against amg_grad_A; the bar is 1e-6 relative to each entry, with a floor
    of 1e-3 of the block gradient's largest entry."""
    from paper_1912_09056_amd import contact_solve

    prob = make_workload("contact3d_6")
    s = _solver(prob, fmt=2, max_levels=2)
    tt = torch.from_numpy(prob.top_dofs).cuda()
    vals = {name: torch.tensor(M.tocsr().data, dtype=torch.float64, device="cuda")
            for name, M in (("K", prob.K), ("G", prob.G), ("B", prob.B), ("C", prob.C))}
    b = torch.from_numpy(prob.b).cuda()
    t = {name: v.clone().requires_grad_(True) for name, v in vals.items()}
    x = contact_solve(s, t["K"], b, rtol=1e-13, G_val=t["G"], B_val=t["B"], C_val=t["C"])
    (0.5 * (x[tt] ** 2).sum()).backward()

    x0 = x.detach()

    def loss(name, v):
        with torch.no_grad():
            s.update_fine_values(**{f"{name}_val": v})
            # warm start: reduce the O(h) initial residual by 1e-9, not below
            # the operator's FP64 rounding floor (about 1e-13 of ||b||)
            r0 = float((b - s.apply_operator(x0)).norm())
            xx, info = s.solve(b, x0=x0, rtol=max(1e-9, 2e-13 * float(b.norm()) / r0))
            assert info["converged"], info
            s.update_fine_values(**{f"{name}_val": vals[name]})
            return 0.5 * float((xx[tt] ** 2).sum())

    rng = np.random.default_rng(21)
    h = 1e-6
    for name in ("G", "B", "C"):
        gA = t[name].grad.cpu().numpy()
        for k in rng.choice(gA.size, 6, replace=False):
            e = torch.zeros_like(vals[name])
            e[k] = h
            fd = (loss(name, vals[name] + e) - loss(name, vals[name] - e)) / (2 * h)
            bar = 1e-6 * max(abs(fd), 1e-3 * np.abs(gA).max())
            print(f"[fdA] d{name}[{k}] adjoint {gA[k]:+.10e} fd {fd:+.10e}", flush=True)
            assert abs(fd - gA[k]) <= bar, (name, k, fd, gA[k])


@pytest.mark.parametrize("fmt", [1, 2])
def test_autograd_dense_reference(fmt):
    from paper_1912_09056_amd import contact_solve

    prob = make_workload("contact3d_6")
    kw = dict(max_levels=2)
    A = prob.full_matrix().toarray()
    top = prob.top_dofs
    x_ref = np.linalg.solve(A, prob.b)
    g = np.zeros(prob.n)
    g[top] = x_ref[top]
    lam_ref = np.linalg.solve(A.T, g)
    rows = np.repeat(np.arange(prob.n_u), np.diff(prob.K.indptr))
    gK_ref = -lam_ref[rows] * x_ref[prob.K.indices]
    for prec in (0, 1):
        s = _solver(prob, precision=prec, fmt=fmt, **kw)
        Kv = torch.tensor(prob.K.data, dtype=torch.float64, device="cuda", requires_grad=True)
        b = torch.tensor(prob.b, dtype=torch.float64, device="cuda", requires_grad=True)
        x = contact_solve(s, Kv, b, rtol=1e-12)
        loss = 0.5 * (x[torch.from_numpy(top).cuda()] ** 2).sum()
        loss.backward()
        assert _rel(x.detach().cpu().numpy(), x_ref) < 1e-10
        assert _rel(b.grad.cpu().numpy(), lam_ref) < 1e-9
        assert _rel(Kv.grad.cpu().numpy(), gK_ref) < 1e-9


def test_autograd_backward_uses_its_forward_operator():
    """Two forwards with different K values, then the backward of the first:
    the adjoint solve and dL/dK use the first forward's operator (the dense
    reference of K1), not the values the second forward left in the solver."""
    from paper_1912_09056_amd import contact_solve

    prob = make_workload("contact3d_6")
    top = prob.top_dofs
    s = _solver(prob, fmt=2, max_levels=2)
    K1 = prob.K.copy()
    K2 = prob.K.copy()
    # same pattern, other values (not symmetric: FGMRES needs no symmetry)
    K2.data = K2.data * (1.0 + 0.2 * np.random.default_rng(31).random(K2.nnz))
    A1 = sp.bmat([[K1, prob.G], [prob.B, prob.C]]).toarray()
    x_ref = np.linalg.solve(A1, prob.b)
    g = np.zeros(prob.n)
    g[top] = x_ref[top]
    lam_ref = np.linalg.solve(A1.T, g)
    rows = np.repeat(np.arange(prob.n_u), np.diff(K1.indptr))
    gK_ref = -lam_ref[rows] * x_ref[K1.indices]
    Kv1 = torch.tensor(K1.data, dtype=torch.float64, device="cuda", requires_grad=True)
    Kv2 = torch.tensor(K2.data, dtype=torch.float64, device="cuda", requires_grad=True)
    b = torch.tensor(prob.b, dtype=torch.float64, device="cuda", requires_grad=True)
    tt = torch.from_numpy(top).cuda()
    x1 = contact_solve(s, Kv1, b, rtol=1e-12)
    x2 = contact_solve(s, Kv2, b, rtol=1e-12)
    assert _rel(x1.detach().cpu().numpy(), x_ref) < 1e-10
    assert _rel(x2.detach().cpu().numpy(), x_ref) > 1e-3  # the second operator differs
    (0.5 * (x1[tt] ** 2).sum()).backward()
    assert _rel(b.grad.cpu().numpy(), lam_ref) < 1e-9
    assert _rel(Kv1.grad.cpu().numpy(), gK_ref) < 1e-9
    assert Kv2.grad is None


@pytest.mark.parametrize("fmt", [1, 2])
def test_finite_differences_gpu(fmt):
    # central differences with step 1e-6 on seeded entries of b and of K's nonzeros;
    # the bar is 1e-6 of the gradient's largest entry (FD accuracy on stiff entries)
    from paper_1912_09056_amd import contact_solve

    prob = make_workload("contact3d_6")
    s = _solver(prob, fmt=fmt, max_levels=2)
    top = torch.from_numpy(prob.top_dofs).cuda()
    Kv0 = torch.tensor(prob.K.data, dtype=torch.float64, device="cuda", requires_grad=True)
    b0 = torch.tensor(prob.b, dtype=torch.float64, device="cuda", requires_grad=True)
    x = contact_solve(s, Kv0, b0, rtol=1e-13)
    (0.5 * (x[top] ** 2).sum()).backward()
    gb, gK = b0.grad.cpu().numpy(), Kv0.grad.cpu().numpy()

    def loss(Kv, b):
        with torch.no_grad():
            xx = contact_solve(s, Kv, b, rtol=1e-13)
            return 0.5 * float((xx[top] ** 2).sum())

    rng = np.random.default_rng(20)
    h = 1e-6
    Kd, bd = Kv0.detach(), b0.detach()
    for i in rng.choice(np.nonzero(~prob.dirichlet)[0], 5, replace=False):
        e = torch.zeros_like(bd)
        e[i] = h
        fd = (loss(Kd, bd + e) - loss(Kd, bd - e)) / (2 * h)
        assert abs(fd - gb[i]) <= 1e-6 * np.abs(gb).max()
    for k in rng.choice(prob.K.nnz, 5, replace=False):
        e = torch.zeros_like(Kd)
        e[k] = h
        fd = (loss(Kd + e, bd) - loss(Kd - e, bd)) / (2 * h)
        assert abs(fd - gK[k]) <= 1e-6 * np.abs(gK).max()
    s.update_fine_values(K_val=Kd)


def test_edge_cases():
    from paper_1912_09056_amd.camg import CamgError

    prob = make_workload("contact2d_16")
    s = _solver(prob, max_levels=2, nu_pre=1, nu_post=1)
    # zero right-hand side: zero solution, no iteration
    x, info = s.solve(torch.zeros(prob.n, dtype=torch.float64))
    assert info["iters"] == 0 and info["converged"] and float(x.abs().max()) == 0.0
    # iteration limit: status NOT_CONVERGED, last iterate returned
    x, info = s.solve(torch.from_numpy(prob.b), max_iters=3)
    assert not info["converged"] and info["iters"] == 3 and info["status"] == 1
    # non-finite right-hand side
    bb = prob.b.copy()
    bb[7] = np.nan
    with pytest.raises(CamgError) as e:
        s.solve(torch.from_numpy(bb))
    assert e.value.code == -3
    # warm start near the solution: the tolerance is relative to the warm residual
    xs, _ = s.solve(torch.from_numpy(prob.b), rtol=1e-6)
    x, info = s.solve(torch.from_numpy(prob.b), x0=xs, rtol=1e-4)
    assert info["converged"]
    A = prob.full_matrix()
    assert np.linalg.norm(prob.b - A @ x.cpu().numpy()) <= 1e-9 * np.linalg.norm(prob.b)
    # one level: the V-cycle is the direct solve, FGMRES needs one iteration
    s1 = _solver(prob, max_levels=1)
    x, info = s1.solve(torch.from_numpy(prob.b))
    assert info["iters"] == 1 and info["converged"]
    # singular coarsest matrix is reported at setup
    pf = make_contact_problem(2, (6, 6), (7, 6), top_bc="free")
    with pytest.raises(CamgError) as e:
        _solver(pf, max_levels=1)
    assert e.value.code == -6


@pytest.mark.parametrize("fmt", [1, 2])
def test_three_level_2d_and_restart(fmt):
    prob = make_contact_problem(2, (24, 24), (25, 24), rhs="random", seed=5)
    kw = dict(max_levels=3, max_coarse_rows=50, nu_pre=1, nu_post=1)
    oopts = OracleOptions(**kw)
    lv = build_hierarchy(prob, oopts)
    s = _solver(prob, fmt=fmt, **kw)
    r = np.random.default_rng(6).standard_normal(prob.n)
    assert _rel(s.vcycle(torch.from_numpy(r)).cpu().numpy(), oracle_vcycle(lv, r, oopts)) < 1e-12
    ref = oracle_solve(lv, oopts, prob.b, m=8, fixed_iters=30)
    x, info = s.solve(torch.from_numpy(prob.b), m=8, fixed_iters=30)
    assert info["restarts"] >= 3
    assert _rel(x.cpu().numpy(), ref.x) < 1e-10


@pytest.mark.parametrize("fmt", [1, 2])
def test_jacobi_sweeps_and_diag_options(fmt):
    # three levels, so the extra Jacobi sweeps also run on a coarse level
    prob = make_contact_problem(2, (24, 24), (25, 24), rhs="random", seed=9)
    for kw in (dict(max_levels=3, max_coarse_rows=50, nu_pre=1, nu_post=2, jacobi_sweeps=2),
               dict(max_levels=3, max_coarse_rows=50, nu_pre=2, nu_post=1, jacobi_diag=1, jacobi_omega=0.5,
                    atilde=1)):
        okw = dict(kw)
        okw["jacobi_diag"] = "diag" if okw.get("jacobi_diag", 0) == 1 else "atilde"
        okw["atilde"] = "diag" if okw.get("atilde", 0) == 1 else "rowsum_abs"
        oopts = OracleOptions(**okw)
        lv = build_hierarchy(prob, oopts)
        s = _solver(prob, fmt=fmt, **kw)
        r = np.random.default_rng(7).standard_normal(prob.n)
        for tr in (False, True):
            z = s.vcycle(torch.from_numpy(r), transpose=tr).cpu().numpy()
            assert _rel(z, oracle_vcycle(lv, r, oopts, transpose=tr)) < 1e-12, (kw, tr)


@pytest.mark.parametrize("fmt", [1, 2])
def test_robust_options_three_level(fmt):
    """Smoothed aggregation, l1 Schur sweeps and three Jacobi sweeps on a
    three-level 2D hierarchy: V-cycle and its transpose (FP64, and mixed to
    FP32 accuracy) and fixed-iteration FGMRES against the oracle."""
    prob = make_contact_problem(2, (24, 24), (25, 24), rhs="random", seed=10)
    kw = dict(max_levels=3, max_coarse_rows=50)
    oopts = OracleOptions(**kw, **ROBUST_ORACLE)
    lv = build_hierarchy(prob, oopts)
    assert lv[1].S is not None
    r = np.random.default_rng(12).standard_normal(prob.n)
    for prec, tol in ((0, 1e-12), (1, 2e-5)):
        s = _solver(prob, precision=prec, fmt=fmt, **kw, **ROBUST_LIB)
        assert s.level_info(1)["k_layout"] in {1: (0,), 2: (1, 3)}[fmt]
        for tr in (False, True):
            z = s.vcycle(torch.from_numpy(r), transpose=tr).cpu().numpy()
            assert _rel(z, oracle_vcycle(lv, r, oopts, transpose=tr)) < tol, (prec, tr)
    s = _solver(prob, fmt=fmt, **kw, **ROBUST_LIB)
    for tr in (False, True):
        ref = oracle_solve(lv, oopts, prob.b, transpose=tr, m=10, fixed_iters=25)
        x, info = s.solve(torch.from_numpy(prob.b), transpose=tr, m=10, fixed_iters=25)
        assert _rel(x.cpu().numpy(), ref.x) < 1e-10, tr


@pytest.mark.parametrize("fmt", [1, 2])
def test_simple_coarse_solver(fmt):
    """CheapSIMPLE sweeps instead of the LU on the coarsest level: V-cycle and
    its transpose (FP64; mixed to FP32 accuracy) and fixed-iteration FGMRES
    against the oracle on a three-level 2D hierarchy, default and robust
    smoother settings."""
    prob = make_contact_problem(2, (24, 24), (25, 24), rhs="random", seed=14)
    for okw, lkw in (({}, {}), (ROBUST_ORACLE, ROBUST_LIB)):
        kw = dict(max_levels=3, max_coarse_rows=50, coarse_sweeps=3)
        oopts = OracleOptions(**kw, coarse_solver="simple", **okw)
        lv = build_hierarchy(prob, oopts)
        r = np.random.default_rng(15).standard_normal(prob.n)
        for prec, tol in ((0, 1e-12), (1, 2e-5)):
            s = _solver(prob, precision=prec, fmt=fmt, coarse_solver=1, **kw, **lkw)
            for tr in (False, True):
                z = s.vcycle(torch.from_numpy(r), transpose=tr).cpu().numpy()
                assert _rel(z, oracle_vcycle(lv, r, oopts, transpose=tr)) < tol, (okw, prec, tr)
        s = _solver(prob, fmt=fmt, coarse_solver=1, **kw, **lkw)
        ref = oracle_solve(lv, oopts, prob.b, m=10, fixed_iters=25)
        x, info = s.solve(torch.from_numpy(prob.b), m=10, fixed_iters=25)
        assert _rel(x.cpu().numpy(), ref.x) < 1e-10, okw


def test_simple_coarse_solver_converges():
    """3D 6^3 workload, two levels, CheapSIMPLE on the coarsest level: both
    precisions reach 1e-8 (true residual) and the FP64 iteration count
    matches the oracle's."""
    prob = make_workload("contact3d_6")
    A = prob.full_matrix()
    oopts = OracleOptions(max_levels=2, coarse_solver="simple", coarse_sweeps=3)
    ref = oracle_solve(build_hierarchy(prob, oopts), oopts, prob.b, rtol=1e-8, max_iters=500)
    assert ref.converged
    for prec in (0, 1):
        s = _solver(prob, precision=prec, max_levels=2, coarse_solver=1, coarse_sweeps=3)
        x, info = s.solve(torch.from_numpy(prob.b), rtol=1e-8, max_iters=500)
        print(f"[simple-coarse] prec={prec} iters={info['iters']} oracle={ref.iters}", flush=True)
        assert info["converged"], (prec, info)
        x = x.cpu().numpy()
        assert np.linalg.norm(prob.b - A @ x) <= 1.0001e-8 * np.linalg.norm(prob.b)
        if prec == 0:
            assert abs(info["iters"] - ref.iters) <= 1


# (oracle options, library options, fixed-iteration parity): with the
# default diagonal Schur step the standard basis makes the smoother a poor
# preconditioner (the diagonal of S is no convergent splitting when D is
# not diagonal), FGMRES stagnates for its first iterations and a
# fixed-iteration comparison there only measures rounding; the l1 Schur
# sweeps fix that
STANDARD_VARIANTS = [
    ({}, {}, False),
    (dict(schur="l1", schur_sweeps=4), dict(schur=1, schur_sweeps=4), True),
    (dict(prolongator="sa", nu_pre=3, nu_post=3, jacobi_sweeps=2, schur="l1", schur_sweeps=8),
     dict(prolongator=1, nu_pre=3, nu_post=3, jacobi_sweeps=2, schur=1, schur_sweeps=8), True),
]


@pytest.mark.parametrize("fmt", [1, 2])
def test_standard_basis_weak_scaling(fmt):
    """Weak-scaling problem with standard multipliers (non-diagonal D), three
    levels: V-cycle and transpose (FP64 1e-12, mixed 2e-5) and both
    precisions solving to 1e-8 for default, l1-Schur and weak-scaling-like
    settings; fixed-iteration FGMRES against the oracle where FGMRES is well
    conditioned."""
    from contactgen import weak_scaling_problem

    prob = weak_scaling_problem(4)
    A = prob.full_matrix()
    r = np.random.default_rng(18).standard_normal(prob.n)
    for okw, lkw, fixed in STANDARD_VARIANTS:
        kw = dict(max_levels=3, max_coarse_rows=200)
        oopts = OracleOptions(**kw, **okw)
        lv = build_hierarchy(prob, oopts)
        for prec, tol in ((0, 1e-12), (1, 2e-5)):
            s = _solver(prob, precision=prec, fmt=fmt, **kw, **lkw)
            for tr in (False, True):
                z = s.vcycle(torch.from_numpy(r), transpose=tr).cpu().numpy()
                assert _rel(z, oracle_vcycle(lv, r, oopts, transpose=tr)) < tol, (okw, prec, tr)
            x, info = s.solve(torch.from_numpy(prob.b), rtol=1e-8, max_iters=500)
            assert info["converged"], (okw, prec, info)
            assert np.linalg.norm(prob.b - A @ x.cpu().numpy()) <= 1.0001e-8 * np.linalg.norm(prob.b)
        if fixed:
            s = _solver(prob, fmt=fmt, **kw, **lkw)
            ref = oracle_solve(lv, oopts, prob.b, m=20, fixed_iters=30)
            x, info = s.solve(torch.from_numpy(prob.b), m=20, fixed_iters=30)
            assert _rel(x.cpu().numpy(), ref.x) < 1e-10, okw


# (oracle options, library options): the paper's block smoothers
BLOCK_SMOOTHERS = [
    (dict(smoother="uzawa", simple_alpha=0.7), dict(smoother=1, simple_alpha=0.7)),
    (dict(smoother="uzawa", simple_alpha=0.7, jacobi_sweeps=2, schur="l1", schur_sweeps=3),
     dict(smoother=1, simple_alpha=0.7, jacobi_sweeps=2, schur=1, schur_sweeps=3)),
    (dict(smoother="braess_sarazin", simple_alpha=1.9), dict(smoother=2, simple_alpha=1.9)),
]


@pytest.mark.parametrize("fmt", [1, 2])
@pytest.mark.parametrize("which", range(len(BLOCK_SMOOTHERS)))
def test_uzawa_and_braess_sarazin(fmt, which):
    """Inexact Uzawa and cheap Braess-Sarazin sweeps: V-cycle and its
    transpose (FP64 1e-12, mixed 2e-5) and fixed-iteration FGMRES against the
    oracle on a three-level 2D hierarchy (three sweeps per level, as in the
    paper's smoother comparison), and a converged 3D solve."""
    okw, lkw = BLOCK_SMOOTHERS[which]
    prob = make_contact_problem(2, (24, 24), (25, 24), rhs="random", seed=19)
    kw = dict(max_levels=3, max_coarse_rows=50, nu_pre=3, nu_post=3)
    oopts = OracleOptions(**kw, **okw)
    lv = build_hierarchy(prob, oopts)
    r = np.random.default_rng(20).standard_normal(prob.n)
    for prec, tol in ((0, 1e-12), (1, 2e-5)):
        s = _solver(prob, precision=prec, fmt=fmt, **kw, **lkw)
        for tr in (False, True):
            z = s.vcycle(torch.from_numpy(r), transpose=tr).cpu().numpy()
            assert _rel(z, oracle_vcycle(lv, r, oopts, transpose=tr)) < tol, (okw, prec, tr)
    s = _solver(prob, fmt=fmt, **kw, **lkw)
    for tr in (False, True):
        ref = oracle_solve(lv, oopts, prob.b, transpose=tr, m=10, fixed_iters=20)
        x, info = s.solve(torch.from_numpy(prob.b), transpose=tr, m=10, fixed_iters=20)
        assert _rel(x.cpu().numpy(), ref.x) < 1e-10, (okw, tr)
    p3 = make_workload("contact3d_6")
    A = p3.full_matrix()
    o3 = OracleOptions(max_levels=2, nu_pre=3, nu_post=3, **okw)
    ref = oracle_solve(build_hierarchy(p3, o3), o3, p3.b, rtol=1e-8, max_iters=500)
    for prec in (0, 1):
        s = _solver(p3, precision=prec, fmt=fmt, max_levels=2, nu_pre=3, nu_post=3, **lkw)
        x, info = s.solve(torch.from_numpy(p3.b), rtol=1e-8, max_iters=500)
        print(f"[block-smoother] {okw} prec={prec} iters={info['iters']} oracle={ref.iters}", flush=True)
        assert info["converged"], (okw, prec, info)
        assert np.linalg.norm(p3.b - A @ x.cpu().numpy()) <= 1.0001e-8 * np.linalg.norm(p3.b)
        if prec == 0:
            assert abs(info["iters"] - ref.iters) <= 1


def _rotated_clamped(angles, se=(5, 5, 4), me=(6, 6, 4)):
    from contactgen import rotate_problem

    p = make_contact_problem(3, se, me, slave_box=((0.1, 0.1, 0.0), (0.8, 0.8, 0.5)),
                             master_box=((0.0, 0.0, -1.0), (1.0, 1.0, 1.0)), top_bc="clamped", rhs="gap",
                             penetration=0.01)
    return rotate_problem(p, *angles)


BLOCK_SCHUR = [
    (dict(simple_alpha=0.7, jacobi_omega=0.7), dict(simple_alpha=0.7, jacobi_omega=0.7)),
    (dict(simple_alpha=0.7, jacobi_omega=0.7, jacobi_sweeps=2, schur_sweeps=3),
     dict(simple_alpha=0.7, jacobi_omega=0.7, jacobi_sweeps=2, schur_sweeps=3)),
    (dict(smoother="uzawa", simple_alpha=0.7, jacobi_omega=0.7), dict(smoother=1, simple_alpha=0.7, jacobi_omega=0.7)),
    (dict(smoother="braess_sarazin", simple_alpha=1.9, schur_sweeps=2), dict(smoother=2, simple_alpha=1.9,
                                                                             schur_sweeps=2)),
]


@pytest.mark.parametrize("fmt", [1, 2])
@pytest.mark.parametrize("which", range(len(BLOCK_SCHUR)))
def test_block_schur_on_rotated_problem(fmt, which):
    """Nodal block relaxation of the Schur system on a rigidly rotated
    clamped two-body problem (three levels, three sweeps per level): V-cycle
    and its transpose (FP64 1e-12, mixed 2e-5), fixed-iteration FGMRES
    (1e-10) and a converged solve against the oracle."""
    okw, lkw = BLOCK_SCHUR[which]
    prob = _rotated_clamped((np.pi / 8, 3 * np.pi / 8))
    kw = dict(max_levels=3, max_coarse_rows=50, nu_pre=3, nu_post=3)
    oopts = OracleOptions(**kw, schur="block", **okw)
    lv = build_hierarchy(prob, oopts)
    r = np.random.default_rng(21).standard_normal(prob.n)
    for prec, tol in ((0, 1e-12), (1, 2e-5)):
        s = _solver(prob, precision=prec, fmt=fmt, schur=2, **kw, **lkw)
        for tr in (False, True):
            z = s.vcycle(torch.from_numpy(r), transpose=tr).cpu().numpy()
            assert _rel(z, oracle_vcycle(lv, r, oopts, transpose=tr)) < tol, (okw, prec, tr)
    s = _solver(prob, fmt=fmt, schur=2, **kw, **lkw)
    for tr in (False, True):
        ref = oracle_solve(lv, oopts, prob.b, transpose=tr, m=10, fixed_iters=20)
        x, info = s.solve(torch.from_numpy(prob.b), transpose=tr, m=10, fixed_iters=20)
        assert _rel(x.cpu().numpy(), ref.x) < 1e-10, (okw, tr)
    ref = oracle_solve(lv, oopts, prob.b, rtol=1e-8, max_iters=300)
    A = prob.full_matrix()
    for prec in (0, 1):
        s = _solver(prob, precision=prec, fmt=fmt, schur=2, **kw, **lkw)
        x, info = s.solve(torch.from_numpy(prob.b), rtol=1e-8, max_iters=300)
        print(f"[block-schur] {okw} fmt={fmt} prec={prec} iters={info['iters']} oracle={ref.iters}", flush=True)
        assert info["converged"], (okw, prec, info)
        assert np.linalg.norm(prob.b - A @ x.cpu().numpy()) <= 1.0001e-8 * np.linalg.norm(prob.b)
        if prec == 0:
            assert abs(info["iters"] - ref.iters) <= 1


NODAL = [
    (dict(simple_alpha=0.7, jacobi_omega=0.7), dict(simple_alpha=0.7, jacobi_omega=0.7)),
    (dict(simple_alpha=0.7, jacobi_omega=0.7, jacobi_sweeps=2, schur_sweeps=3, prolongator="sa"),
     dict(simple_alpha=0.7, jacobi_omega=0.7, jacobi_sweeps=2, schur_sweeps=3, prolongator=1)),
    (dict(smoother="uzawa", simple_alpha=0.7, jacobi_omega=0.7, jacobi_sweeps=2),
     dict(smoother=1, simple_alpha=0.7, jacobi_omega=0.7, jacobi_sweeps=2)),
    (dict(smoother="braess_sarazin", simple_alpha=1.9), dict(smoother=2, simple_alpha=1.9)),
    (dict(simple_alpha=0.7, jacobi_omega=0.7, schur="l1", schur_sweeps=2),
     dict(simple_alpha=0.7, jacobi_omega=0.7, schur=1, schur_sweeps=2)),
]


@pytest.mark.parametrize("fmt", [1, 2])
@pytest.mark.parametrize("which", range(len(NODAL)))
def test_nodal_lumping_on_rotated_problem(fmt, which):
    """Nodal lumping blocks (block Jacobi prediction, block back-substitution,
    Schur matrix and smoothed prolongator from them) on a rigidly rotated
    clamped problem, three levels: V-cycle and its transpose (FP64 1e-12,
    mixed 2e-5), fixed-iteration FGMRES (1e-10) and a converged solve against
    the oracle."""
    okw, lkw = NODAL[which]
    okw = dict({"schur": "block"}, **okw)
    lkw = dict({"schur": 2}, **lkw)
    prob = _rotated_clamped((0.3, 1.1))
    kw = dict(max_levels=3, max_coarse_rows=50, nu_pre=3, nu_post=3)
    oopts = OracleOptions(**kw, atilde="nodal", **okw)
    lv = build_hierarchy(prob, oopts)
    r = np.random.default_rng(22).standard_normal(prob.n)
    for prec, tol in ((0, 1e-12), (1, 2e-5)):
        s = _solver(prob, precision=prec, fmt=fmt, atilde=2, **kw, **lkw)
        for tr in (False, True):
            z = s.vcycle(torch.from_numpy(r), transpose=tr).cpu().numpy()
            assert _rel(z, oracle_vcycle(lv, r, oopts, transpose=tr)) < tol, (okw, prec, tr)
    s = _solver(prob, fmt=fmt, atilde=2, **kw, **lkw)
    for tr in (False, True):
        ref = oracle_solve(lv, oopts, prob.b, transpose=tr, m=10, fixed_iters=20)
        x, info = s.solve(torch.from_numpy(prob.b), transpose=tr, m=10, fixed_iters=20)
        assert _rel(x.cpu().numpy(), ref.x) < 1e-10, (okw, tr)
    ref = oracle_solve(lv, oopts, prob.b, rtol=1e-8, max_iters=300)
    A = prob.full_matrix()
    for prec in (0, 1):
        s = _solver(prob, precision=prec, fmt=fmt, atilde=2, **kw, **lkw)
        x, info = s.solve(torch.from_numpy(prob.b), rtol=1e-8, max_iters=300)
        print(f"[nodal] {okw} fmt={fmt} prec={prec} iters={info['iters']} oracle={ref.iters}", flush=True)
        assert info["converged"], (okw, prec, info)
        assert np.linalg.norm(prob.b - A @ x.cpu().numpy()) <= 1.0001e-8 * np.linalg.norm(prob.b)
        if prec == 0:
            assert abs(info["iters"] - ref.iters) <= 1


NODAL_2D = [
    (dict(atilde="nodal", schur="block"), dict(atilde=2, schur=2)),
    (dict(atilde="nodal", schur="block", smoother="uzawa", simple_alpha=0.7, jacobi_sweeps=2),
     dict(atilde=2, schur=2, smoother=1, simple_alpha=0.7, jacobi_sweeps=2)),
    (dict(schur="block", schur_sweeps=2), dict(schur=2, schur_sweeps=2)),
]


@pytest.mark.parametrize("fmt", [1, 2])
@pytest.mark.parametrize("which", range(len(NODAL_2D)))
def test_nodal_options_2d(fmt, which):
    """The nodal options in 2D (2x2 fine and 3x3 coarse lumping blocks, 2x2
    multiplier blocks), three levels: V-cycle and its transpose against the
    oracle (FP64 1e-12, mixed 2e-5) and the converged solve's iteration
    count."""
    okw, lkw = NODAL_2D[which]
    prob = make_contact_problem(2, (24, 24), (25, 24), rhs="random", seed=19)
    kw = dict(max_levels=3, max_coarse_rows=50, nu_pre=3, nu_post=3)
    oopts = OracleOptions(**kw, **okw)
    lv = build_hierarchy(prob, oopts)
    r = np.random.default_rng(23).standard_normal(prob.n)
    for prec, tol in ((0, 1e-12), (1, 2e-5)):
        s = _solver(prob, precision=prec, fmt=fmt, **kw, **lkw)
        for tr in (False, True):
            z = s.vcycle(torch.from_numpy(r), transpose=tr).cpu().numpy()
            assert _rel(z, oracle_vcycle(lv, r, oopts, transpose=tr)) < tol, (okw, prec, tr)
    ref = oracle_solve(lv, oopts, prob.b, rtol=1e-8, max_iters=300)
    x, info = _solver(prob, fmt=fmt, **kw, **lkw).solve(torch.from_numpy(prob.b), rtol=1e-8, max_iters=300)
    assert info["converged"] and abs(info["iters"] - ref.iters) <= 1, (info, ref.iters)


def test_nodal_lumping_iterations_do_not_depend_on_the_angles():
    """The rotation experiment at the paper's size with the nodal lumping and
    nodal Schur blocks: each smoother's FP64 iteration count is the same for
    every rotation (within one iteration of rounding)."""
    kw = dict(max_levels=3, max_coarse_rows=50, nu_pre=3, nu_post=3, atilde=2, schur=2)
    sm = {0: dict(smoother=0, simple_alpha=0.7, jacobi_omega=0.7), 1: dict(smoother=1, simple_alpha=0.7,
                                                                          jacobi_omega=0.7),
          2: dict(smoother=2, simple_alpha=1.9)}
    its = {k: [] for k in sm}
    for ang in [(0.0, 0.0), (np.pi / 8, np.pi / 4), (3 * np.pi / 8, np.pi / 8), (np.pi / 2, 3 * np.pi / 8)]:
        prob = _rotated_clamped(ang, (9, 9, 9), (9, 9, 9))
        b = torch.from_numpy(prob.b)
        for k, skw in sm.items():
            x, info = _solver(prob, precision=0, **kw, **skw).solve(b, rtol=1e-8, max_iters=300)
            assert info["converged"], (k, ang, info)
            its[k].append(info["iters"])
    print(f"[rotation-nodal] {its}", flush=True)
    for k, v in its.items():
        assert max(v) - min(v) <= 1, (k, v)


def test_rotation_insensitive_iterations_with_block_schur():
    """The two-body rotation experiment at the paper's size (two 10x10x10
    node blocks, 6300 unknowns; three levels, three CheapSIMPLE(0.7) sweeps):
    with the nodal block Schur relaxation the FGMRES iteration counts over
    rotations about y and z stay within 25% of each other, while the
    diagonal Schur step stalls once the interface is tilted."""
    kw = dict(max_levels=3, max_coarse_rows=50, nu_pre=3, nu_post=3, simple_alpha=0.7, jacobi_omega=0.7)
    its = {}
    for ang in [(0.0, 0.0), (np.pi / 8, np.pi / 4), (np.pi / 4, np.pi / 8), (3 * np.pi / 8, 3 * np.pi / 8),
                (np.pi / 2, np.pi / 4)]:
        prob = _rotated_clamped(ang, (9, 9, 9), (9, 9, 9))
        b = torch.from_numpy(prob.b)
        for schur in (0, 2):
            from paper_1912_09056_amd.camg import CamgError

            s = _solver(prob, precision=1, schur=schur, **kw)
            try:
                x, info = s.solve(b, rtol=1e-8, max_iters=300)
                its[schur, ang] = info["iters"] if info["converged"] else 10**9
            except CamgError as e:  # the diagonal step can blow up (non-finite residual)
                assert schur == 0 and e.code == -3, e
                its[schur, ang] = 10**9
    blk = [v for (sc, _), v in its.items() if sc == 2]
    print(f"[rotation] {its}", flush=True)
    assert max(blk) <= 1.25 * min(blk), its
    assert abs(its[0, (0.0, 0.0)] - its[2, (0.0, 0.0)]) <= 2, its
    assert its[0, (np.pi / 4, np.pi / 8)] > 3 * its[2, (np.pi / 4, np.pi / 8)], its


@pytest.mark.parametrize("prec", [0, 1])
def test_two_pass_cgs2_matches_three_pass(prec):
    """The two-pass CGS2 (Gram-matrix second projection, the default) against
    the three-pass form on the 40^3 workload: 30 fixed iterations agree to
    1e-10 (FP64 hierarchy) / 1e-8 (mixed), the converged solves take the same
    number of iterations, and the basis stays orthogonal to 1e-12 over a
    whole restart cycle (checked through the Hessenberg residual estimate
    against the true residual)."""
    prob = make_workload("contact3d_40")
    s = _solver(prob, precision=prec, max_levels=4)
    b = torch.from_numpy(prob.b)
    xs, its = [], []
    for ortho in (1, 0):
        x, info = s.solve(b, fixed_iters=30, ortho=ortho)
        xs.append(x.cpu().numpy())
        _, info = s.solve(b, rtol=1e-8, ortho=ortho)
        assert info["converged"], info
        its.append(info["iters"])
        # the Hessenberg estimate tracks the true residual: no loss of orthogonality
        assert abs(info["rel_res_est"] - info["rel_res_true"]) <= 1e-3 * info["rel_res_true"] + 1e-13, info
    assert _rel(xs[0], xs[1]) < (1e-10 if prec == 0 else 1e-8)
    assert its[0] == its[1], its


def test_bench_workload_parity():
    """The 40^3 / 41x41x40 workload at full size, in the launch configuration the
    benchmark times: V-cycle (FP64) against the oracle on a seeded vector, and both
    precisions solving to 1e-8."""
    prob = make_workload("contact3d_40")
    kw = dict(max_levels=4)
    oopts = OracleOptions(**kw)
    lv = build_hierarchy(prob, oopts)
    s = _solver(prob, **kw)
    r = np.random.default_rng(8).standard_normal(prob.n)
    z = s.vcycle(torch.from_numpy(r)).cpu().numpy()
    assert _rel(z, oracle_vcycle(lv, r, oopts)) < 1e-12
    zt = s.vcycle(torch.from_numpy(r), transpose=True).cpu().numpy()
    assert _rel(zt, oracle_vcycle(lv, r, oopts, transpose=True)) < 1e-12
    sm = _solver(prob, precision=1, **kw)
    for tr, ref in ((False, z), (True, zt)):
        assert _rel(sm.vcycle(torch.from_numpy(r), transpose=tr).cpu().numpy(), ref) < 2e-5, tr
    del sm
    A = prob.full_matrix()
    sc = _solver(prob, fmt=1, **kw)
    assert _rel(sc.vcycle(torch.from_numpy(r)).cpu().numpy(), z) < 1e-13
    for prec, fmt in ((0, 0), (1, 0), (0, 1), (1, 1)):
        sp_ = _solver(prob, precision=prec, fmt=fmt, **kw)
        x, info = sp_.solve(torch.from_numpy(prob.b), rtol=1e-8)
        print(f"[bench-workload] prec={prec} fmt={fmt} iters={info['iters']} t={info['seconds']:.4f}s", flush=True)
        x = x.cpu().numpy()
        assert info["converged"]
        assert np.linalg.norm(prob.b - A @ x) <= 1.0001e-8 * np.linalg.norm(prob.b)


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_replay_matches_eager(prec):
    """The V-cycle replayed from a captured HIP graph equals the eager launch
    sequence bit for bit, on every replay, with eager work and
    synchronisations between replays."""
    prob = make_workload("contact3d_6")
    sg = _solver(prob, precision=prec, fmt=2, max_levels=2, graphs=1)
    se = _solver(prob, precision=prec, fmt=2, max_levels=2, graphs=0)
    rng = np.random.default_rng(30)
    for rep in range(5):
        r = torch.from_numpy(rng.standard_normal(prob.n))
        for tr in (False, True):
            zg = sg.vcycle(r, transpose=tr)
            _ = sg.apply_operator(zg)  # eager work between replays
            torch.cuda.synchronize()
            ze = se.vcycle(r, transpose=tr)
            torch.cuda.synchronize()
            assert torch.equal(zg.cpu(), ze.cpu()), (rep, tr)
    xg, ig = sg.solve(torch.from_numpy(prob.b), rtol=1e-10)
    xe, ie = se.solve(torch.from_numpy(prob.b), rtol=1e-10)
    assert ig["iters"] == ie["iters"] and torch.equal(xg.cpu(), xe.cpu())


def test_lookahead_depth_does_not_change_results():
    """Reading the residual estimate 1, 2 or 5 steps behind the launches
    discards the speculative steps: iterates and counts are identical."""
    prob = make_contact_problem(2, (24, 24), (25, 24), rhs="random", seed=9)
    s = _solver(prob, max_levels=3, max_coarse_rows=50, nu_pre=1, nu_post=1)
    for m in (8, 50):
        ref = None
        for la in (1, 2, 5):
            x, info = s.solve(torch.from_numpy(prob.b), m=m, rtol=1e-9, lookahead=la)
            assert info["converged"]
            if ref is None:
                ref = (x.cpu(), info["iters"])
            else:
                assert info["iters"] == ref[1] and torch.equal(x.cpu(), ref[0]), (la, m)


def test_bench_workload_fgmres_fixed_iterations():
    """FGMRES(50) on the 40^3 / 41x41x40 workload for 60 fixed iterations, one
    full restart cycle plus ten steps, forward and transposed, against the
    oracle (FP64, 1e-10): the widest two-pass CGS2 kernels (up to 51 basis
    vectors per pass) in the launch configuration the benchmark times."""
    prob = make_workload("contact3d_40")
    kw = dict(max_levels=4)
    oopts = OracleOptions(**kw)
    lv = build_hierarchy(prob, oopts)
    s = _solver(prob, **kw)
    for tr in (False, True):
        ref = oracle_solve(lv, oopts, prob.b, transpose=tr, m=50, fixed_iters=60)
        x, info = s.solve(torch.from_numpy(prob.b), transpose=tr, m=50, fixed_iters=60)
        err = _rel(x.cpu().numpy(), ref.x)
        print(f"[fixed60] tr={tr} err={err:.2e} res={info['rel_res_true']:.3e} oracle={ref.rel_res_true:.3e}",
              flush=True)
        assert info["iters"] == 60 and info["restarts"] == 1
        assert err < 1e-10, (tr, err)
        assert abs(info["rel_res_true"] - ref.rel_res_true) <= 1e-6 * ref.rel_res_true


@pytest.mark.parametrize("name,levels", [("contact3d_6", 2), ("contact3d_40", 4)])
def test_setup_from_device_arrays(name, levels):
    """amg_setup with device_ptrs = 1 (blocks, interface lists, multiplier
    nodes and null space as CUDA tensors) builds the same hierarchy as the
    host-pointer setup: identical aggregates on every level and bit-identical
    V-cycles in both directions."""
    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver

    prob = make_workload(name)

    def dev_block(M):
        M = M.tocsr()
        M.sort_indices()
        return (torch.from_numpy(M.indptr.astype(np.int64)).cuda(), torch.from_numpy(M.indices.astype(np.int32)).cuda(),
                torch.from_numpy(M.data.astype(np.float64)).cuda(), M.shape)

    blocks = {k: dev_block(getattr(prob, k)) for k in ("K", "G", "B", "C")}
    ns = torch.from_numpy(np.ascontiguousarray(prob.nullspace.T)).cuda()
    opts = AMGOptions(max_levels=levels)
    sd = AMGSolver.from_device(prob.dim, blocks, torch.from_numpy(prob.slave_dofs).cuda(),
                               torch.from_numpy(prob.master_dofs).cuda(), nullspace=ns,
                               lm_node=None if prob.lm_node is None else torch.from_numpy(prob.lm_node).cuda(),
                               options=opts)
    sh = AMGSolver.from_problem(prob, opts)
    assert sd.n_levels == sh.n_levels
    for l in range(sh.n_levels - 1):
        for a, b in zip(sd.aggregates(l), sh.aggregates(l)):
            assert np.array_equal(a, b)
    r = torch.from_numpy(np.random.default_rng(8).standard_normal(prob.n)).cuda()
    for tr in (False, True):
        assert torch.equal(sd.vcycle(r, transpose=tr), sh.vcycle(r, transpose=tr))


def _rel_fro(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_dense_inverse_random():
    """amg_dense_inverse (device LU with partial pivoting, matrix-core
    updates) on well-conditioned matrices whose rows are shuffled, so that
    pivoting must move them back: sizes across the 64-wide panels, the
    inverse against numpy's to 1e-12 and A X = I to 1e-12; a matrix with a
    zero row is reported singular."""
    from paper_1912_09056_amd.camg import CamgError, dense_inverse

    rng = np.random.default_rng(17)
    for n in (1, 5, 63, 64, 65, 130, 257):
        A = n * np.eye(n) + rng.standard_normal((n, n))
        A = A[rng.permutation(n)]
        X = dense_inverse(torch.from_numpy(A).cuda()).cpu().numpy()
        ref = np.linalg.inv(A)
        print(f"[dense-inverse] n={n} vs numpy {_rel_fro(X, ref):.2e}", flush=True)
        assert _rel_fro(X, ref) < 1e-12, n
        assert np.linalg.norm(A @ X - np.eye(n)) < 1e-12 * np.sqrt(n), n
    A = n * np.eye(n) + rng.standard_normal((n, n))
    A[7] = 0.0
    with pytest.raises(CamgError) as e:
        dense_inverse(torch.from_numpy(A).cuda())
    assert e.value.code == -6


def test_dense_inverse_coarsest_level_matches_oracle():
    """The merged coarsest matrix of the 40^3 workload's 4-level hierarchy
    (108 rows): the device inverse against the oracle's LU inverse."""
    from paper_1912_09056_amd.camg import dense_inverse

    prob = make_workload("contact3d_40")
    lv = build_hierarchy(prob, OracleOptions(max_levels=4))
    Ad = lv[-1].A().toarray()
    X = dense_inverse(torch.from_numpy(Ad).cuda()).cpu().numpy()
    err = _rel_fro(X, lv[-1].A_inv)
    print(f"[dense-inverse] coarsest of contact3d_40: n={Ad.shape[0]} cond={np.linalg.cond(Ad):.1e} "
          f"vs oracle {err:.2e}", flush=True)
    assert err < 1e-12


def test_dense_inverse_weak_scaling_coarsest():
    """The weak-scaling problem at kappa = 36 (1.2M unknowns) with the
    study's settings (smoothed aggregation, coarsening below 5000 rows): the
    setup inverts its 4,131-row merged coarsest matrix on the device.  The
    same matrix's device inverse against numpy's (LAPACK) and A X = I, with
    the timings of the device inverse at this and two smaller sizes."""
    import time

    from contactgen import weak_scaling_problem
    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver, dense_inverse

    prob = weak_scaling_problem(36)
    t0 = time.time()
    s = AMGSolver.from_problem(prob, AMGOptions.robust(max_levels=10, max_coarse_rows=5000, precision=1))
    t_setup = time.time() - t0
    L = s.n_levels - 1
    Ad = sp.bmat([[s.level_matrix(L, "K"), s.level_matrix(L, "G")],
                  [s.level_matrix(L, "B"), s.level_matrix(L, "C")]]).toarray()
    n = Ad.shape[0]
    assert n == 4131, n
    At = torch.from_numpy(Ad).cuda()
    dense_inverse(At)  # warm-up (module load)
    t0 = time.time()
    X = dense_inverse(At).cpu().numpy()
    t_dev = time.time() - t0
    ref = np.linalg.inv(Ad)
    err = _rel_fro(X, ref)
    res = np.linalg.norm(Ad @ X - np.eye(n)) / np.sqrt(n)
    times = {}
    rng = np.random.default_rng(5)
    for m in (108, 816):
        B = torch.from_numpy(m * np.eye(m) + rng.standard_normal((m, m))).cuda()
        dense_inverse(B)
        t0 = time.time()
        dense_inverse(B)
        times[m] = time.time() - t0
    print(f"[dense-inverse] weak-scaling kappa=36 coarsest n={n} cond={np.linalg.cond(Ad):.1e}: vs numpy {err:.2e}, "
          f"|AX-I|/sqrt(n) {res:.2e}; device inverse {t_dev * 1e3:.1f} ms (108: {times[108] * 1e3:.1f} ms, "
          f"816: {times[816] * 1e3:.1f} ms); whole setup {t_setup:.1f} s", flush=True)
    assert res < 1e-10
    assert err < 1e-10
    # the hierarchy built on that inverse solves the problem
    x, info = s.solve(torch.from_numpy(prob.b).cuda(), rtol=1e-8, max_iters=500)
    assert info["converged"], info


def _permute_nodes(prob, seed):
    """The same contact problem with its displacement nodes renumbered by a
    seeded random permutation (multipliers unchanged)."""
    import dataclasses

    d = prob.dim
    nn = prob.n_u // d
    newnode_old = np.random.default_rng(seed).permutation(nn)  # new node -> old node
    P = (newnode_old[:, None] * d + np.arange(d)[None, :]).ravel()  # new dof -> old dof
    inv = np.empty_like(P)
    inv[P] = np.arange(P.size)  # old dof -> new dof
    K = prob.K.tocsr()[P][:, P].tocsr()
    K.sort_indices()
    G = prob.G.tocsr()[P].tocsr()
    B = prob.B.tocsc()[:, P].tocsr()
    B.sort_indices()
    b = np.concatenate([prob.b[:prob.n_u][P], prob.b[prob.n_u:]])
    return dataclasses.replace(
        prob, K=K, G=G, B=B, b=b, slave_dofs=np.sort(inv[prob.slave_dofs]).astype(np.int32),
        master_dofs=np.sort(inv[prob.master_dofs]).astype(np.int32), nullspace=prob.nullspace[P],
        coords=prob.coords[newnode_old] if prob.coords.shape[0] == nn else prob.coords,
        dirichlet=prob.dirichlet[np.concatenate([P, np.arange(prob.n_u, prob.n)])]
        if prob.dirichlet.size == prob.n else prob.dirichlet[P],
        top_dofs=np.sort(inv[prob.top_dofs]))


def test_blocked_ell_block_index_widths():
    """The fine level's blocked-ELL K keeps 16-bit block-column deltas when
    the node numbering is banded (the generator's lexicographic order) and
    full 32-bit indices when it is not (the same 40^3 problem with its nodes
    shuffled); both V-cycles match the oracle's on their own problem."""
    prob = make_workload("contact3d_40")
    shuffled = _permute_nodes(prob, 12)
    kw = dict(max_levels=2)
    r = np.random.default_rng(6).standard_normal(prob.n)
    # banded: symmetric storage (K = K^T, 16-bit deltas); shuffled: the deltas
    # do not fit, so the full layout with 32-bit columns
    for p, width, layout in ((prob, 2, 3), (shuffled, 4, 1)):
        s = _solver(p, **kw)
        info = s.level_info(0)
        assert info["k_layout"] == layout and info["k_index_bytes"] == width, info
        lv = build_hierarchy(p, OracleOptions(**kw))
        for tr in (False, True):
            z = s.vcycle(torch.from_numpy(r), transpose=tr).cpu().numpy()
            ref = oracle_vcycle(lv, r, OracleOptions(**kw), transpose=tr)
            assert _rel(z, ref) < 1e-12, (width, tr)


@pytest.mark.parametrize("name,levels", [("contact3d_6", 2), ("contact3d_40", 4)])
def test_bf16_fine_level_storage(name, levels):
    """precision = mixed with bfloat16 storage of the fine level's K (sliced
    blocked-ELL): the V-cycle and its transpose against the oracle's V-cycle
    on the hierarchy whose level-0 K holds the bfloat16-rounded values (FP32
    arithmetic: 2e-5), and the solve reaching 1e-8 with the FP64 true
    residual, within a few iterations of the FP32 hierarchy's count and with
    a solution within 1e-7 of the FP64 solve."""
    from oracle.storage import fine_k_bf16_levels
    from paper_1912_09056_amd.camg import PREC_MIXED_BF16

    prob = make_workload(name)
    kw = dict(max_levels=levels)
    lv = fine_k_bf16_levels(build_hierarchy(prob, OracleOptions(**kw)))
    s16 = _solver(prob, precision=PREC_MIXED_BF16, fmt=2, **kw)
    rng = np.random.default_rng(9)
    for tr in (False, True):
        r = rng.standard_normal(prob.n)
        z = s16.vcycle(torch.from_numpy(r), transpose=tr).cpu().numpy()
        ref = oracle_vcycle(lv, r, OracleOptions(**kw), transpose=tr)
        assert _rel(z, ref) < 2e-5, tr
    b = torch.from_numpy(prob.b)
    x16, i16 = s16.solve(b, rtol=1e-8)
    s32 = _solver(prob, precision=1, fmt=2, **kw)
    x32, i32 = s32.solve(b, rtol=1e-8)
    x64, _ = _solver(prob, precision=0, fmt=2, **kw).solve(b, rtol=1e-12)
    A = prob.full_matrix()
    xh = x16.cpu().numpy()
    res = np.linalg.norm(prob.b - A @ xh) / np.linalg.norm(prob.b)
    err = _rel(xh, x64.cpu().numpy())
    print(f"[bf16] {name}: iterations bf16 {i16['iters']} fp32 {i32['iters']}, residual {res:.2e}, "
          f"error vs FP64 {err:.2e}", flush=True)
    assert i16["converged"] and res <= 1.0001e-8
    assert i16["iters"] <= i32["iters"] + 3
    assert err < 1e-7


@pytest.mark.parametrize("name,levels", [("contact3d_6", 2), ("contact3d_40", 4)])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_symmetric_storage_matches_full_layout(name, levels, prec):
    """K = K^T exactly, so the blocked-ELL kernels keep only the blocks on and
    right of the block diagonal and read the others transposed from their
    mirrors.  Each row still visits its blocks in ascending column order, so
    the V-cycle (both directions), the FP64 operator and the whole solve
    equal those of the full layout bit for bit, in every precision."""
    prob = make_workload(name)
    kw = dict(max_levels=levels)
    ssym = _solver(prob, precision=prec, fmt=2, **kw)
    sful = _solver(prob, precision=prec, fmt=2 | 4, **kw)  # CAMG_SPMV_BELL | CAMG_SPMV_FULL
    i_sym, i_ful = ssym.level_info(0), sful.level_info(0)
    assert i_sym["k_layout"] == 3 and i_ful["k_layout"] == 1, (i_sym, i_ful)
    assert i_sym["k_blocks"] == i_ful["k_blocks"]
    assert 0 < i_sym["k_lower_blocks"] < i_sym["k_blocks"] / 2
    assert i_ful["k_nnz_stored"] == prob.K.nnz and i_sym["k_nnz_stored"] < prob.K.nnz
    rng = np.random.default_rng(44)
    for tr in (False, True):
        r = torch.from_numpy(rng.standard_normal(prob.n)).cuda()
        a = ssym.vcycle(r, transpose=tr).cpu().numpy()
        b = sful.vcycle(r, transpose=tr).cpu().numpy()
        assert np.array_equal(a, b), (tr, _rel(a, b))
        a = ssym.apply_operator(r, transpose=tr).cpu().numpy()
        b = sful.apply_operator(r, transpose=tr).cpu().numpy()
        assert np.array_equal(a, b), (tr, _rel(a, b))
    bb = torch.from_numpy(prob.b).cuda()
    xs, fs = ssym.solve(bb, rtol=1e-8)
    xf, ff = sful.solve(bb, rtol=1e-8)
    print(f"[sym] {name} prec={prec}: iterations {fs['iters']} / {ff['iters']}", flush=True)
    assert fs["converged"] and fs["iters"] == ff["iters"]
    assert np.array_equal(xs.cpu().numpy(), xf.cpu().numpy())


@pytest.mark.parametrize("prec", [0, 1])
def test_symmetric_storage_after_nonsymmetric_update(prec):
    """New level-0 K values that are not symmetric cannot live in the
    symmetric storage: the FP64 operator (and an FP64 V-cycle) switch to the
    CSR copies, which hold the new values; symmetric values switch back."""
    prob = make_workload("contact3d_6")
    s = _solver(prob, precision=prec, fmt=2, max_levels=2)
    assert s.level_info(0)["k_layout"] == 3
    K1 = prob.K.tocsr()
    K2 = K1.copy()
    K2.data = K2.data * (1.0 + 0.2 * np.random.default_rng(5).random(K2.nnz))
    rng = np.random.default_rng(6)
    x = rng.standard_normal(prob.n)
    xt = torch.from_numpy(x).cuda()
    for K, stale in ((K2, 1), (K1, 0), (K2, 1), (K1, 0)):
        s.update_fine_values(K_val=torch.from_numpy(K.data.copy()).cuda())
        assert s.level_info(0)["k_sym_stale"] == stale
        A = sp.bmat([[K, prob.G], [prob.B, prob.C]]).tocsr()
        for tr in (False, True):
            y = s.apply_operator(xt, transpose=tr).cpu().numpy()
            ref = (A.T if tr else A) @ x
            assert _rel(y, ref) < 1e-14, (stale, tr)
        xx, fi = s.solve(torch.from_numpy(prob.b).cuda(), rtol=1e-10)
        res = np.linalg.norm(prob.b - A @ xx.cpu().numpy()) / np.linalg.norm(prob.b)
        assert fi["converged"] and res <= 1.0001e-10, (stale, res)
    # back on the symmetric values: the V-cycle equals a fresh solver's
    fresh = _solver(prob, precision=prec, fmt=2, max_levels=2)
    r = torch.from_numpy(rng.standard_normal(prob.n)).cuda()
    for tr in (False, True):
        assert np.array_equal(s.vcycle(r, transpose=tr).cpu().numpy(), fresh.vcycle(r, transpose=tr).cpu().numpy())
