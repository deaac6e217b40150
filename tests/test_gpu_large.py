"""Full-size checks on the GPU through the C-ABI.

The 40^3 / 41x41x40 gradient check, the 100^3 lognormal(0, 1) workload (FP64
and mixed precision, with the V-cycle compared against the oracle's at full
size) and the 150^3 curved lognormal(0, 2) workload (mixed precision with the
robustness settings) run with every `-m gpu` invocation.  At 150^3 the
oracle does not finish in reasonable time, so the checks there are
properties that hold at any size: the true FP64 residual recomputed on the
host, the adjoint identity g.x = lam.b and the transposed V-cycle's
dot-product test (these run at 100^3 too, next to the oracle comparison).
"""

import numpy as np
import pytest
import torch

from contactgen import make_workload

pytestmark = pytest.mark.gpu



@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1912_09056_amd.camg import load_library

    load_library()


def _solver(prob, precision=0, **kw):
    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver

    return AMGSolver.from_problem(prob, AMGOptions(precision=precision, **kw))


@pytest.mark.parametrize("prec", [0, 1])
def test_gradients_40_central_differences(prec):
    """40^3 workload: dL/db and dL/dK (L = 0.5 ||u_top||^2) from the adjoint
    solve against central differences with step 1e-6 on 20 seeded entries of
    b and 20 of K's nonzeros.  Bars: 1e-6 of the gradient's largest entry for
    every sampled entry, and 1e-5 relative to the entry itself for entries of
    at least 1 % of the largest (below that the differences of the loss are
    dominated by the solves' FP64 rounding floor).  Every entry's error is
    printed."""
    from paper_1912_09056_amd import contact_solve

    prob = make_workload("contact3d_40")
    s = _solver(prob, precision=prec, max_levels=4)
    top = torch.from_numpy(prob.top_dofs).cuda()
    Kv0 = torch.tensor(prob.K.data, dtype=torch.float64, device="cuda", requires_grad=True)
    b0 = torch.tensor(prob.b, dtype=torch.float64, device="cuda", requires_grad=True)
    # 1e-12: the FP64 rounding floor of this operator is about 1e-13
    x = contact_solve(s, Kv0, b0, rtol=1e-12)
    (0.5 * (x[top] ** 2).sum()).backward()
    gb, gK = b0.grad.cpu().numpy(), Kv0.grad.cpu().numpy()
    Kd, bd = Kv0.detach(), b0.detach()
    x0 = x.detach()

    def loss(Kv, b):
        with torch.no_grad():
            s.update_fine_values(K_val=Kv)
            # warm start: the initial residual is the O(h) perturbation; reduce it by
            # 1e-9, but not below the operator's rounding floor (~1e-13 of ||b||)
            r0 = float((b - s.apply_operator(x0)).norm())
            rtol = max(1e-9, 2e-13 * float(b.norm()) / r0)
            xx, info = s.solve(b, x0=x0, rtol=rtol)
            assert info["converged"], info
            return 0.5 * float((xx[top] ** 2).sum())

    rng = np.random.default_rng(40)
    h = 1e-6

    def report(name, idx, adj, fds, gmax):
        """Per-entry errors of the adjoint gradient against central
        differences: relative to the entry itself and to the gradient's
        largest entry."""
        err = np.abs(np.asarray(fds) - adj[idx])
        rel = err / np.maximum(np.abs(adj[idx]), 1e-300)
        for i, a, f, e in zip(idx, adj[idx], fds, rel):
            print(f"[fd40] prec={prec} d{name}[{i}] adjoint {a:+.10e} fd {f:+.10e} rel {e:.2e}", flush=True)
        big = np.abs(adj[idx]) >= 1e-2 * gmax
        print(f"[fd40] prec={prec} d{name}: worst per-entry rel {rel.max():.2e} (entries >= 1% of max|g|: "
              f"{rel[big].max() if big.any() else 0.0:.2e}), worst vs max|g| {err.max() / gmax:.2e}", flush=True)
        assert (rel[big] <= 1e-5).all(), rel[big]
        return err / gmax

    ib = rng.choice(np.nonzero(~prob.dirichlet)[0], 20, replace=False)
    fdb = []
    for i in ib:
        e = torch.zeros_like(bd)
        e[i] = h
        fdb.append((loss(Kd, bd + e) - loss(Kd, bd - e)) / (2 * h))
    worst_b = report("b", ib, gb, fdb, np.abs(gb).max())
    ik = rng.choice(prob.K.nnz, 20, replace=False)
    fdk = []
    for k in ik:
        e = torch.zeros_like(Kd)
        e[k] = h
        fdk.append((loss(Kd + e, bd) - loss(Kd - e, bd)) / (2 * h))
    s.update_fine_values(K_val=Kd)
    worst_k = report("K", ik, gK, fdk, np.abs(gK).max())
    assert worst_b.max() <= 1e-6, worst_b
    assert worst_k.max() <= 1e-6, worst_k


# settings for strong stiffness contrast, after the paper's weak-scaling
# configuration (smoothed aggregation with omega = 4/3, three CheapSIMPLE
# sweeps per level, a two-sweep prediction), with eight l1-lumped Jacobi
# sweeps standing in for its ILU on the Schur system; the plain settings stall
# on lognormal(0, 2) moduli (the diagonal Schur step is not a convergent
# splitting there)
ROBUST = dict(prolongator=1, schur=1, schur_sweeps=8, jacobi_sweeps=2, nu_pre=3, nu_post=3)  # AMGOptions.robust()


def _large_case(name, levels, precisions=(0, 1), oracle=False, **opts):
    import time

    t0 = time.time()
    prob = make_workload(name)
    print(f"[large] {name}: n={prob.n} nnz(K)={prob.K.nnz} generated in {time.time() - t0:.0f}s", flush=True)
    A = prob.full_matrix()
    b = torch.from_numpy(prob.b).cuda()
    top = prob.top_dofs
    rng = np.random.default_rng(3)
    u = torch.from_numpy(rng.standard_normal(prob.n)).cuda()
    v = torch.from_numpy(rng.standard_normal(prob.n)).cuda()
    zo = None
    if oracle:
        from oracle.hierarchy import AMGOptions as OracleOptions
        from oracle.hierarchy import build_hierarchy
        from oracle.vcycle import vcycle as oracle_vcycle

        t0 = time.time()
        oo = OracleOptions(max_levels=levels)
        lv = build_hierarchy(prob, oo)
        uh = u.cpu().numpy()
        zo = {tr: oracle_vcycle(lv, uh, oo, transpose=tr) for tr in (False, True)}
        print(f"[large] {name} oracle hierarchy + 2 V-cycles {time.time() - t0:.0f}s, levels "
              f"{[L.K.shape[0] + L.C.shape[0] for L in lv]}", flush=True)
        del lv
    out = {}
    for prec in precisions:
        t0 = time.time()
        s = _solver(prob, precision=prec, max_levels=levels, **opts)
        print(f"[large] {name} prec={prec} setup {time.time() - t0:.0f}s, levels "
              f"{[s.level_info(l)['n_u'] + s.level_info(l)['n_l'] for l in range(s.n_levels)]}", flush=True)
        if zo is not None:
            # the full-size V-cycle (forward and transposed) against the oracle's
            tol = 1e-12 if prec == 0 else 2e-5
            for tr in (False, True):
                z = s.vcycle(u, transpose=tr).cpu().numpy()
                err = np.linalg.norm(z - zo[tr]) / np.linalg.norm(zo[tr])
                print(f"[large] {name} prec={prec} transpose={tr} V-cycle vs oracle {err:.2e}", flush=True)
                assert err < tol, (prec, tr, err)
        x, fi = s.solve(b, rtol=1e-8, max_iters=3000)
        assert fi["converged"], fi
        xh = x.cpu().numpy()
        rel = np.linalg.norm(prob.b - A @ xh) / np.linalg.norm(prob.b)
        assert rel <= 1.0001e-8, rel
        g = np.zeros(prob.n)
        g[top] = xh[top]
        lam, ai = s.solve(torch.from_numpy(g).cuda(), transpose=True, rtol=1e-10, max_iters=3000)
        assert ai["converged"], ai
        lamh = lam.cpu().numpy()
        relT = np.linalg.norm(g - A.T @ lamh) / np.linalg.norm(g)
        assert relT <= 1.0001e-10, relT
        # adjoint identity: g.x = lam.b (both sides within the solve tolerances)
        lhs, rhs = g @ xh, lamh @ prob.b
        assert abs(lhs - rhs) <= 1e-7 * abs(lhs), (lhs, rhs)
        # transposed V-cycle is the exact transpose of the forward one
        a1 = float(v @ s.vcycle(u))
        a2 = float(s.vcycle(v, transpose=True) @ u)
        tol = 1e-11 if prec == 0 else 1e-4
        assert abs(a1 - a2) <= tol * abs(a1), (a1, a2)
        out[prec] = (xh, fi, ai)
        print(f"[large] {name} prec={prec} fwd iters={fi['iters']} t={fi['seconds']:.3f}s "
              f"adj iters={ai['iters']} t={ai['seconds']:.3f}s rel={rel:.2e}", flush=True)
        del s
        torch.cuda.empty_cache()
    if len(out) == 2:
        err = np.linalg.norm(out[1][0] - out[0][0]) / np.linalg.norm(out[0][0])
        print(f"[large] {name} FP64 iterations {out[0][1]['iters']} / adjoint {out[0][2]['iters']}, mixed "
              f"iterations {out[1][1]['iters']} / adjoint {out[1][2]['iters']}, mixed-vs-FP64 solution "
              f"difference {err:.2e}", flush=True)
        assert err < 1e-7


def test_large_100_lognormal():
    """100^3 / 101x101x100, lognormal(0, 1) moduli, 4 levels: FP64 and mixed
    V-cycles against the oracle at full size, both solves to 1e-8 (true
    residual on the host), FP64-vs-mixed iterations and solution error."""
    _large_case("contact3d_100_lognormal", 4, oracle=True)


def test_large_150_curved():
    """150^3 / 151x151x150, curved interface, lognormal(0, 2) moduli, 5
    levels, mixed precision with the robustness settings: forward and adjoint
    solves checked by their host-recomputed residuals and the adjoint
    identity."""
    _large_case("contact3d_150_curved", 5, precisions=(1,), **ROBUST)
