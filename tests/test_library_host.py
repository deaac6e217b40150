"""CPU tests of libcamg: the library loads and exports every declared
symbol, and its host-side hierarchy construction (amg_setup_host: no HIP
call) matches the oracle -- integer outputs bit for bit, Galerkin blocks to
rounding."""
import os
import re

import numpy as np
import pytest

from contactgen import make_contact_problem, make_workload
from oracle.hierarchy import AMGOptions as OracleOptions
from oracle.hierarchy import build_hierarchy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1912_09056_amd", "libcamg.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libcamg.so not built")


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "camg.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s+(\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    import ctypes

    from paper_1912_09056_amd import camg

    lib = ctypes.CDLL(LIB)
    declared = _declared_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(camg.SIGNATURES) == declared


def test_strerror_without_gpu():
    from paper_1912_09056_amd.camg import load_library

    lib = load_library()
    assert lib.amg_strerror(-6).decode() == "singular coarsest matrix"


def _pair(prob, **kw):
    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver

    lib_opts = AMGOptions(**kw)
    ora = build_hierarchy(prob, OracleOptions(**kw))
    lib = AMGSolver.from_problem(prob, lib_opts, host_only=True)
    return ora, lib


CASES = [
    ("contact2d_16", dict(max_levels=2, nu_pre=1, nu_post=1)),
    ("contact3d_6", dict(max_levels=2)),
]


@pytest.mark.parametrize("name,kw", CASES)
def test_host_hierarchy_matches_oracle(name, kw):
    prob = make_workload(name)
    ora, lib = _pair(prob, **kw)
    assert lib.n_levels == len(ora)
    for l, L in enumerate(ora):
        info = lib.level_info(l)
        assert (info["n_u"], info["n_l"]) == (L.n_u, L.n_l)
        for blk in ("K", "G", "B", "C"):
            A = lib.level_matrix(l, blk)
            R = getattr(L, blk)
            # identical symbolic pattern, values to rounding
            assert np.array_equal(A.indptr, R.indptr) and np.array_equal(A.indices, R.indices), (l, blk)
            scale = max(1.0, np.abs(R.data).max()) if R.nnz else 1.0
            assert np.abs(A.data - R.data).max(initial=0.0) <= 1e-13 * scale, (l, blk)
        if l + 1 < len(ora):
            du, dl = lib.aggregates(l)
            assert np.array_equal(du, L.agg_u), l
            assert np.array_equal(dl, L.agg_l), l
            for blk, R in (("P_u", L.P_u), ("P_l", L.P_l)):
                A = lib.level_matrix(l, blk)
                assert np.array_equal(A.indptr, R.indptr) and np.array_equal(A.indices, R.indices)
                assert np.abs(A.data - R.data).max(initial=0.0) <= 1e-13


def test_host_hierarchy_three_levels_2d():
    prob = make_contact_problem(2, (24, 24), (25, 24))
    ora, lib = _pair(prob, max_levels=3, max_coarse_rows=50)
    assert lib.n_levels == len(ora) == 3
    for l in range(2):
        du, dl = lib.aggregates(l)
        assert np.array_equal(du, ora[l].agg_u) and np.array_equal(dl, ora[l].agg_l)
    Kc = lib.level_matrix(2, "K")
    assert np.array_equal(Kc.indices, ora[2].K.indices)
    assert np.abs(Kc.data - ora[2].K.data).max() <= 1e-12 * np.abs(ora[2].K.data).max()


@pytest.mark.slow
def test_host_aggregates_bench_workload():
    # integer outputs of the 3D 40^3 / 41x41x40 workload, all four levels, bit for bit
    prob = make_workload("contact3d_40")
    ora, lib = _pair(prob, max_levels=4)
    assert lib.n_levels == 4
    for l in range(3):
        du, dl = lib.aggregates(l)
        assert np.array_equal(du, ora[l].agg_u)
        assert np.array_equal(dl, ora[l].agg_l)
    sizes = [(lib.level_info(l)["n_u"], lib.level_info(l)["n_l"]) for l in range(4)]
    assert sizes == [(L.n_u, L.n_l) for L in ora]


def test_error_codes_from_host_setup():
    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver, CamgError

    p = make_contact_problem(2, (6, 6), (7, 6), top_bc="free")
    with pytest.raises(CamgError) as e:
        AMGSolver.from_problem(p, AMGOptions(max_levels=1), host_only=True)
    assert e.value.code == -6
    # shape error: multiplier block of the wrong size
    p = make_workload("contact2d_16")
    import scipy.sparse as sp

    with pytest.raises(CamgError) as e:
        AMGSolver(2, p.K, p.G, p.B, sp.identity(p.n_lam + 1, format="csr"), p.slave_dofs, p.master_dofs,
                  host_only=True)
    assert e.value.code == -2 and "G: wrong dimensions" in str(e.value)
    # shape error: column index out of range
    Kb = p.K.copy()
    Kb.indices = Kb.indices.copy()
    Kb.indices[-1] = p.n_u + 3
    with pytest.raises(CamgError) as e:
        AMGSolver(2, Kb, p.G, p.B, p.C, p.slave_dofs, p.master_dofs, host_only=True)
    assert e.value.code == -2
    # non-finite value
    K = p.K.copy()
    K.data[5] = np.nan
    with pytest.raises(CamgError) as e:
        AMGSolver(2, K, p.G, p.B, p.C, p.slave_dofs, p.master_dofs, nullspace=p.nullspace, host_only=True)
    assert e.value.code == -3


ROBUST_CASES = [
    ("contact2d_16", dict(slave_elems=(24, 24), master_elems=(25, 24)), 3),
    ("contact3d_6", {}, 2),
    ("contact3d_150_curved", dict(slave_elems=(6, 6, 6), master_elems=(7, 7, 6)), 2),
]


@pytest.mark.parametrize("name,gen,levels", ROBUST_CASES, ids=[c[0] for c in ROBUST_CASES])
def test_host_hierarchy_robust_options_match_oracle(name, gen, levels):
    # smoothed displacement prolongator and the kept Schur matrix with its
    # signed l1 diagonal: identical patterns, values to rounding
    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver

    prob = make_workload(name, **gen)
    ora = build_hierarchy(prob, OracleOptions(max_levels=levels, max_coarse_rows=50, prolongator="sa", schur="l1",
                                              schur_sweeps=3, jacobi_sweeps=3))
    lib = AMGSolver.from_problem(prob, AMGOptions(max_levels=levels, max_coarse_rows=50, prolongator=1, schur=1,
                                                  schur_sweeps=3, jacobi_sweeps=3), host_only=True)
    assert lib.n_levels == len(ora) == levels
    for l, L in enumerate(ora):
        blocks = ["K", "G", "B", "C"]
        if l + 1 < len(ora):
            blocks += ["P_u", "P_l", "S"]
        for blk in blocks:
            A = lib.level_matrix(l, blk)
            R = getattr(L, blk)
            assert np.array_equal(A.indptr, R.indptr) and np.array_equal(A.indices, R.indices), (l, blk)
            scale = max(1.0, np.abs(R.data).max()) if R.nnz else 1.0
            assert np.abs(A.data - R.data).max(initial=0.0) <= 1e-13 * scale, (l, blk)
    # without Schur sweeps nothing is kept
    lib1 = AMGSolver.from_problem(prob, AMGOptions(max_levels=2, schur=1), host_only=True)
    assert lib1.level_matrix(0, "S").shape == (0, 0)


def test_robust_options_validated():
    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver, CamgError

    p = make_workload("contact2d_16")
    for bad in (dict(schur_sweeps=0), dict(schur_sweeps=65), dict(schur=3), dict(prolongator=2),
                dict(sa_omega=0.0), dict(sa_omega=float("nan"))):
        with pytest.raises(CamgError) as e:
            AMGSolver.from_problem(p, AMGOptions(max_levels=2, **bad), host_only=True)
        assert e.value.code == -1, bad


def test_simple_coarse_solver_host_setup():
    # the 3-level 6^3 hierarchy is singular on its coarsest level: the LU
    # variant reports SINGULAR_COARSE, the CheapSIMPLE variant builds
    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver, CamgError

    p = make_workload("contact3d_6")
    with pytest.raises(CamgError) as e:
        AMGSolver.from_problem(p, AMGOptions(max_levels=3, max_coarse_rows=10), host_only=True)
    assert e.value.code == -6
    s = AMGSolver.from_problem(p, AMGOptions(max_levels=3, max_coarse_rows=10, coarse_solver=1, coarse_sweeps=3),
                               host_only=True)
    assert s.n_levels == 3
    for bad in (dict(coarse_solver=2), dict(coarse_solver=1, coarse_sweeps=0), dict(coarse_sweeps=65)):
        with pytest.raises(CamgError) as e:
            AMGSolver.from_problem(p, AMGOptions(max_levels=2, **bad), host_only=True)
        assert e.value.code == -1, bad


@pytest.mark.parametrize("kappa,levels", [(3, 3), (6, 3)])
def test_host_hierarchy_standard_basis_matches_oracle(kappa, levels):
    # weak-scaling problem with the standard multiplier basis (non-diagonal
    # D): Alg. 1's first-assignment rule bit for bit, every level's blocks
    # and transfers with identical patterns, values to rounding
    from contactgen import weak_scaling_problem

    prob = weak_scaling_problem(kappa)
    ora, lib = _pair(prob, max_levels=levels, max_coarse_rows=100)
    assert lib.n_levels == len(ora) == levels
    for l, L in enumerate(ora):
        blocks = ["K", "G", "B", "C"] + (["P_u", "P_l"] if l + 1 < len(ora) else [])
        for blk in blocks:
            A = lib.level_matrix(l, blk)
            R = getattr(L, blk)
            assert np.array_equal(A.indptr, R.indptr) and np.array_equal(A.indices, R.indices), (l, blk)
            scale = max(1.0, np.abs(R.data).max()) if R.nnz else 1.0
            assert np.abs(A.data - R.data).max(initial=0.0) <= 1e-13 * scale, (l, blk)
        if l + 1 < len(ora):
            du, dl = lib.aggregates(l)
            assert np.array_equal(du, L.agg_u) and np.array_equal(dl, L.agg_l), l


@pytest.mark.parametrize("smoother", [0, 2])
def test_host_block_schur_matches_oracle(smoother):
    # rotated clamped two-body problem: the kept Schur matrix and the inverse
    # nodal blocks (of S_a for Braess-Sarazin) on every smoothing level
    import scipy.sparse as sp

    from contactgen import rotate_problem
    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver

    p = make_contact_problem(3, (4, 4, 3), (5, 5, 3), slave_box=((0.1, 0.1, 0.0), (0.8, 0.8, 0.5)),
                             master_box=((0.0, 0.0, -1.0), (1.0, 1.0, 1.0)), top_bc="clamped", rhs="gap",
                             penetration=0.01)
    prob = rotate_problem(p, np.pi / 8, 3 * np.pi / 8)
    names = {0: "simple", 2: "braess_sarazin"}
    ora = build_hierarchy(prob, OracleOptions(max_levels=3, max_coarse_rows=50, schur="block", schur_sweeps=2,
                                              smoother=names[smoother], simple_alpha=1.9))
    lib = AMGSolver.from_problem(prob, AMGOptions(max_levels=3, max_coarse_rows=50, schur=2, schur_sweeps=2,
                                                  smoother=smoother, simple_alpha=1.9), host_only=True)
    assert lib.n_levels == len(ora) == 3
    for l, L in enumerate(ora[:-1]):
        key = "bs_sb_inv" if smoother == 2 else "sb_inv"
        S_ref = L.extra["bs_S"] if smoother == 2 else L.S
        S = lib.level_matrix(l, "S")
        assert np.array_equal(S.indptr, S_ref.indptr) and np.array_equal(S.indices, S_ref.indices), l
        assert np.abs(S.data - S_ref.data).max() <= 1e-13 * np.abs(S_ref.data).max(), l
        Bi = lib.level_matrix(l, "Sblk_inv").toarray()
        ref = sp.block_diag(list(L.extra[key])).toarray()
        assert np.abs(Bi - ref).max() <= 1e-11 * np.abs(ref).max(), l
    # the diagonal options keep no blocks
    lib0 = AMGSolver.from_problem(prob, AMGOptions(max_levels=2, max_coarse_rows=50, schur=1), host_only=True)
    assert lib0.level_matrix(0, "Sblk_inv").shape == (0, 0)


@pytest.mark.parametrize("smoother,prolongator", [(0, 0), (0, 1), (1, 1), (2, 0)])
def test_host_nodal_lumping_matches_oracle(smoother, prolongator):
    # nodal lumping blocks, the smoothed prolongator and the Schur matrix
    # formed with them, and the nodal Schur blocks (of S_a for
    # Braess-Sarazin, whose alpha the library folds into its lumping blocks)
    import scipy.sparse as sp

    from contactgen import rotate_problem
    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver

    p = make_contact_problem(3, (4, 4, 3), (5, 5, 3), slave_box=((0.1, 0.1, 0.0), (0.8, 0.8, 0.5)),
                             master_box=((0.0, 0.0, -1.0), (1.0, 1.0, 1.0)), top_bc="clamped", rhs="gap",
                             penetration=0.01)
    prob = rotate_problem(p, 0.3, 1.1)
    names = {0: "simple", 1: "uzawa", 2: "braess_sarazin"}
    al = 1.9 if smoother == 2 else 0.7
    ora = build_hierarchy(prob, OracleOptions(max_levels=3, max_coarse_rows=50, atilde="nodal", schur="block",
                                              schur_sweeps=2, smoother=names[smoother], simple_alpha=al,
                                              prolongator="sa" if prolongator else "pa"))
    lib = AMGSolver.from_problem(prob, AMGOptions(max_levels=3, max_coarse_rows=50, atilde=2, schur=2, schur_sweeps=2,
                                                  smoother=smoother, simple_alpha=al, prolongator=prolongator),
                                 host_only=True)
    assert lib.n_levels == len(ora) == 3
    for l, L in enumerate(ora[:-1]):
        for blk in ("K", "G", "B", "C", "P_u", "P_l"):
            A, R = lib.level_matrix(l, blk), getattr(L, blk)
            assert np.array_equal(A.indptr, R.indptr) and np.array_equal(A.indices, R.indices), (l, blk)
            scale = max(1.0, np.abs(R.data).max()) if R.nnz else 1.0
            assert np.abs(A.data - R.data).max(initial=0.0) <= 1e-12 * scale, (l, blk)
        S_ref = L.extra["bs_S"] if smoother == 2 else L.S
        S = lib.level_matrix(l, "S")
        assert np.array_equal(S.indptr, S_ref.indptr) and np.array_equal(S.indices, S_ref.indices), l
        assert np.abs(S.data - S_ref.data).max() <= 1e-12 * np.abs(S_ref.data).max(), l
        Ab = lib.level_matrix(l, "Ablk_inv").toarray()
        ref = sp.block_diag(list(L.atilde_inv / (al if smoother == 2 else 1.0))).toarray()
        assert np.abs(Ab - ref).max() <= 1e-11 * np.abs(ref).max(), l
        Sb = lib.level_matrix(l, "Sblk_inv").toarray()
        ref = sp.block_diag(list(L.extra["bs_sb_inv" if smoother == 2 else "sb_inv"])).toarray()
        assert np.abs(Sb - ref).max() <= 1e-10 * np.abs(ref).max(), l
    from paper_1912_09056_amd.camg import CamgError

    with pytest.raises(CamgError) as e:  # the nodal blocks are the prediction's relaxation too
        AMGSolver.from_problem(prob, AMGOptions(max_levels=2, atilde=2, jacobi_diag=1), host_only=True)
    assert e.value.code == -1


def test_block_schur_needs_node_contiguous_multipliers():
    # the nodal Schur blocks take the d multipliers of a node as consecutive
    # dofs; a problem whose lm_node map is not j / d is a shape error (-2)
    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver, CamgError

    p = make_workload("contact3d_6")
    ln = np.arange(p.n_lam) // 3
    ln[[0, 3]] = ln[[3, 0]]  # swap two multipliers between nodes 0 and 1
    with pytest.raises(CamgError) as e:
        AMGSolver(3, p.K, p.G, p.B, p.C, p.slave_dofs, p.master_dofs, nullspace=p.nullspace, lm_node=ln,
                  options=AMGOptions(max_levels=2, schur=2), host_only=True)
    assert e.value.code == -2
    # the point options accept any pseudo-node map
    AMGSolver(3, p.K, p.G, p.B, p.C, p.slave_dofs, p.master_dofs, nullspace=p.nullspace, lm_node=ln,
              options=AMGOptions(max_levels=2), host_only=True)


def test_option_presets():
    from paper_1912_09056_amd.camg import AMGOptions

    r = AMGOptions.robust(max_levels=5)
    assert (r.prolongator, r.schur, r.schur_sweeps, r.jacobi_sweeps, r.nu_pre, r.nu_post, r.max_levels) == \
        (1, 1, 8, 2, 3, 3, 5)
    q = AMGOptions.rotation_robust()
    assert (q.atilde, q.schur, q.jacobi_diag) == (2, 2, 0)


def _drop_diagonal_entry(K, row):
    """K without its stored (row, row) entry (same other entries)."""
    import scipy.sparse as sp

    C = K.tocoo()
    keep = ~((C.row == row) & (C.col == row))
    out = sp.csr_matrix((C.data[keep], (C.row[keep], C.col[keep])), shape=K.shape)
    out.sort_indices()
    return out


def test_zero_diagonal_is_reported():
    """CAMG_ERR_ZERO_DIAG (-4) from the host setup, for a displacement row
    without a diagonal entry and for a Schur diagonal that vanishes (a normal
    constraint row whose B row is empty and whose C entry is zero); the
    oracle refuses both cases too."""
    import scipy.sparse as sp

    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver, CamgError

    p = make_workload("contact2d_16")
    free = np.nonzero(~p.dirichlet)[0]
    K = _drop_diagonal_entry(p.K, int(free[10]))
    with pytest.raises(CamgError) as e:
        AMGSolver(2, K, p.G, p.B, p.C, p.slave_dofs, p.master_dofs, nullspace=p.nullspace, host_only=True,
                  options=AMGOptions(max_levels=2))
    assert e.value.code == -4 and "zero diagonal" in str(e.value)
    pk = make_workload("contact2d_16")
    pk.K = K
    with pytest.raises(ZeroDivisionError):
        build_hierarchy(pk, OracleOptions(max_levels=2))
    # normal constraint row 2 j + 1 of slave node j: empty B row, C entry 0
    j = 5
    B = p.B.tolil()
    B[2 * j + 1, :] = 0.0
    B = sp.csr_matrix(B)
    B.eliminate_zeros()
    assert p.C[2 * j + 1, 2 * j + 1] == 0.0
    with pytest.raises(CamgError) as e:
        AMGSolver(2, p.K, p.G, B, p.C, p.slave_dofs, p.master_dofs, nullspace=p.nullspace, host_only=True,
                  options=AMGOptions(max_levels=2))
    assert e.value.code == -4 and "Schur" in str(e.value)
    pb = make_workload("contact2d_16")
    pb.B = B
    with pytest.raises(ZeroDivisionError):
        build_hierarchy(pb, OracleOptions(max_levels=2))


def test_rank_deficient_aggregate_is_reported():
    """CAMG_ERR_RANK_DEFICIENT_AGG (-5): a null space with two equal columns
    cannot be orthonormalised on any aggregate; the oracle refuses it too."""
    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver, CamgError

    p = make_workload("contact2d_16")
    ns = p.nullspace.copy()
    ns[:, 2] = ns[:, 0]
    with pytest.raises(CamgError) as e:
        AMGSolver(2, p.K, p.G, p.B, p.C, p.slave_dofs, p.master_dofs, nullspace=ns, host_only=True,
                  options=AMGOptions(max_levels=2))
    assert e.value.code == -5
    pn = make_workload("contact2d_16")
    pn.nullspace = ns
    with pytest.raises(Exception) as e:
        build_hierarchy(pn, OracleOptions(max_levels=2))
    assert "rank" in str(e.value).lower()


def _exactly_symmetric(A):
    At = A.T.tocsr()
    At.sort_indices()
    return (np.array_equal(A.indptr, At.indptr) and np.array_equal(A.indices, At.indices)
            and np.array_equal(A.data, At.data))


def _pair2(prob, okw, lkw):
    from paper_1912_09056_amd.camg import AMGOptions, AMGSolver

    return build_hierarchy(prob, OracleOptions(**okw)), AMGSolver.from_problem(prob, AMGOptions(**lkw),
                                                                              host_only=True)


@pytest.mark.parametrize("okw,lkw", [(dict(max_levels=4), dict(max_levels=4)),
                                     (dict(max_levels=4, prolongator="sa"), dict(max_levels=4, prolongator=1))])
def test_coarse_stiffness_symmetric_iff_fine_is(okw, lkw):
    """A fine K equal to its transpose gives coarse K's equal to theirs bit
    for bit (each mirrored pair of the Galerkin product replaced by its mean),
    within the 1e-13 bar of the oracle's unsymmetrised product; a fine K that
    is not symmetric leaves the Galerkin products as computed."""
    import dataclasses

    prob = make_workload("contact3d_6", slave_elems=(8, 8, 8), master_elems=(9, 9, 8))
    ora, lib = _pair2(prob, okw, lkw)
    assert _exactly_symmetric(prob.K.tocsr())
    for l in range(lib.n_levels):
        K = lib.level_matrix(l, "K")
        assert _exactly_symmetric(K), l
        R = ora[l].K
        assert np.abs(K.data - R.data).max() <= 1e-13 * max(1.0, np.abs(R.data).max()), l
    # one entry off its mirror by one unit in the last place
    K1 = prob.K.tocsr().copy()
    rows = np.repeat(np.arange(K1.shape[0]), np.diff(K1.indptr))
    k = int(np.argmax(np.abs(K1.data) * (rows != K1.indices)))  # the largest off-diagonal entry
    K1.data[k] = np.nextafter(K1.data[k], np.inf)
    ora1, lib1 = _pair2(dataclasses.replace(prob, K=K1), okw, lkw)
    assert not _exactly_symmetric(lib1.level_matrix(0, "K"))
    for l in range(1, lib1.n_levels):
        K = lib1.level_matrix(l, "K")
        R = ora1[l].K
        assert np.abs(K.data - R.data).max() <= 1e-13 * max(1.0, np.abs(R.data).max()), l
