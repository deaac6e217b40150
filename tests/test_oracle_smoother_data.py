"""Direct pins of the oracle's smoother data (CPU).

The SIMPLEC lumping Atilde = diag(sum_j |K_ij|), the relaxation diagonal of
the Jacobi prediction and the diagonal of the Schur approximation
S = B Atilde^-1 G - C (Sec. 5.1.3, SIMPLE variants, written with the stored
C = -Z) are compared entry by entry with values built another way on every
smoothing level:

* Atilde and the Jacobi diagonal from the dense level matrix, row by row;
* the Schur diagonal from the dense triple product B diag(1/Atilde) G - C,
  and on the fine level of a flat interface from the mortar matrices D and M
  themselves (normal row j: D_jj^2 / Atilde of its slave dof plus
  sum_k M_jk^2 / Atilde of the master dofs; tangential rows: -1, their C
  entry with an empty B row);
* the oracle's own inverse lumping against the spectral bound it must give:
  every eigenvalue of Atilde^-1 K in [0, 1] (Gershgorin; K is only
  semi-definite), so damped Jacobi with it amplifies no mode.
"""
import numpy as np
import pytest

from contactgen import make_contact_problem, make_workload
from contactgen.mortar import mortar_face
from oracle.hierarchy import AMGOptions, build_hierarchy

CASES = {
    "2d16-2lev": (lambda: make_workload("contact2d_16"), dict(max_levels=2, nu_pre=1, nu_post=1)),
    "2d24-3lev": (lambda: make_contact_problem(2, (24, 24), (25, 24), rhs="random", seed=5),
                  dict(max_levels=3, max_coarse_rows=50)),
    "3d6-2lev": (lambda: make_workload("contact3d_6"), dict(max_levels=2)),
    "3d-3lev": (lambda: make_contact_problem(3, (8, 8, 8), (9, 9, 8)), dict(max_levels=3, max_coarse_rows=200)),
}
VARIANTS = [
    dict(),
    dict(atilde="diag", jacobi_diag="diag", jacobi_omega=0.5),
    dict(jacobi_diag="diag"),
]


@pytest.fixture(scope="module", params=list(CASES))
def problem(request):
    make, kw = CASES[request.param]
    return make(), kw


def _smoothing_levels(lv):
    return lv[:-1]  # the coarsest level is solved directly


@pytest.mark.parametrize("variant", range(len(VARIANTS)))
def test_lumping_and_jacobi_diagonal_dense(problem, variant):
    prob, kw = problem
    opts = AMGOptions(**kw, **VARIANTS[variant])
    lv = build_hierarchy(prob, opts, factor_coarsest=False)
    assert len(lv) >= 2
    for l, L in enumerate(_smoothing_levels(lv)):
        K = L.K.toarray()
        n = K.shape[0]
        row_abs = np.array([sum(abs(v) for v in K[i]) for i in range(n)])
        diag = np.array([K[i, i] for i in range(n)])
        at = row_abs if opts.atilde == "rowsum_abs" else diag
        jd = at if opts.jacobi_diag == "atilde" else diag
        assert np.allclose(1.0 / L.atilde_inv, at, rtol=1e-13, atol=0), (l, "atilde")
        assert np.allclose(1.0 / L.dinv, jd, rtol=1e-13, atol=0), (l, "jacobi diagonal")


def test_schur_diagonal_dense_triple_product(problem):
    prob, kw = problem
    for okw in (dict(), dict(atilde="diag")):
        opts = AMGOptions(**kw, **okw)
        lv = build_hierarchy(prob, opts, factor_coarsest=False)
        for l, L in enumerate(_smoothing_levels(lv)):
            S = L.B.toarray() @ np.diag(L.atilde_inv) @ L.G.toarray() - L.C.toarray()
            sd = np.diag(S)
            scale = np.abs(sd).max()
            assert np.abs(1.0 / L.sd_inv - sd).max() <= 1e-13 * scale, (l, okw)


@pytest.mark.parametrize("name", ["contact2d_16", "contact3d_6"])
def test_schur_diagonal_from_mortar_matrices(name):
    """Fine level of a flat interface: S_d from D, M and the lumping alone."""
    prob = make_workload(name)
    opts = AMGOptions(max_levels=2)
    L = build_hierarchy(prob, opts, factor_coarsest=False)[0]
    d = prob.dim
    info = prob.info
    # interface parameter axes of both bodies, as the generator lays them out
    se, me = info["slave_elems"], info["master_elems"]
    face_s = [np.arange(se[a] + 1) / se[a] for a in range(d - 1)]
    face_m = [np.arange(me[a] + 1) / me[a] for a in range(d - 1)]
    D, M = mortar_face(face_s, face_m)
    D = np.diag(D) if D.ndim == 1 else D
    at = 1.0 / L.atilde_inv
    s_nodes = prob.slave_dofs[::d] // d  # slave interface nodes, ascending = face order
    m_nodes = prob.master_dofs[::d] // d
    ns = len(s_nodes)
    expect = np.empty(d * ns)
    for j in range(ns):
        dn = d - 1  # normal component (flat interface: the last axis)
        slave_dof = s_nodes[j] * d + dn
        v = D[j, j] ** 2 / at[slave_dof]
        for k in np.nonzero(M[j])[0]:
            v += M[j, k] ** 2 / at[m_nodes[k] * d + dn]
        for c in range(d):
            expect[j * d + c] = v if c == dn else -1.0
    assert np.abs(1.0 / L.sd_inv - expect).max() <= 1e-13 * np.abs(expect).max()


def test_lumping_bounds_the_spectrum(problem):
    prob, kw = problem
    opts = AMGOptions(**kw)
    lv = build_hierarchy(prob, opts, factor_coarsest=False)
    for l, L in enumerate(_smoothing_levels(lv)):
        K = L.K.toarray()
        lam = np.linalg.eigvals(L.atilde_inv[:, None] * K)
        assert np.abs(lam.imag).max() <= 1e-9, l
        lam = lam.real
        # K is only semi-definite (the slave block slides normal to its rollers)
        assert lam.min() >= -1e-12 and lam.max() <= 1.0 + 1e-12, (l, lam.min(), lam.max())
        # damped Jacobi never amplifies a mode: |1 - omega lambda| <= 1
        assert np.abs(1.0 - opts.jacobi_omega * lam).max() <= 1.0 + 1e-12, l
