"""Pins for the oracle's hierarchy setup (CPU): aggregation, Alg. 1,
tentative transfers, Galerkin blocks."""
import numpy as np
import pytest
import scipy.sparse as sp

from contactgen import make_contact_problem, make_workload
from oracle.hierarchy import (
    AMGOptions,
    aggregate,
    build_hierarchy,
    dirichlet_dofs,
    galerkin,
    lagmult_aggregation,
    node_graph,
    tentative_prolongator,
)


def _chain(n):
    A = sp.diags([np.ones(n - 1), np.ones(n - 1)], [-1, 1], format="csr")
    return A.indptr, A.indices


def test_aggregation_chain_by_hand():
    # path 0-1-2-3-4-5-6: roots 0 ({0,1}), 3 ({2,3,4}); node 5's neighbour 4 is taken,
    # node 6 has the free neighbour 5 -> root {5,6}
    indptr, indices = _chain(7)
    agg, n = aggregate(indptr, indices, np.ones(7, bool))
    assert n == 3
    assert agg.tolist() == [0, 0, 1, 1, 1, 2, 2]


def test_aggregation_chain_phase2_by_hand():
    # path of 6: roots 0 ({0,1}) and 3 ({2,3,4}); node 5 joins aggregate 1 in phase 2
    indptr, indices = _chain(6)
    agg, n = aggregate(indptr, indices, np.ones(6, bool))
    assert n == 2 and agg.tolist() == [0, 0, 1, 1, 1, 1]


def _graph(n, edges):
    r = [a for a, b in edges] + [b for a, b in edges]
    c = [b for a, b in edges] + [a for a, b in edges]
    A = sp.csr_matrix((np.ones(len(r)), (r, c)), shape=(n, n))
    A.sort_indices()
    return A.indptr, A.indices


def test_aggregation_phase2_tie_smallest_id():
    # root 0 takes {0,1,2}; root 3 takes {3,4,5}; node 6 touches one node of each
    # aggregate -> tie -> smallest id
    indptr, indices = _graph(7, [(0, 1), (0, 2), (3, 4), (3, 5), (6, 1), (6, 4)])
    agg, n = aggregate(indptr, indices, np.ones(7, bool))
    assert n == 2 and agg.tolist() == [0, 0, 0, 1, 1, 1, 0]
    # node 6 touching aggregate 1 twice -> joins 1
    indptr, indices = _graph(7, [(0, 1), (0, 2), (3, 4), (3, 5), (6, 1), (6, 4), (6, 5)])
    agg, n = aggregate(indptr, indices, np.ones(7, bool))
    assert agg[6] == 1


def test_aggregation_inactive_nodes_ignored():
    indptr, indices = _graph(5, [(0, 1), (2, 3), (1, 4), (2, 4)])
    act = np.array([True, True, True, True, False])
    agg, n = aggregate(indptr, indices, act)
    assert agg.tolist() == [0, 0, 1, 1, -1] and n == 2


def test_aggregation_phase3_isolated():
    # 0-1 chain plus an isolated active node 2: phase 1 roots 0 and 2
    indptr, indices = _graph(3, [(0, 1)])
    agg, n = aggregate(indptr, indices, np.ones(3, bool))
    assert agg.tolist() == [0, 0, 1] and n == 2


def _agg_count_closed_form(nodes_per_axis):
    return int(np.prod([(na - 1) // 3 + 1 for na in nodes_per_axis]))


@pytest.mark.parametrize(
    "dim,se,me",
    [(2, (16, 16), (17, 16)), (3, (6, 6, 6), (7, 7, 6)), (3, (8, 5, 7), (9, 6, 7)), (2, (10, 7), (11, 9))],
)
def test_aggregate_count_closed_form_and_validity(dim, se, me):
    p = make_contact_problem(dim, se, me)
    lv = build_hierarchy(p, AMGOptions(max_levels=2, max_coarse_rows=10))
    L = lv[0]
    agg = L.agg_u
    # slave body: all nodes active; master: bottom layer clamped (inactive)
    ns_nodes = [n + 1 for n in se]
    nm_nodes = [n + 1 for n in me]
    nm_active = nm_nodes[:-1] + [nm_nodes[-1] - 1]
    expect = _agg_count_closed_form(ns_nodes) + _agg_count_closed_form(nm_active)
    assert agg.max() + 1 == expect
    n_s = int(np.prod(ns_nodes))
    # every active node aggregated, clamped nodes not; bodies never mixed
    dir_nodes = L.dirichlet.reshape(-1, dim).all(axis=1)
    assert np.all((agg >= 0) == ~dir_nodes)
    assert set(agg[:n_s]).isdisjoint(set(agg[n_s:][agg[n_s:] >= 0]))
    # aggregates are connected in the node graph and have at least 2^dim nodes
    indptr, indices = node_graph(L.K, dim, L.dirichlet, L.slave_nodes, L.master_nodes)
    for a in range(agg.max() + 1):
        members = np.nonzero(agg == a)[0]
        assert len(members) >= 2 ** dim
        seen = {members[0]}
        stack = [members[0]]
        mset = set(members.tolist())
        while stack:
            i = stack.pop()
            for j in indices[indptr[i]:indptr[i + 1]]:
                if j in mset and j not in seen:
                    seen.add(j)
                    stack.append(j)
        assert len(seen) == len(members)


def test_dirichlet_detection_matches_generator():
    p = make_workload("contact3d_6")
    assert np.array_equal(dirichlet_dofs(p.K, p.G), p.dirichlet)


def test_interface_couplings_dropped():
    # a synthetic coupling between a slave and a master interface node is ignored
    p = make_workload("contact2d_16")
    d = p.dim
    K = p.K.tolil()
    i, j = p.slave_dofs[4], p.master_dofs[6]
    K[i, j] = K[j, i] = -0.1
    K = K.tocsr()
    n_nodes = p.n_u // d
    s = np.zeros(n_nodes, bool)
    m = np.zeros(n_nodes, bool)
    s[p.slave_dofs // d] = True
    m[p.master_dofs // d] = True
    dirich = dirichlet_dofs(K, p.G)
    ip, ix = node_graph(K, d, dirich, s, m)
    assert j // d not in ix[ip[i // d]:ip[i // d + 1]]
    ip2, ix2 = node_graph(K, d, dirich, np.zeros_like(s), np.zeros_like(m))
    assert j // d in ix2[ip2[i // d]:ip2[i // d + 1]]


def test_alg1_by_hand():
    # 3 slave nodes (2 dofs each) in displacement aggregates [5, 5, 2]; diagonal D couples
    # slave node k with multiplier pseudo-node k.  Ascending slave dofs meet aggregate 5
    # first -> multiplier aggregate 0 = {0, 1}; aggregate 2 -> multiplier aggregate 1 = {2}.
    disp_agg = np.array([5, 5, 2])
    slave_dofs = np.arange(6)
    G = sp.identity(6, format="csr")
    lm_node = np.arange(6) // 2
    lm_agg, dmap, n = lagmult_aggregation(disp_agg, 6, slave_dofs, G, 2, lm_node, 3)
    assert n == 2
    assert lm_agg.tolist() == [0, 0, 1]
    assert dmap.tolist() == [-1, -1, 1, -1, -1, 0]


def test_alg1_image_of_slave_aggregates():
    # dual D is diagonal: every multiplier aggregate is the image of exactly one slave aggregate
    for name in ["contact2d_16", "contact3d_6"]:
        p = make_workload(name)
        lv = build_hierarchy(p, AMGOptions(max_levels=2))
        L = lv[0]
        d = p.dim
        slave_iface_nodes = np.unique(p.slave_dofs // d)  # ascending = pseudo-node order
        expect = L.dmap[L.agg_u[slave_iface_nodes]]
        assert np.array_equal(L.agg_l, expect)
        used = L.dmap[L.dmap >= 0]
        assert sorted(used.tolist()) == list(range(L.agg_l.max() + 1))


def test_tentative_prolongator_orthonormal_and_reproduces_nullspace():
    p = make_workload("contact3d_6")
    lv = build_hierarchy(p, AMGOptions(max_levels=3, max_coarse_rows=50), factor_coarsest=False)
    for l in range(len(lv) - 1):
        L, Lc = lv[l], lv[l + 1]
        for P, agg, node_of, Zf, Zc, zero in (
            (L.P_u, L.agg_u, np.arange(L.n_u) // L.bs_u, L.nullspace_u, Lc.nullspace_u, L.dirichlet),
            (L.P_l, L.agg_l, L.lm_node, L.nullspace_l, Lc.nullspace_l, np.zeros(L.n_l, bool)),
        ):
            Pd = P.toarray()
            assert np.allclose(Pd.T @ Pd, np.eye(P.shape[1]), atol=1e-13)
            Zf0 = Zf.copy()
            Zf0[zero] = 0.0
            assert np.allclose(P @ Zc, Zf0, atol=1e-12)
            # block structure: a fine dof only feeds the coarse dofs of its aggregate
            n_ns = Zf.shape[1]
            rows, cols = P.nonzero()
            assert np.all(cols // n_ns == agg[node_of[rows]])


def test_galerkin_matches_dense_triple_product():
    p = make_workload("contact2d_16")
    lv = build_hierarchy(p, AMGOptions(max_levels=3, max_coarse_rows=50))
    for l in range(len(lv) - 1):
        L, Lc = lv[l], lv[l + 1]
        Pu, Pl = L.P_u.toarray(), L.P_l.toarray()
        for coarse, R, A, P in (
            (Lc.K, Pu.T, L.K.toarray(), Pu),
            (Lc.G, Pu.T, L.G.toarray(), Pl),
            (Lc.B, Pl.T, L.B.toarray(), Pu),
            (Lc.C, Pl.T, L.C.toarray(), Pl),
        ):
            ref = R @ A @ P
            assert np.abs(coarse.toarray() - ref).max() <= 1e-13 * max(1.0, np.abs(ref).max())


def test_galerkin_symbolic_pattern_keeps_cancellations():
    R = sp.csr_matrix(np.array([[1.0, 1.0]]))
    A = sp.csr_matrix(np.array([[1.0], [-1.0]]))
    P = sp.csr_matrix(np.array([[1.0]]))
    C = galerkin(R, A, P)
    assert C.nnz == 1 and C.data[0] == 0.0


def test_level_sizes_2d_workload():
    p = make_workload("contact2d_16")
    lv = build_hierarchy(p, AMGOptions(max_levels=2, nu_pre=1, nu_post=1))
    assert [L.n for L in lv] == [1224, 228]
