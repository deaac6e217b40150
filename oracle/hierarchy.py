"""Oracle: setup of the fully coupled aggregation AMG hierarchy (FP64, CPU).

Test infrastructure only (see the package docstring).

Paper passages followed:
* fully coupled multigrid with segregated transfers P = blkdiag(P^u, P^l)
  and R = P^T (Sec. 4.1, segregated transfer operators);
* displacement aggregation on K with slave/master interface couplings
  dropped on the fly (Sec. 4.2);
* multiplier aggregates as images of the slave displacement aggregates
  (Sec. 4.3, Alg. 1);
* tentative (non-smoothed) transfers from aggregates plus null space
  (Sec. 3.1.2);
* Galerkin coarse blocks and the merged direct solve on the coarsest level
  (weak-scaling study, solver settings);
* SIMPLEC lumping of |K| and the Schur approximation (Sec. 5.1.3, SIMPLE
  variants);
* optionally, smoothed aggregation for the displacement transfers
  (Sec. 3.1.2, prolongator smoothing equation; the weak-scaling settings
  smooth the displacement prolongator with omega = 4/3 and keep the
  multiplier transfers unsmoothed);
* optionally, the CheapSIMPLE level smoother instead of the direct solve on
  the coarsest level (the second coarse-solver variant of the weak-scaling
  study), which needs smoother data there and no merged factorisation.

Readings where the paper is silent (all listed in the design notes):
* Dirichlet dof = row of K whose only stored entry is its diagonal and whose
  G row is empty;
* standard aggregation = three-phase greedy aggregation in natural order
  (phase 1: root + all neighbours when none is taken; phase 2 on a snapshot:
  join the neighbouring aggregate holding most neighbours, ties to the
  smallest id; phase 3: leftovers seed new aggregates with their free
  neighbours);
* "D_ij != 0" in Alg. 1 = a stored entry of G's slave rows; sparsity
  patterns of coarse blocks are symbolic (no numerical dropping);
* coarse slave / master interface nodes = aggregates containing such nodes;
* tentative prolongator by per-aggregate modified Gram-Schmidt QR of the
  null-space rows (Dirichlet rows zeroed), columns in order, R_ii > 0;
* multiplier null space = one constant per Cartesian component;
* prolongator smoothing divides by the lumped diagonal Atilde = diag(sum_j
  |K_ij|) instead of diag(K): its spectrum bound lambda(Atilde^-1 K) <= 1
  lets omega = 4/3 be applied as printed (with diag(K), whose spectrum on
  hex8 elasticity reaches about 3.15, omega = 4/3 would amplify);
* the Schur system of the correction step (solved by ILU(0) or KLU in the
  paper's runs) is either inverted by its diagonal or relaxed by a few
  undamped Jacobi sweeps with the signed l1 lumping
  sign(S_jj) sum_k |S_jk|, the Schur analogue of Atilde.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp


@dataclass
class AMGOptions:
    max_levels: int = 4
    max_coarse_rows: int = 1000
    nu_pre: int = 2
    nu_post: int = 2
    jacobi_sweeps: int = 1
    jacobi_omega: float = 0.8
    simple_alpha: float = 0.8
    atilde: str = "rowsum_abs"  # or "diag", or "nodal" (block lumping per node, see nodal_lumping)
    jacobi_diag: str = "atilde"  # relaxation diagonal of the prediction: "atilde" or "diag"
    prolongator: str = "pa"  # displacement transfers: "pa" tentative, "sa" smoothed
    sa_omega: float = 4.0 / 3.0  # prolongator smoothing factor (with the lumped diagonal)
    schur: str = "diag"  # relaxation of the Schur approximation: "diag", "l1" or "block" (nodal blocks)
    schur_sweeps: int = 1  # Jacobi sweeps on the Schur system (1 = divide by the diagonal)
    coarse_solver: str = "lu"  # coarsest level: "lu" (merged dense LU) or "simple" (CheapSIMPLE sweeps)
    coarse_sweeps: int = 2  # sweeps from zero on the coarsest level with "simple"
    smoother: str = "simple"  # block smoother: "simple" (CheapSIMPLE), "uzawa", "braess_sarazin"


@dataclass
class Level:
    K: sp.csr_matrix
    G: sp.csr_matrix
    B: sp.csr_matrix
    C: sp.csr_matrix
    bs_u: int
    bs_l: int
    slave_nodes: np.ndarray  # bool per displacement node
    master_nodes: np.ndarray
    lm_node: np.ndarray  # multiplier dof -> pseudo-node
    nullspace_u: np.ndarray
    nullspace_l: np.ndarray
    dirichlet: np.ndarray = None
    agg_u: np.ndarray = None  # node -> aggregate (this level's nodes), -1 = none
    agg_l: np.ndarray = None  # multiplier pseudo-node -> multiplier aggregate
    dmap: np.ndarray = None  # displacement aggregate -> multiplier aggregate (-1 none)
    P_u: sp.csr_matrix = None
    P_l: sp.csr_matrix = None
    dinv: np.ndarray = None
    atilde_inv: np.ndarray = None
    sd_inv: np.ndarray = None
    S: sp.csr_matrix = None  # Schur approximation B Atilde^-1 G - C (when relaxed by sweeps)
    A_inv: np.ndarray = None  # coarsest level only
    extra: dict = field(default_factory=dict)

    @property
    def n_u(self):
        return self.K.shape[0]

    @property
    def n_l(self):
        return self.C.shape[0]

    @property
    def n(self):
        return self.n_u + self.n_l

    def A(self) -> sp.csr_matrix:
        return sp.bmat([[self.K, self.G], [self.B, self.C]], format="csr")

    def nnz(self) -> int:
        return self.K.nnz + self.G.nnz + self.B.nnz + self.C.nnz


# ----------------------------------------------------------------------------
# graph and aggregation


def dirichlet_dofs(K: sp.csr_matrix, G: sp.csr_matrix) -> np.ndarray:
    """Rows of K holding only their diagonal entry, with an empty G row."""
    n = K.shape[0]
    cnt = np.diff(K.indptr)
    first = np.where(cnt > 0, K.indices[np.minimum(K.indptr[:-1], max(K.nnz - 1, 0))], -1)
    diag_only = (cnt == 1) & (first == np.arange(n))
    g_empty = np.diff(G.indptr) == 0
    return diag_only & g_empty


def node_graph(K, bs, dirichlet, slave_nodes, master_nodes):
    """Node adjacency (CSR arrays, sorted, no self loops).

    Nodes i != j are adjacent when a stored entry of K's (i, j) block lies in
    a non-Dirichlet row and a non-Dirichlet column.  Pairs of a slave
    interface node and a master interface node are dropped (Sec. 4.2).
    """
    n_nodes = K.shape[0] // bs
    coo = K.tocoo()
    keep = ~dirichlet[coo.row] & ~dirichlet[coo.col]
    r = coo.row[keep] // bs
    c = coo.col[keep] // bs
    keep = r != c
    keep &= ~((slave_nodes[r] & master_nodes[c]) | (master_nodes[r] & slave_nodes[c]))
    Gn = sp.csr_matrix((np.ones(int(keep.sum())), (r[keep], c[keep])), shape=(n_nodes, n_nodes))
    Gn.sum_duplicates()
    Gn.sort_indices()
    return Gn.indptr.astype(np.int64), Gn.indices.astype(np.int64)


def aggregate(indptr, indices, active):
    """Three-phase greedy aggregation in natural node order.

    Only active nodes take part; edges to inactive nodes are ignored.
    Returns (agg, n_agg): agg[i] = aggregate id, -1 for inactive nodes.
    """
    n = len(active)
    agg = np.full(n, -1, dtype=np.int64)
    n_agg = 0

    def nbrs(i):
        nb = indices[indptr[i]:indptr[i + 1]]
        return nb[active[nb]]

    # phase 1: a node whose neighbourhood is untouched becomes a root and
    # takes all of its neighbours
    for i in range(n):
        if not active[i] or agg[i] >= 0:
            continue
        nb = nbrs(i)
        if nb.size and (agg[nb] >= 0).any():
            continue
        agg[i] = n_agg
        agg[nb] = n_agg
        n_agg += 1
    # phase 2: leftovers join the adjacent phase-1 aggregate holding most of
    # their neighbours (ties: smallest aggregate id), decided on a snapshot
    snap = agg.copy()
    for i in range(n):
        if not active[i] or snap[i] >= 0:
            continue
        a = snap[nbrs(i)]
        a = a[a >= 0]
        if a.size == 0:
            continue
        ids, counts = np.unique(a, return_counts=True)  # ids ascending
        agg[i] = ids[np.argmax(counts)]  # argmax takes the first (smallest id) maximum
    # phase 3: remaining nodes seed new aggregates with their free neighbours
    for i in range(n):
        if not active[i] or agg[i] >= 0:
            continue
        nb = nbrs(i)
        agg[i] = n_agg
        agg[nb[agg[nb] < 0]] = n_agg
        n_agg += 1
    return agg, n_agg


def lagmult_aggregation(disp_agg, n_disp_agg, slave_dofs, Gmat, bs_u, lm_node, n_lm_nodes):
    """Alg. 1 (Sec. 4.3): multiplier aggregates from displacement aggregates.

    Walks the slave displacement dofs i in ascending order; k is the
    aggregate of i's node; every multiplier j coupled to i (a stored entry
    G[i, j], i.e. D_ij != 0 with D^T held in G's slave rows) puts j's
    pseudo-node into the multiplier aggregate d(k).  A pseudo-node keeps its
    first assignment, and d(k) is created when the first pseudo-node is put
    into it: with a non-diagonal D an aggregate whose multipliers were all
    claimed before gets none (an empty multiplier aggregate would have no
    null-space rows).  With a dual (diagonal) D this is the order of first
    encounter.
    Returns (lm_agg per pseudo-node, dmap per displacement aggregate, count).
    """
    lm_agg = np.full(n_lm_nodes, -1, dtype=np.int64)
    dmap = np.full(n_disp_agg, -1, dtype=np.int64)
    n_l = 0
    for i in slave_dofs:
        k = disp_agg[i // bs_u]
        if k < 0:
            continue
        for j in Gmat.indices[Gmat.indptr[i]:Gmat.indptr[i + 1]]:
            nl = lm_node[j]
            if lm_agg[nl] < 0:
                if dmap[k] < 0:
                    dmap[k] = n_l
                    n_l += 1
                lm_agg[nl] = dmap[k]
    return lm_agg, dmap, n_l


def tentative_prolongator(agg, n_agg, node_of_dof, nullspace, zero_rows, rank_tol=1e-12):
    """Tentative prolongator of aggregation AMG (Sec. 3.1.2).

    For each aggregate the null-space rows of its dofs (rows in zero_rows
    set to zero) are factored by modified Gram-Schmidt, column by column:
    Q becomes the aggregate's block of P, R the coarse null-space rows.
    The pattern of P holds all n_ns coarse columns for every fine dof of an
    aggregated node that is not a zeroed row (explicit zeros kept).
    Returns (P csr, coarse nullspace).
    """
    n_rows, n_ns = nullspace.shape
    dof_agg = np.where(node_of_dof >= 0, agg[np.maximum(node_of_dof, 0)], -1)
    dof_agg = np.where(zero_rows, -1, dof_agg)
    order = np.argsort(dof_agg, kind="stable")
    order = order[dof_agg[order] >= 0]
    starts = np.searchsorted(dof_agg[order], np.arange(n_agg + 1))
    Pvals = np.zeros((n_rows, n_ns))
    coarse = np.zeros((n_agg * n_ns, n_ns))
    for a in range(n_agg):
        rows = order[starts[a]:starts[a + 1]]  # ascending dof order
        Bm = nullspace[rows, :].copy()
        Q = np.zeros_like(Bm)
        R = np.zeros((n_ns, n_ns))
        for k in range(n_ns):
            v = Bm[:, k].copy()
            for i in range(k):
                R[i, k] = np.dot(Q[:, i], v)
                v = v - R[i, k] * Q[:, i]
            nv = np.sqrt(np.dot(v, v))
            if not nv > rank_tol * np.sqrt(np.dot(Bm[:, k], Bm[:, k])):
                raise np.linalg.LinAlgError(f"rank-deficient aggregate {a}")
            R[k, k] = nv
            Q[:, k] = v / nv
        Pvals[rows, :] = Q
        coarse[a * n_ns:(a + 1) * n_ns, :] = R
    has = dof_agg >= 0
    rows_idx = np.repeat(np.nonzero(has)[0], n_ns)
    cols_idx = (dof_agg[has][:, None] * n_ns + np.arange(n_ns)[None, :]).ravel()
    vals = Pvals[has].ravel()
    indptr = np.zeros(n_rows + 1, dtype=np.int64)
    np.cumsum(np.where(has, n_ns, 0), out=indptr[1:])
    P = sp.csr_matrix((vals, cols_idx, indptr), shape=(n_rows, n_agg * n_ns))
    return P, coarse


def _pattern(M):
    S = sp.csr_matrix((np.ones(M.nnz), M.indices.copy(), M.indptr.copy()), shape=M.shape)
    return S


def _on_pattern(N, S):
    """The values of N on the (sorted, wider) pattern S; zeros elsewhere."""
    S = S.tocsr()
    S.sort_indices()
    N = N.tocsr()
    N.sort_indices()
    out = sp.csr_matrix((np.zeros(S.nnz), S.indices.copy(), S.indptr.copy()), shape=S.shape)
    if N.nnz:
        nrow = np.repeat(np.arange(N.shape[0]), np.diff(N.indptr))
        key_s = np.repeat(np.arange(S.shape[0]), np.diff(S.indptr)).astype(np.int64) * S.shape[1] + S.indices
        key_n = nrow.astype(np.int64) * S.shape[1] + N.indices
        pos = np.searchsorted(key_s, key_n)
        assert np.all(key_s[pos] == key_n)
        out.data[pos] = N.data
    return out


def galerkin(R, A, P):
    """R A P on the symbolic pattern of the product (no numerical dropping)."""
    return _on_pattern(R @ A @ P, _pattern(R) @ _pattern(A) @ _pattern(P))


def nodal_lumping(K, bs):
    """Nodal SIMPLEC lumping: for every node i (bs consecutive dofs) the
    bs x bs block K_ii plus (sum over nodes j != i of ||K_ij||_F) times the
    identity.  For symmetric K, 2|x_i^T K_ij x_j| <= ||K_ij|| (|x_i|^2 +
    |x_j|^2) gives x^T K x <= x^T Atilde x, the block analogue of the row-sum
    bound, and a rotation of the node's frame (K_ij -> R K_ij R^T) maps the
    blocks to R Atilde_i R^T since the Frobenius norm is invariant.
    Returns the blocks, shape (n / bs, bs, bs)."""
    n = K.shape[0]
    if bs <= 0 or n % bs:
        raise ValueError("dof count is not a multiple of the node block size")
    nb = n // bs
    coo = K.tocoo()
    rn, cn = coo.row // bs, coo.col // bs
    A = np.zeros((nb, bs, bs))
    d = rn == cn
    np.add.at(A, (rn[d], coo.row[d] % bs, coo.col[d] % bs), coo.data[d])
    key = rn[~d].astype(np.int64) * nb + cn[~d]
    uk, inv = np.unique(key, return_inverse=True)
    fro = np.sqrt(np.bincount(inv, weights=coo.data[~d] ** 2, minlength=len(uk)))
    off = np.zeros(nb)
    np.add.at(off, uk // nb, fro)
    return A + off[:, None, None] * np.eye(bs)[None, :, :]


def block_diag_matrix(blocks):
    """The block-diagonal CSR matrix of a (nb, bs, bs) stack."""
    nb, bs, _ = blocks.shape
    rows = np.repeat(np.arange(nb * bs), bs)
    cols = (np.arange(nb)[:, None, None] * bs + np.zeros((1, bs, 1), int) + np.arange(bs)[None, None, :]).ravel()
    return sp.csr_matrix((blocks.reshape(-1), (rows, cols)), shape=(nb * bs, nb * bs))


def smoothed_prolongator(K, P_hat, omega, Ainv_blocks=None):
    """P = P_hat - omega Atilde^-1 K P_hat (Sec. 3.1.2, prolongator smoothing)
    with the lumped diagonal Atilde = diag(sum_j |K_ij|), on the symbolic
    pattern of P_hat plus that of K P_hat.  With Ainv_blocks (the inverse
    nodal lumping blocks) Atilde^-1 is that block-diagonal matrix, on the
    pattern of P_hat plus that of Atilde^-1 K P_hat."""
    if Ainv_blocks is not None:
        D = block_diag_matrix(Ainv_blocks)
        DKP = _on_pattern(D @ (K @ P_hat), _pattern(D) @ _pattern(K) @ _pattern(P_hat) + _pattern(P_hat))
        Ph = _on_pattern(P_hat, DKP)
        out = DKP.copy()
        out.data = Ph.data - omega * DKP.data
        return out
    w = omega / np.asarray(abs(K).sum(axis=1)).ravel()
    KP = _on_pattern(K @ P_hat, _pattern(K) @ _pattern(P_hat) + _pattern(P_hat))
    Ph = _on_pattern(P_hat, KP)
    rows = np.repeat(np.arange(KP.shape[0]), np.diff(KP.indptr))
    out = KP.copy()
    out.data = Ph.data - w[rows] * KP.data
    return out


def schur_matrix(L: "Level", At_inv):
    """B Atilde^-1 G - C on the symbolic pattern of B G plus that of C (of
    B Atilde^-1 G plus C's for nodal lumping blocks, At_inv of shape
    (nb, bs, bs))."""
    if np.ndim(At_inv) == 3:
        D = block_diag_matrix(At_inv)
        return _on_pattern(L.B @ D @ L.G - L.C, _pattern(L.B) @ _pattern(D) @ _pattern(L.G) + _pattern(L.C))
    BA = L.B @ sp.diags(At_inv)
    return _on_pattern(BA @ L.G - L.C, _pattern(L.B) @ _pattern(L.G) + _pattern(L.C))


# ----------------------------------------------------------------------------
# smoother data and coarsest level


def smoother_data(L: Level, opts: AMGOptions):
    """The SIMPLEC lumping Atilde = diag(sum_j |K_ij|) (or diag K), the
    diagonal of the Schur approximation B Atilde^-1 G - C (Sec. 5.1.3, SIMPLE
    variants; written with the stored C = -Z), and the relaxation diagonal of
    the Jacobi prediction.

    Reading: the paper's cheap prediction is a few sweeps of a convergent
    relaxation (SGS in its runs, Sec. 5.2).  Plain damped Jacobi on diag(K)
    with the damping 0.8 diverges on 3D hex8 elasticity (the spectrum of
    diag(K)^-1 K reaches about 3.15), so the default relaxation diagonal is
    the same lumped Atilde, which bounds the spectrum of Atilde^-1 K by one
    for symmetric positive semi-definite K (Gershgorin) and keeps the damped
    sweep convergent.  "diag" selects plain diag(K).

    Schur options: "diag" takes the exact diagonal of the Schur
    approximation; "l1" the signed absolute row sums sign(S_jj) sum_k |S_jk|,
    which bound the spectrum of diag^-1 S by one for symmetric positive
    semi-definite S (as Atilde does for K), so Jacobi sweeps on the Schur
    system converge even where the mortar coupling M dominates D (a much
    softer master side).  "block" relaxes with the inverses of S's nodal
    diagonal blocks (the d multipliers of one node): with Cartesian
    multipliers and normal/tangential constraint rows a node's block of S
    mixes all its components once the interface normal leaves the
    coordinate axes, and its diagonal alone can vanish (a rigidly rotated
    problem), while the block transforms with the rotation.  With
    schur_sweeps > 1 the matrix itself is kept."""
    dK = L.K.diagonal()
    if np.any(dK == 0.0):
        raise ZeroDivisionError("zero diagonal in K")
    if opts.atilde == "nodal":
        return _smoother_data_nodal(L, opts)
    if opts.atilde == "rowsum_abs":
        At = np.asarray(abs(L.K).sum(axis=1)).ravel()
    else:
        At = dK.copy()
    if np.any(At == 0.0):
        raise ZeroDivisionError("zero Atilde")
    At_inv = 1.0 / At
    # diag(B Atilde^-1 G)_j = sum_i B[j, i] G[i, j] / Atilde_i
    L.extra.pop("sb_inv", None)
    L.extra.pop("bs_sb_inv", None)
    if opts.schur == "block":
        S = schur_matrix(L, At_inv)
        L.extra["sb_inv"] = node_block_inverse(S, L.bs_l, L.lm_node)
        Sd = S.diagonal()
        L.S = S if opts.schur_sweeps > 1 else None
    elif opts.schur == "l1" or opts.schur_sweeps > 1:
        S = schur_matrix(L, At_inv)
        if opts.schur == "l1":
            Sd = np.sign(S.diagonal()) * np.asarray(abs(S).sum(axis=1)).ravel()
        else:
            Sd = S.diagonal()
        L.S = S if opts.schur_sweeps > 1 else None
    else:
        BG = L.B.multiply(L.G.T.tocsr()).tocsr()
        Sd = np.asarray(BG @ At_inv).ravel() - L.C.diagonal()
    if opts.schur != "block" and np.any(Sd == 0.0):
        raise ZeroDivisionError("zero Schur diagonal")
    L.dinv = At_inv.copy() if opts.jacobi_diag == "atilde" else 1.0 / dK
    L.atilde_inv = At_inv
    L.sd_inv = None if opts.schur == "block" else 1.0 / Sd
    if opts.smoother == "braess_sarazin":
        # S_a = B Atilde^-1 G / alpha - C (Sec. 5.1.2), same diagonal rule
        Sa = schur_matrix(L, At_inv / opts.simple_alpha)
        if opts.schur == "block":
            L.extra["bs_sb_inv"] = node_block_inverse(Sa, L.bs_l, L.lm_node)
            L.extra.pop("bs_sd_inv", None)
            if opts.schur_sweeps > 1:
                L.extra["bs_S"] = Sa
            return
        if opts.schur == "l1":
            da = np.sign(Sa.diagonal()) * np.asarray(abs(Sa).sum(axis=1)).ravel()
        else:
            da = Sa.diagonal()
        if np.any(da == 0.0):
            raise ZeroDivisionError("zero Schur diagonal")
        L.extra["bs_sd_inv"] = 1.0 / da
        if opts.schur_sweeps > 1:
            L.extra["bs_S"] = Sa


def _smoother_data_nodal(L: Level, opts: AMGOptions):
    """Smoother data with the nodal lumping (atilde="nodal"): the inverse
    blocks serve as Atilde^-1 in the back-substitution, the Schur matrix and
    (jacobi_diag="atilde" only) as the block relaxation of the prediction;
    Schur relaxation as for the point lumping, from S = B Atilde^-1 G - C."""
    if opts.jacobi_diag != "atilde":
        raise ValueError("the nodal lumping relaxes the prediction with its own blocks")
    blocks = nodal_lumping(L.K, L.bs_u)
    try:
        At_inv = np.linalg.inv(blocks)
    except np.linalg.LinAlgError:
        raise ZeroDivisionError("singular nodal lumping block") from None
    L.dinv = At_inv
    L.atilde_inv = At_inv
    L.extra.pop("sb_inv", None)
    L.extra.pop("bs_sb_inv", None)
    Sa_inv = At_inv / opts.simple_alpha if opts.smoother == "braess_sarazin" else At_inv
    S = schur_matrix(L, Sa_inv)
    key_blk, key_d = ("bs_sb_inv", "bs_sd_inv") if opts.smoother == "braess_sarazin" else ("sb_inv", None)
    if opts.schur == "block":
        L.extra[key_blk] = node_block_inverse(S, L.bs_l, L.lm_node)
        Sd = None
    elif opts.schur == "l1":
        Sd = np.sign(S.diagonal()) * np.asarray(abs(S).sum(axis=1)).ravel()
    else:
        Sd = S.diagonal()
    if Sd is not None and np.any(Sd == 0.0):
        raise ZeroDivisionError("zero Schur diagonal")
    if opts.smoother == "braess_sarazin":
        L.sd_inv = None
        if Sd is not None:
            L.extra[key_d] = 1.0 / Sd
        if opts.schur_sweeps > 1:
            L.extra["bs_S"] = S
        L.S = None
    else:
        L.sd_inv = None if Sd is None else 1.0 / Sd
        L.S = S if opts.schur_sweeps > 1 else None


def node_block_inverse(S, bs, lm_node=None):
    """Inverses of the bs x bs diagonal blocks of S over multiplier nodes
    (bs consecutive dofs each): shape (n_l / bs, bs, bs).  The nodal block
    Jacobi relaxation of the Schur system (block option) divides by these."""
    n = S.shape[0]
    if bs <= 0 or n % bs:
        raise ValueError("multiplier count is not a multiple of the node block size")
    if lm_node is not None and len(lm_node) and not np.array_equal(np.asarray(lm_node), np.arange(n) // bs):
        raise ValueError("block Schur relaxation needs node-contiguous multipliers")
    Sd = S.toarray() if n <= 4096 else None
    out = np.empty((n // bs, bs, bs))
    for j in range(n // bs):
        sl = slice(j * bs, (j + 1) * bs)
        blk = Sd[sl, sl] if Sd is not None else S[sl, sl].toarray()
        try:
            out[j] = np.linalg.inv(blk)
        except np.linalg.LinAlgError:
            raise ZeroDivisionError(f"singular Schur node block {j}") from None
    return out


class SingularCoarse(np.linalg.LinAlgError):
    pass


def coarse_inverse(L: Level, pivot_tol=1e-13):
    """Merged dense coarsest matrix, LU with partial pivoting (LAPACK) and
    its inverse.  A pivot below pivot_tol times the largest entry of A_c
    marks the coarsest matrix singular."""
    import scipy.linalg as sla

    Ad = L.A().toarray()
    lu, piv = sla.lu_factor(Ad, check_finite=True)
    if np.min(np.abs(np.diag(lu))) <= pivot_tol * np.max(np.abs(Ad)):
        raise SingularCoarse("singular coarsest matrix")
    L.A_inv = sla.lu_solve((lu, piv), np.eye(Ad.shape[0]))


# ----------------------------------------------------------------------------
# hierarchy


def _level_from_problem(prob) -> Level:
    d = prob.dim
    n_nodes = prob.n_u // d
    slave_nodes = np.zeros(n_nodes, dtype=bool)
    master_nodes = np.zeros(n_nodes, dtype=bool)
    slave_nodes[np.asarray(prob.slave_dofs) // d] = True
    master_nodes[np.asarray(prob.master_dofs) // d] = True
    n_l = prob.n_lam
    Zl = np.zeros((n_l, d))
    Zl[np.arange(n_l), np.arange(n_l) % d] = 1.0
    return Level(
        K=sp.csr_matrix(prob.K),
        G=sp.csr_matrix(prob.G),
        B=sp.csr_matrix(prob.B),
        C=sp.csr_matrix(prob.C),
        bs_u=d,
        bs_l=d,
        slave_nodes=slave_nodes,
        master_nodes=master_nodes,
        lm_node=np.asarray(prob.lm_node, dtype=np.int64),
        nullspace_u=np.asarray(prob.nullspace, dtype=float),
        nullspace_l=Zl,
    )


def coarsen(L: Level, opts: AMGOptions = None):
    """Aggregate level L and return the next coarser level."""
    opts = opts or AMGOptions()
    dirichlet = dirichlet_dofs(L.K, L.G)
    L.dirichlet = dirichlet
    n_nodes = L.n_u // L.bs_u
    node_dirichlet_all = dirichlet.reshape(n_nodes, L.bs_u).all(axis=1)
    active = ~node_dirichlet_all
    indptr, indices = node_graph(L.K, L.bs_u, dirichlet, L.slave_nodes, L.master_nodes)
    agg_u, n_agg_u = aggregate(indptr, indices, active)

    slave_dofs = np.nonzero(np.repeat(L.slave_nodes, L.bs_u))[0]
    n_lm_nodes = int(L.lm_node.max()) + 1 if L.n_l else 0
    agg_l, dmap, n_agg_l = lagmult_aggregation(agg_u, n_agg_u, slave_dofs, L.G, L.bs_u, L.lm_node, n_lm_nodes)
    if np.any(agg_l < 0):
        raise ValueError("multiplier pseudo-node without a slave coupling")

    node_of_dof_u = np.arange(L.n_u) // L.bs_u
    P_u, ns_u_c = tentative_prolongator(agg_u, n_agg_u, node_of_dof_u, L.nullspace_u, dirichlet)
    P_l, ns_l_c = tentative_prolongator(agg_l, n_agg_l, L.lm_node, L.nullspace_l, np.zeros(L.n_l, bool))
    if opts.prolongator == "sa":
        if opts.atilde == "nodal":
            P_u = smoothed_prolongator(L.K, P_u, opts.sa_omega, np.linalg.inv(nodal_lumping(L.K, L.bs_u)))
        else:
            P_u = smoothed_prolongator(L.K, P_u, opts.sa_omega)
    R_u = P_u.T.tocsr()
    R_l = P_l.T.tocsr()
    L.agg_u, L.agg_l, L.dmap, L.P_u, L.P_l = agg_u, agg_l, dmap, P_u, P_l

    n_ns_u = L.nullspace_u.shape[1]
    n_ns_l = L.nullspace_l.shape[1]
    slave_c = np.zeros(n_agg_u, dtype=bool)
    master_c = np.zeros(n_agg_u, dtype=bool)
    sel = agg_u >= 0
    slave_c[agg_u[sel & L.slave_nodes]] = True
    master_c[agg_u[sel & L.master_nodes]] = True
    return Level(
        K=galerkin(R_u, L.K, P_u),
        G=galerkin(R_u, L.G, P_l),
        B=galerkin(R_l, L.B, P_u),
        C=galerkin(R_l, L.C, P_l),
        bs_u=n_ns_u,
        bs_l=n_ns_l,
        slave_nodes=slave_c,
        master_nodes=master_c,
        lm_node=np.arange(n_agg_l * n_ns_l) // n_ns_l,
        nullspace_u=ns_u_c,
        nullspace_l=ns_l_c,
    )


def build_hierarchy(prob, opts: AMGOptions = None, factor_coarsest: bool = True):
    """Levels 0..L-1; the last one carries the dense coarsest inverse.

    Coarsening continues while fewer than max_levels exist and the current
    coarsest level has more than max_coarse_rows rows.
    """
    opts = opts or AMGOptions()
    levels = [_level_from_problem(prob)]
    while len(levels) < opts.max_levels and levels[-1].n > opts.max_coarse_rows:
        nxt = coarsen(levels[-1], opts)
        if nxt.n >= levels[-1].n:
            break
        levels.append(nxt)
    simple_coarse = opts.coarse_solver == "simple"
    for L in levels if simple_coarse else levels[:-1]:
        smoother_data(L, opts)
    if factor_coarsest and not simple_coarse:
        coarse_inverse(levels[-1])
    return levels


def operator_complexity(levels) -> float:
    return sum(L.nnz() for L in levels) / levels[0].nnz()
