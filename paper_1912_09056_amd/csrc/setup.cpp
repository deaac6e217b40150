// Host construction of the fully coupled aggregation-AMG hierarchy for the
// mortar-contact saddle-point system (Sec. 4 of the paper; smoother data of
// Sec. 5.1.3; merged direct solve on the coarsest level as in the
// weak-scaling study's solver settings).
//
// Readings taken where the paper leaves details open:
//  * Dirichlet dof: a K row whose only stored entry is its diagonal and whose
//    G row is empty.  Nodes with all dofs Dirichlet are not aggregated; the
//    null-space rows of Dirichlet dofs are zero, so are their P rows.
//  * Node graph: stored K entries between non-Dirichlet dofs of different
//    nodes; pairs (slave interface node, master interface node) dropped
//    (Sec. 4.2).
//  * Aggregation: three greedy phases in natural node order -- roots whose
//    neighbourhood is untouched take all neighbours; leftovers join the
//    adjacent phase-1 aggregate with most neighbours (snapshot, ties to the
//    smallest id); remaining nodes seed aggregates with their free
//    neighbours.
//  * Alg. 1: slave displacement dofs in ascending order, "D_ij != 0" is a
//    stored entry of G's slave row; a pseudo-node keeps its first aggregate,
//    and a multiplier aggregate is created with its first member (with a
//    non-diagonal D an aggregate whose multipliers were all claimed earlier
//    gets none).
//  * Tentative transfers: per-aggregate modified Gram-Schmidt QR of the
//    null-space rows (ascending dof order, columns in order, R_kk > 0); the
//    pattern of P holds all n_ns coarse columns of the aggregate for every
//    contributing fine dof (explicit zeros kept); the multiplier null space
//    is one constant per Cartesian component.
//  * Galerkin blocks on the symbolic pattern of R A P (no dropping).
//  * Coarse interface nodes: aggregates containing interface nodes.
//  * Optional smoothed aggregation (Sec. 3.1.2, prolongator smoothing):
//    P = P_tent - omega Atilde^-1 K P_tent with the lumped diagonal
//    Atilde = diag(sum_j |K_ij|), whose bound lambda(Atilde^-1 K) <= 1 lets
//    the printed omega = 4/3 be used as is; pattern = P_tent's plus the
//    symbolic pattern of K P_tent.
//  * Braess-Sarazin (Sec. 5.1.2, Alg. 3) with damping alpha maps onto the
//    CheapSIMPLE data with the lumping alpha * Ahat (see smoother_data).
//  * Optional CheapSIMPLE coarse solver (the weak-scaling study's second
//    coarse-solver variant): smoother data on the coarsest level too, no
//    merged matrix and no factorisation.
//  * Optional Schur sweeps: S = B Atilde^-1 G - C on the symbolic pattern of
//    B G plus C's, diagonal either S_jj or sign(S_jj) sum_k |S_jk|.
#include "setup.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <numeric>
#include <thread>

namespace camg {

namespace {

[[noreturn]] void fail(int code, const std::string& m) { throw SetupError{code, m}; }

// Rows [r0, r1) of a CSR result computed by one chunk.
struct RowBlock {
  std::vector<int64_t> len;
  std::vector<int32_t> ci;
  std::vector<double> v;
};

// Concatenates per-chunk row blocks (in chunk order) into out.
void append_blocks(HostCSR& out, std::vector<RowBlock>& blocks) {
  int64_t total = 0;
  for (auto& b : blocks) total += (int64_t)b.ci.size();
  out.ci.reserve((size_t)total);
  out.v.reserve((size_t)total);
  int64_t r = 0;
  for (auto& b : blocks) {
    for (int64_t l : b.len) {
      out.rp[r + 1] = out.rp[r] + l;
      ++r;
    }
    out.ci.insert(out.ci.end(), b.ci.begin(), b.ci.end());
    out.v.insert(out.v.end(), b.v.begin(), b.v.end());
    RowBlock().len.swap(b.len);
    std::vector<int32_t>().swap(b.ci);
    std::vector<double>().swap(b.v);
  }
}

constexpr int kErrShape = -2;
constexpr int kErrZeroDiag = -4;
constexpr int kErrRankDeficient = -5;
constexpr int kErrSingularCoarse = -6;
constexpr int kErrUnmapped = -9;

std::vector<uint8_t> find_dirichlet(const HostCSR& K, const HostCSR& G) {
  std::vector<uint8_t> d((size_t)K.nrows, 0);
  for (int64_t i = 0; i < K.nrows; ++i) {
    int64_t a = K.rp[i], b = K.rp[i + 1];
    bool only_diag = (b - a == 1) && K.ci[a] == i;
    bool g_empty = G.rp[i + 1] == G.rp[i];
    d[i] = (only_diag && g_empty) ? 1 : 0;
  }
  return d;
}

// Node adjacency as CSR (sorted, unique, no self loops).
void node_graph(const HostLevel& L, std::vector<int64_t>& gp, std::vector<int32_t>& gi) {
  const int bs = L.bs_u;
  const int64_t nn = L.n_u() / bs;
  gp.assign((size_t)nn + 1, 0);
  gi.clear();
  std::vector<int64_t> mark((size_t)nn, -1);
  std::vector<int32_t> row;
  for (int64_t a = 0; a < nn; ++a) {
    row.clear();
    for (int c = 0; c < bs; ++c) {
      int64_t r = a * bs + c;
      if (L.dirichlet[r]) continue;
      for (int64_t k = L.K.rp[r]; k < L.K.rp[r + 1]; ++k) {
        int32_t col = L.K.ci[k];
        if (L.dirichlet[col]) continue;
        int64_t b = col / bs;
        if (b == a) continue;
        if ((L.slave_node[a] && L.master_node[b]) || (L.master_node[a] && L.slave_node[b])) continue;
        if (mark[b] != a) {
          mark[b] = a;
          row.push_back((int32_t)b);
        }
      }
    }
    std::sort(row.begin(), row.end());
    gi.insert(gi.end(), row.begin(), row.end());
    gp[a + 1] = (int64_t)gi.size();
  }
}

int64_t aggregate_nodes(const std::vector<int64_t>& gp, const std::vector<int32_t>& gi,
                        const std::vector<uint8_t>& active, std::vector<int32_t>& agg) {
  const int64_t n = (int64_t)active.size();
  agg.assign((size_t)n, -1);
  int64_t n_agg = 0;
  // phase 1: roots with untouched neighbourhoods
  for (int64_t i = 0; i < n; ++i) {
    if (!active[i] || agg[i] >= 0) continue;
    bool free_nbhd = true;
    for (int64_t k = gp[i]; k < gp[i + 1]; ++k) {
      int32_t j = gi[k];
      if (active[j] && agg[j] >= 0) {
        free_nbhd = false;
        break;
      }
    }
    if (!free_nbhd) continue;
    agg[i] = (int32_t)n_agg;
    for (int64_t k = gp[i]; k < gp[i + 1]; ++k)
      if (active[gi[k]]) agg[gi[k]] = (int32_t)n_agg;
    ++n_agg;
  }
  // phase 2: attach leftovers to the most connected phase-1 aggregate
  std::vector<int32_t> snap = agg;
  std::vector<int32_t> cand;
  for (int64_t i = 0; i < n; ++i) {
    if (!active[i] || snap[i] >= 0) continue;
    cand.clear();
    for (int64_t k = gp[i]; k < gp[i + 1]; ++k) {
      int32_t j = gi[k];
      if (active[j] && snap[j] >= 0) cand.push_back(snap[j]);
    }
    if (cand.empty()) continue;
    std::sort(cand.begin(), cand.end());
    int32_t best = cand[0];
    int best_cnt = 0;
    for (size_t s = 0; s < cand.size();) {
      size_t e = s;
      while (e < cand.size() && cand[e] == cand[s]) ++e;
      int cnt = (int)(e - s);
      if (cnt > best_cnt) {  // strict: equal counts keep the smaller id
        best_cnt = cnt;
        best = cand[s];
      }
      s = e;
    }
    agg[i] = best;
  }
  // phase 3: leftovers seed new aggregates with their free neighbours
  for (int64_t i = 0; i < n; ++i) {
    if (!active[i] || agg[i] >= 0) continue;
    agg[i] = (int32_t)n_agg;
    for (int64_t k = gp[i]; k < gp[i + 1]; ++k) {
      int32_t j = gi[k];
      if (active[j] && agg[j] < 0) agg[j] = (int32_t)n_agg;
    }
    ++n_agg;
  }
  return n_agg;
}

// Alg. 1 of the paper (Sec. 4.3).
int64_t lagmult_aggregation(const HostLevel& L, std::vector<int32_t>& agg_l) {
  const int bs = L.bs_u;
  agg_l.assign((size_t)L.n_nodes_l, -1);
  std::vector<int32_t> dmap((size_t)L.n_agg_u, -1);
  int64_t count = 0;
  const int64_t nn = L.n_u() / bs;
  for (int64_t node = 0; node < nn; ++node) {
    if (!L.slave_node[node]) continue;
    for (int c = 0; c < bs; ++c) {  // ascending slave dofs
      int64_t i = node * bs + c;
      int32_t k = L.agg_u[node];
      if (k < 0) continue;
      for (int64_t e = L.G.rp[i]; e < L.G.rp[i + 1]; ++e) {
        const int32_t pn = L.lm_node[L.G.ci[e]];
        if (agg_l[pn] >= 0) continue;  // first assignment wins
        if (dmap[k] < 0) dmap[k] = (int32_t)count++;  // created with its first member
        agg_l[pn] = dmap[k];
      }
    }
  }
  for (int64_t p = 0; p < L.n_nodes_l; ++p)
    if (agg_l[p] < 0) fail(kErrUnmapped, "multiplier pseudo-node coupled to no slave displacement dof");
  return count;
}

// Tentative prolongator by per-aggregate modified Gram-Schmidt.
// node_of(r) gives the node of fine row r (or -1), zero(r) marks zeroed rows.
template <class NodeOf, class Zero>
void tentative(int64_t n_rows, int n_ns, const std::vector<double>& ns, const std::vector<int32_t>& agg,
               int64_t n_agg, NodeOf node_of, Zero zero, HostCSR& P, std::vector<double>& ns_coarse) {
  std::vector<int32_t> row_agg((size_t)n_rows, -1);
  std::vector<int64_t> cnt((size_t)n_agg + 1, 0);
  for (int64_t r = 0; r < n_rows; ++r) {
    int64_t nd = node_of(r);
    if (nd < 0 || zero(r)) continue;
    int32_t a = agg[nd];
    if (a < 0) continue;
    row_agg[r] = a;
    cnt[a + 1]++;
  }
  for (int64_t a = 0; a < n_agg; ++a) cnt[a + 1] += cnt[a];
  std::vector<int64_t> rows((size_t)cnt[n_agg]);
  {
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t r = 0; r < n_rows; ++r)
      if (row_agg[r] >= 0) rows[pos[row_agg[r]]++] = r;  // ascending within each aggregate
  }
  std::vector<double> Pv((size_t)n_rows * n_ns, 0.0);
  const int64_t nc = n_agg * n_ns;
  ns_coarse.assign((size_t)nc * n_ns, 0.0);  // column-major, nc rows
  std::vector<double> Q, R((size_t)n_ns * n_ns);
  for (int64_t a = 0; a < n_agg; ++a) {
    const int64_t m = cnt[a + 1] - cnt[a];
    const int64_t* rr = rows.data() + cnt[a];
    Q.assign((size_t)m * n_ns, 0.0);  // column-major m x n_ns
    std::fill(R.begin(), R.end(), 0.0);
    for (int k = 0; k < n_ns; ++k) {
      double* v = Q.data() + (size_t)k * m;
      double orig = 0.0;
      for (int64_t s = 0; s < m; ++s) {
        v[s] = ns[(size_t)k * n_rows + rr[s]];
        orig += v[s] * v[s];
      }
      for (int i = 0; i < k; ++i) {
        const double* q = Q.data() + (size_t)i * m;
        double dot = 0.0;
        for (int64_t s = 0; s < m; ++s) dot += q[s] * v[s];
        R[(size_t)i * n_ns + k] = dot;
        for (int64_t s = 0; s < m; ++s) v[s] -= dot * q[s];
      }
      double nv = 0.0;
      for (int64_t s = 0; s < m; ++s) nv += v[s] * v[s];
      nv = std::sqrt(nv);
      if (!(nv > 1e-12 * std::sqrt(orig))) fail(kErrRankDeficient, "null space rank-deficient on an aggregate");
      R[(size_t)k * n_ns + k] = nv;
      for (int64_t s = 0; s < m; ++s) v[s] /= nv;
    }
    for (int64_t s = 0; s < m; ++s)
      for (int k = 0; k < n_ns; ++k) Pv[(size_t)rr[s] * n_ns + k] = Q[(size_t)k * m + s];
    for (int i = 0; i < n_ns; ++i)
      for (int k = 0; k < n_ns; ++k) ns_coarse[(size_t)k * nc + a * n_ns + i] = R[(size_t)i * n_ns + k];
  }
  P.init_empty(n_rows, nc);
  for (int64_t r = 0; r < n_rows; ++r) {
    if (row_agg[r] >= 0) {
      for (int k = 0; k < n_ns; ++k) {
        P.ci.push_back(row_agg[r] * n_ns + k);
        P.v.push_back(Pv[(size_t)r * n_ns + k]);
      }
    }
    P.rp[r + 1] = P.nnz();
  }
}

// Whether a square CSR matrix (sorted columns) equals its transpose bit for
// bit: every entry has a mirror entry holding the same value.
bool csr_equals_transpose(const HostCSR& A) {
  if (A.nrows != A.ncols) return false;
  std::atomic<bool> ok{true};
  parallel_for(A.nrows, [&](int64_t r0, int64_t r1) {
    for (int64_t i = r0; i < r1 && ok; ++i)
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int32_t j = A.ci[k];
        const auto b = A.ci.begin() + A.rp[j], e = A.ci.begin() + A.rp[j + 1];
        const auto it = std::lower_bound(b, e, (int32_t)i);
        if (it == e || *it != (int32_t)i || !(A.v[(size_t)(it - A.ci.begin())] == A.v[(size_t)k])) {
          ok = false;
          break;
        }
      }
  });
  return ok;
}

// Mirrored entries of a square CSR matrix with a symmetric pattern replaced
// by their mean, (A_ij + A_ji) / 2, the same number for both: the matrix
// then equals its transpose bit for bit.  Each pair is written by the row of
// its upper entry.
void symmetrize_values(HostCSR& A) {
  parallel_for(A.nrows, [&](int64_t r0, int64_t r1) {
    for (int64_t i = r0; i < r1; ++i)
      for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int32_t j = A.ci[k];
        if (j <= i) continue;
        const auto b = A.ci.begin() + A.rp[j], e = A.ci.begin() + A.rp[j + 1];
        const auto it = std::lower_bound(b, e, (int32_t)i);
        if (it == e || *it != (int32_t)i) continue;
        const size_t m = (size_t)(it - A.ci.begin());
        const double v = (A.v[(size_t)k] + A.v[m]) * 0.5;
        A.v[(size_t)k] = v;
        A.v[m] = v;
      }
  });
}

// R A P on the symbolic pattern.  Consecutive rows of R with identical
// column sets (the rows of one aggregate) share one pass over A P; groups
// are independent and run on the setup threads.
HostCSR galerkin(const HostCSR& R, const HostCSR& A, const HostCSR& P) {
  HostCSR out;
  out.init_empty(R.nrows, P.ncols);
  auto same = [&](int64_t a, int64_t b) {
    int64_t la = R.rp[a + 1] - R.rp[a], lb = R.rp[b + 1] - R.rp[b];
    if (la != lb) return false;
    return std::equal(R.ci.begin() + R.rp[a], R.ci.begin() + R.rp[a + 1], R.ci.begin() + R.rp[b]);
  };
  std::vector<int64_t> gstart;  // first row of each group, plus R.nrows
  for (int64_t r = 0; r < R.nrows; ++r)
    if (r == 0 || !same(r - 1, r)) gstart.push_back(r);
  gstart.push_back(R.nrows);
  const int64_t n_groups = (int64_t)gstart.size() - 1;
  constexpr int64_t kGroupsPerChunk = 64;
  const int64_t n_chunks = (n_groups + kGroupsPerChunk - 1) / kGroupsPerChunk;
  std::vector<RowBlock> blocks((size_t)n_chunks);
  const int nt = (int)std::min<int64_t>(setup_threads(), std::max<int64_t>(n_chunks, 1));
  std::vector<std::vector<int32_t>> locs((size_t)nt);
  parallel_chunks(n_chunks, nt, [&](int64_t c, int t) {
    std::vector<int32_t>& loc = locs[(size_t)t];
    if (loc.empty()) loc.assign((size_t)P.ncols, -1);
    std::vector<int32_t> touched, fine;
    std::vector<double> tmp;  // fine.size() x touched.size()
    RowBlock& blk = blocks[(size_t)c];
    const int64_t g1 = std::min(n_groups, (c + 1) * kGroupsPerChunk);
    for (int64_t g = c * kGroupsPerChunk; g < g1; ++g) {
      const int64_t r0 = gstart[(size_t)g], r1 = gstart[(size_t)g + 1];
      fine.assign(R.ci.begin() + R.rp[r0], R.ci.begin() + R.rp[r0 + 1]);
      touched.clear();
      for (int32_t i : fine)
        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
          int32_t j = A.ci[k];
          for (int64_t q = P.rp[j]; q < P.rp[j + 1]; ++q) {
            int32_t col = P.ci[q];
            if (loc[col] < 0) {
              loc[col] = (int32_t)touched.size();
              touched.push_back(col);
            }
          }
        }
      std::sort(touched.begin(), touched.end());
      for (size_t t = 0; t < touched.size(); ++t) loc[touched[t]] = (int32_t)t;
      const size_t ntc = touched.size();
      tmp.assign(fine.size() * ntc, 0.0);
      for (size_t f = 0; f < fine.size(); ++f) {
        int32_t i = fine[f];
        double* trow = tmp.data() + f * ntc;
        for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
          int32_t j = A.ci[k];
          double a = A.v[k];
          for (int64_t q = P.rp[j]; q < P.rp[j + 1]; ++q) trow[loc[P.ci[q]]] += a * P.v[q];
        }
      }
      for (int64_t r = r0; r < r1; ++r) {
        size_t base = blk.ci.size();
        blk.ci.insert(blk.ci.end(), touched.begin(), touched.end());
        blk.v.resize(base + ntc, 0.0);
        double* orow = blk.v.data() + base;
        int64_t f = 0;
        for (int64_t k = R.rp[r]; k < R.rp[r + 1]; ++k, ++f) {
          double w = R.v[k];
          const double* trow = tmp.data() + (size_t)f * ntc;
          for (size_t t = 0; t < ntc; ++t) orow[t] += w * trow[t];
        }
        blk.len.push_back((int64_t)ntc);
      }
      for (int32_t col : touched) loc[col] = -1;
    }
  });
  append_blocks(out, blocks);
  return out;
}

// Sorted union of the column patterns gathered by `visit`, with loc[] set to
// each column's position; returns the count.  loc must be all -1 on entry.
template <typename Visit>
size_t gather_pattern(std::vector<int32_t>& cols, std::vector<int32_t>& loc, Visit visit) {
  cols.clear();
  visit([&](int32_t c) {
    if (loc[c] < 0) {
      loc[c] = 0;
      cols.push_back(c);
    }
  });
  std::sort(cols.begin(), cols.end());
  for (size_t t = 0; t < cols.size(); ++t) loc[cols[t]] = (int32_t)t;
  return cols.size();
}

HostCSR smooth_prolongator(const HostCSR& K, const HostCSR& Pt, double omega) {
  HostCSR out;
  out.init_empty(K.nrows, Pt.ncols);
  constexpr int64_t kRowsPerChunk = 4096;
  const int64_t n_chunks = (K.nrows + kRowsPerChunk - 1) / kRowsPerChunk;
  std::vector<RowBlock> blocks((size_t)n_chunks);
  const int nt = (int)std::min<int64_t>(setup_threads(), std::max<int64_t>(n_chunks, 1));
  std::vector<std::vector<int32_t>> locs((size_t)nt);
  parallel_chunks(n_chunks, nt, [&](int64_t c, int t) {
    std::vector<int32_t>& loc = locs[(size_t)t];
    if (loc.empty()) loc.assign((size_t)Pt.ncols, -1);
    std::vector<int32_t> cols;
    std::vector<double> acc, ph;
    RowBlock& blk = blocks[(size_t)c];
    const int64_t i1 = std::min(K.nrows, (c + 1) * kRowsPerChunk);
    for (int64_t i = c * kRowsPerChunk; i < i1; ++i) {
      const size_t nc = gather_pattern(cols, loc, [&](auto add) {
        for (int64_t q = Pt.rp[i]; q < Pt.rp[i + 1]; ++q) add(Pt.ci[q]);
        for (int64_t k = K.rp[i]; k < K.rp[i + 1]; ++k)
          for (int64_t q = Pt.rp[K.ci[k]]; q < Pt.rp[K.ci[k] + 1]; ++q) add(Pt.ci[q]);
      });
      acc.assign(nc, 0.0);
      ph.assign(nc, 0.0);
      double rs = 0.0;
      for (int64_t k = K.rp[i]; k < K.rp[i + 1]; ++k) {
        const double a = K.v[k];
        rs += std::fabs(a);
        const int32_t j = K.ci[k];
        for (int64_t q = Pt.rp[j]; q < Pt.rp[j + 1]; ++q) acc[(size_t)loc[Pt.ci[q]]] += a * Pt.v[q];
      }
      for (int64_t q = Pt.rp[i]; q < Pt.rp[i + 1]; ++q) ph[(size_t)loc[Pt.ci[q]]] = Pt.v[q];
      if (rs == 0.0) fail(kErrZeroDiag, "zero row of K in prolongator smoothing");
      const double w = omega / rs;
      for (size_t t = 0; t < nc; ++t) {
        blk.ci.push_back(cols[t]);
        blk.v.push_back(ph[t] - w * acc[t]);
        loc[cols[t]] = -1;
      }
      blk.len.push_back((int64_t)nc);
    }
  });
  append_blocks(out, blocks);
  return out;
}

HostCSR schur_matrix(const HostLevel& L) {
  const int64_t nl = L.n_l();
  HostCSR out;
  out.init_empty(nl, nl);
  std::vector<int32_t> loc((size_t)nl, -1), cols;
  std::vector<double> acc;
  for (int64_t j = 0; j < nl; ++j) {
    const size_t nc = gather_pattern(cols, loc, [&](auto add) {
      for (int64_t k = L.B.rp[j]; k < L.B.rp[j + 1]; ++k)
        for (int64_t q = L.G.rp[L.B.ci[k]]; q < L.G.rp[L.B.ci[k] + 1]; ++q) add(L.G.ci[q]);
      for (int64_t q = L.C.rp[j]; q < L.C.rp[j + 1]; ++q) add(L.C.ci[q]);
    });
    acc.assign(nc, 0.0);
    for (int64_t k = L.B.rp[j]; k < L.B.rp[j + 1]; ++k) {
      const int32_t i = L.B.ci[k];
      const double bk = L.B.v[k] * L.atilde_inv[i];
      for (int64_t q = L.G.rp[i]; q < L.G.rp[i + 1]; ++q) acc[(size_t)loc[L.G.ci[q]]] += bk * L.G.v[q];
    }
    for (int64_t q = L.C.rp[j]; q < L.C.rp[j + 1]; ++q) acc[(size_t)loc[L.C.ci[q]]] -= L.C.v[q];
    for (size_t t = 0; t < nc; ++t) {
      out.ci.push_back(cols[t]);
      out.v.push_back(acc[t]);
      loc[cols[t]] = -1;
    }
    out.rp[j + 1] = out.nnz();
  }
  return out;
}

// In-place Gauss-Jordan inverse of a small dense row-major matrix with
// partial pivoting; false when a pivot is exactly zero.
bool invert_small(const double* a_in, double* inv, int bs) {
  double a[6][12] = {};
  for (int r = 0; r < bs; ++r) {
    for (int c = 0; c < bs; ++c) a[r][c] = a_in[r * bs + c];
    a[r][bs + r] = 1.0;
  }
  for (int c = 0; c < bs; ++c) {
    int piv = c;
    for (int r = c + 1; r < bs; ++r)
      if (std::fabs(a[r][c]) > std::fabs(a[piv][c])) piv = r;
    if (a[piv][c] == 0.0) return false;
    if (piv != c)
      for (int k = 0; k < 2 * bs; ++k) std::swap(a[c][k], a[piv][k]);
    const double d = 1.0 / a[c][c];
    for (int k = 0; k < 2 * bs; ++k) a[c][k] *= d;
    for (int r = 0; r < bs; ++r) {
      if (r == c || a[r][c] == 0.0) continue;
      const double f = a[r][c];
      for (int k = 0; k < 2 * bs; ++k) a[r][k] -= f * a[c][k];
    }
  }
  for (int r = 0; r < bs; ++r)
    for (int c = 0; c < bs; ++c) inv[r * bs + c] = a[r][bs + c];
  return true;
}

// Inverse nodal lumping blocks (scale * (K_ii + sum_{j != i} ||K_ij||_F I))^-1
// per node of bs consecutive dofs, row-major, n_u * bs values.  For symmetric
// K the blocks bound x^T K x from above (the block analogue of the row-sum
// bound), and a rotation of the node frames maps them to R A_i R^T.
std::vector<double> nodal_lumping_inverse(const HostCSR& K, int bs, double scale) {
  const int64_t n = K.nrows;
  if (bs < 1 || bs > 6 || n % bs) fail(kErrShape, "nodal lumping: node block size must be 1..6 and divide n_u");
  const int64_t nb = n / bs;
  std::vector<double> out((size_t)(n * bs));
  constexpr int64_t kNodesPerChunk = 2048;
  const int64_t n_chunks = (nb + kNodesPerChunk - 1) / kNodesPerChunk;
  const int nt = (int)std::min<int64_t>(setup_threads(), std::max<int64_t>(n_chunks, 1));
  std::vector<std::vector<double>> sqs((size_t)nt);
  parallel_chunks(n_chunks, nt, [&](int64_t c, int t) {
    std::vector<double>& sq = sqs[(size_t)t];
    if (sq.empty()) sq.assign((size_t)nb, 0.0);
    std::vector<int64_t> touched;
    const int64_t a1 = std::min(nb, (c + 1) * kNodesPerChunk);
    for (int64_t a = c * kNodesPerChunk; a < a1; ++a) {
      double blk[36] = {};
      touched.clear();
      for (int r = 0; r < bs; ++r) {
        const int64_t i = a * bs + r;
        for (int64_t k = K.rp[i]; k < K.rp[i + 1]; ++k) {
          const int64_t b = K.ci[k] / bs;
          if (b == a) {
            blk[r * bs + K.ci[k] % bs] += K.v[k];
          } else {
            if (sq[(size_t)b] == 0.0) touched.push_back(b);
            sq[(size_t)b] += K.v[k] * K.v[k];
          }
        }
      }
      std::sort(touched.begin(), touched.end());
      double off = 0.0;
      for (int64_t b : touched) {
        off += std::sqrt(sq[(size_t)b]);
        sq[(size_t)b] = 0.0;
      }
      for (int r = 0; r < bs; ++r) {
        blk[r * bs + r] += off;
        for (int q = 0; q < bs; ++q) blk[r * bs + q] *= scale;
      }
      if (!invert_small(blk, &out[(size_t)(a * bs * bs)], bs)) fail(kErrZeroDiag, "singular nodal lumping block");
    }
  });
  return out;
}

// P = P_tent - omega Atilde^-1 K P_tent with the inverse nodal lumping blocks,
// on the pattern of P_tent plus that of Atilde^-1 K P_tent (rows of a node
// share the union of their K P_tent patterns).
HostCSR smooth_prolongator_nodal(const HostCSR& K, const HostCSR& Pt, double omega, const std::vector<double>& ainv,
                                 int bs) {
  HostCSR out;
  out.init_empty(K.nrows, Pt.ncols);
  const int64_t nb = K.nrows / bs;
  constexpr int64_t kNodesPerChunk = 1024;
  const int64_t n_chunks = (nb + kNodesPerChunk - 1) / kNodesPerChunk;
  std::vector<RowBlock> blocks((size_t)n_chunks);
  const int nt = (int)std::min<int64_t>(setup_threads(), std::max<int64_t>(n_chunks, 1));
  std::vector<std::vector<int32_t>> locs((size_t)nt);
  parallel_chunks(n_chunks, nt, [&](int64_t c, int t) {
    std::vector<int32_t>& loc = locs[(size_t)t];
    if (loc.empty()) loc.assign((size_t)Pt.ncols, -1);
    std::vector<int32_t> cols, rowcols;
    std::vector<double> kp;
    RowBlock& blk = blocks[(size_t)c];
    const int64_t a1 = std::min(nb, (c + 1) * kNodesPerChunk);
    for (int64_t a = c * kNodesPerChunk; a < a1; ++a) {
      const size_t nc = gather_pattern(cols, loc, [&](auto add) {
        for (int r = 0; r < bs; ++r) {
          const int64_t i = a * bs + r;
          for (int64_t q = Pt.rp[i]; q < Pt.rp[i + 1]; ++q) add(Pt.ci[q]);
          for (int64_t k = K.rp[i]; k < K.rp[i + 1]; ++k)
            for (int64_t q = Pt.rp[K.ci[k]]; q < Pt.rp[K.ci[k] + 1]; ++q) add(Pt.ci[q]);
        }
      });
      // (K P_tent) rows of the node on the union pattern; inkp marks the
      // columns of that product's pattern
      kp.assign(nc * (size_t)bs, 0.0);
      std::vector<char> inkp(nc, 0), inrow(nc, 0);
      for (int r = 0; r < bs; ++r) {
        const int64_t i = a * bs + r;
        for (int64_t k = K.rp[i]; k < K.rp[i + 1]; ++k) {
          const int32_t j = K.ci[k];
          for (int64_t q = Pt.rp[j]; q < Pt.rp[j + 1]; ++q) {
            const size_t u = (size_t)loc[Pt.ci[q]];
            kp[(size_t)r * nc + u] += K.v[k] * Pt.v[q];
            inkp[u] = 1;
          }
        }
      }
      const double* M = &ainv[(size_t)(a * bs * bs)];
      std::vector<double> val(nc);
      for (int r = 0; r < bs; ++r) {
        const int64_t i = a * bs + r;
        std::fill(val.begin(), val.end(), 0.0);
        std::fill(inrow.begin(), inrow.end(), 0);
        for (int64_t q = Pt.rp[i]; q < Pt.rp[i + 1]; ++q) {
          val[(size_t)loc[Pt.ci[q]]] = Pt.v[q];
          inrow[(size_t)loc[Pt.ci[q]]] = 1;
        }
        for (int rr = 0; rr < bs; ++rr) {
          const double m = omega * M[r * bs + rr];
          if (m == 0.0) continue;
          for (size_t u = 0; u < nc; ++u) val[u] -= m * kp[(size_t)rr * nc + u];
        }
        int64_t len = 0;
        for (size_t u = 0; u < nc; ++u) {
          if (!inkp[u] && !inrow[u]) continue;  // row pattern: P_tent's row plus the node's K P_tent pattern
          blk.ci.push_back(cols[u]);
          blk.v.push_back(val[u]);
          ++len;
        }
        blk.len.push_back(len);
      }
      for (size_t u = 0; u < nc; ++u) loc[cols[u]] = -1;
    }
  });
  append_blocks(out, blocks);
  return out;
}

// B Atilde^-1 G - C with the inverse nodal lumping blocks, on the pattern of
// B Atilde^-1 G (every dof of a node B touches) plus C's.
HostCSR schur_matrix_nodal(const HostLevel& L, const std::vector<double>& ainv, int bs) {
  const int64_t nl = L.n_l();
  HostCSR out;
  out.init_empty(nl, nl);
  std::vector<int32_t> loc((size_t)nl, -1), cols;
  std::vector<double> acc;
  for (int64_t j = 0; j < nl; ++j) {
    const size_t nc = gather_pattern(cols, loc, [&](auto add) {
      for (int64_t k = L.B.rp[j]; k < L.B.rp[j + 1]; ++k) {
        const int64_t a = L.B.ci[k] / bs;
        for (int64_t i2 = a * bs; i2 < (a + 1) * bs; ++i2)
          for (int64_t q = L.G.rp[i2]; q < L.G.rp[i2 + 1]; ++q) add(L.G.ci[q]);
      }
      for (int64_t q = L.C.rp[j]; q < L.C.rp[j + 1]; ++q) add(L.C.ci[q]);
    });
    acc.assign(nc, 0.0);
    for (int64_t k = L.B.rp[j]; k < L.B.rp[j + 1]; ++k) {
      const int64_t i = L.B.ci[k], a = i / bs;
      const double* M = &ainv[(size_t)(a * bs * bs + (i % bs) * bs)];
      for (int c = 0; c < bs; ++c) {
        const double bk = L.B.v[k] * M[c];
        const int64_t i2 = a * bs + c;
        for (int64_t q = L.G.rp[i2]; q < L.G.rp[i2 + 1]; ++q) acc[(size_t)loc[L.G.ci[q]]] += bk * L.G.v[q];
      }
    }
    for (int64_t q = L.C.rp[j]; q < L.C.rp[j + 1]; ++q) acc[(size_t)loc[L.C.ci[q]]] -= L.C.v[q];
    for (size_t t = 0; t < nc; ++t) {
      out.ci.push_back(cols[t]);
      out.v.push_back(acc[t]);
      loc[cols[t]] = -1;
    }
    out.rp[j + 1] = out.nnz();
  }
  return out;
}

// Relaxation data of the Schur system from S: inverse nodal blocks
// (schur = 2), else the inverse diagonal (schur = 0) or signed l1 row sums
// (schur = 1); S itself is kept for schur_sweeps > 1.
void schur_relaxation(HostLevel& L, HostCSR S, const SetupOptions& opt) {
  const int64_t nl = L.n_l();
  L.sd_inv.assign((size_t)nl, 0.0);
  L.sblk_inv.clear();
  if (opt.schur == 2) {
    // nodal block Jacobi: inverses of S's bs_l x bs_l diagonal blocks (the
    // multipliers of one node are consecutive)
    const int bs = L.bs_l;
    if (bs <= 0 || bs > 3 || nl % bs) fail(kErrShape, "multiplier count is not a multiple of the node block size");
    for (int64_t j = 0; j < (int64_t)L.lm_node.size(); ++j)
      if (L.lm_node[(size_t)j] != j / bs) fail(kErrShape, "block Schur relaxation needs node-contiguous multipliers");
    L.sblk_inv.assign((size_t)(nl * bs), 0.0);
    for (int64_t nd = 0; nd < nl / bs; ++nd) {
      double a[9] = {};
      for (int r = 0; r < bs; ++r) {
        const int64_t j = nd * bs + r;
        for (int64_t k = S.rp[j]; k < S.rp[j + 1]; ++k) {
          const int64_t c = S.ci[k] - nd * bs;
          if (c >= 0 && c < bs) a[r * bs + c] = S.v[k];
        }
      }
      if (!invert_small(a, &L.sblk_inv[(size_t)(nd * bs * bs)], bs)) fail(kErrZeroDiag, "singular Schur node block");
    }
  } else {
    for (int64_t j = 0; j < nl; ++j) {
      double d = 0.0, l1 = 0.0;
      for (int64_t k = S.rp[j]; k < S.rp[j + 1]; ++k) {
        l1 += std::fabs(S.v[k]);
        if (S.ci[k] == j) d = S.v[k];
      }
      const double sd = opt.schur == 1 ? (d > 0.0 ? l1 : (d < 0.0 ? -l1 : 0.0)) : d;
      if (sd == 0.0) fail(kErrZeroDiag, "zero diagonal of the Schur approximation");
      L.sd_inv[(size_t)j] = 1.0 / sd;
    }
  }
  if (opt.schur_sweeps > 1) L.S = std::move(S);
}

void smoother_data(HostLevel& L, const SetupOptions& opt) {
  const int64_t nu = L.n_u(), nl = L.n_l();
  std::vector<double> at((size_t)nu), dg((size_t)nu, 0.0);
  for (int64_t i = 0; i < nu; ++i) {
    double s = 0.0;
    for (int64_t k = L.K.rp[i]; k < L.K.rp[i + 1]; ++k) {
      s += std::fabs(L.K.v[k]);
      if (L.K.ci[k] == i) dg[i] = L.K.v[k];
    }
    at[i] = s;
  }
  for (int64_t i = 0; i < nu; ++i)
    if (dg[i] == 0.0) fail(kErrZeroDiag, "zero diagonal entry in K");
  L.ablk_inv.clear();
  if (opt.atilde == 2) {
    // nodal lumping: its blocks relax the prediction, back-substitute and
    // form S; Braess-Sarazin folds its alpha into them
    const int bs = L.bs_u;
    L.ablk_inv = nodal_lumping_inverse(L.K, bs, opt.bs_alpha > 0.0 ? opt.bs_alpha : 1.0);
    L.atilde_inv.assign((size_t)nu, 0.0);  // the point vectors are unused
    L.jac_inv.assign((size_t)nu, 0.0);
    schur_relaxation(L, schur_matrix_nodal(L, L.ablk_inv, bs), opt);
    return;
  }
  L.atilde_inv.resize((size_t)nu);
  L.jac_inv.resize((size_t)nu);
  for (int64_t i = 0; i < nu; ++i) {
    double a = opt.atilde == 0 ? at[i] : dg[i];
    if (a == 0.0) fail(kErrZeroDiag, "zero SIMPLEC lumping");
    if (opt.bs_alpha > 0.0) {
      // Braess-Sarazin with damping alpha is the CheapSIMPLE sweep with the
      // lumping alpha * Ahat, unit dampings and that lumping as the
      // prediction's diagonal: its Schur matrix is B Ahat^-1 G / alpha - C
      a *= opt.bs_alpha;
      L.atilde_inv[i] = 1.0 / a;
      L.jac_inv[i] = 1.0 / a;
      continue;
    }
    L.atilde_inv[i] = 1.0 / a;
    L.jac_inv[i] = opt.jacobi_diag == 0 ? 1.0 / a : 1.0 / dg[i];
  }
  L.sd_inv.resize((size_t)nl);
  L.sblk_inv.clear();
  if (opt.schur == 2 || opt.schur == 1 || opt.schur_sweeps > 1) {
    schur_relaxation(L, schur_matrix(L), opt);
    return;
  }
  // S_d[j] = sum_i B[j,i] G[i,j] / Atilde_i - C[j,j]
  for (int64_t j = 0; j < nl; ++j) {
    double s = 0.0;
    for (int64_t k = L.B.rp[j]; k < L.B.rp[j + 1]; ++k) {
      int32_t i = L.B.ci[k];
      auto b = L.G.ci.begin() + L.G.rp[i], e = L.G.ci.begin() + L.G.rp[i + 1];
      auto it = std::lower_bound(b, e, (int32_t)j);
      if (it != e && *it == j) s += L.B.v[k] * L.G.v[it - L.G.ci.begin()] * L.atilde_inv[i];
    }
    double c = 0.0;
    {
      auto b = L.C.ci.begin() + L.C.rp[j], e = L.C.ci.begin() + L.C.rp[j + 1];
      auto it = std::lower_bound(b, e, (int32_t)j);
      if (it != e && *it == j) c = L.C.v[it - L.C.ci.begin()];
    }
    double sd = s - c;
    if (sd == 0.0) fail(kErrZeroDiag, "zero diagonal of the Schur approximation");
    L.sd_inv[j] = 1.0 / sd;
  }
}

// Dense LU with partial pivoting (largest magnitude, first index on ties)
// of the merged coarsest matrix, then its explicit inverse.
// The coarsest level's blocks merged into one dense row-major matrix, and
// its largest entry magnitude.
static double merge_dense(const HostLevel& L, std::vector<double>& A) {
  const int64_t nu = L.n_u(), n = L.n();
  A.assign((size_t)(n * n), 0.0);
  auto put = [&](const HostCSR& M, int64_t r0, int64_t c0) {
    for (int64_t i = 0; i < M.nrows; ++i)
      for (int64_t k = M.rp[i]; k < M.rp[i + 1]; ++k) A[(size_t)((r0 + i) * n + c0 + M.ci[k])] += M.v[k];
  };
  put(L.K, 0, 0);
  put(L.G, 0, nu);
  put(L.B, nu, 0);
  put(L.C, nu, nu);
  double amax = 0.0;
  for (double a : A) amax = std::max(amax, std::fabs(a));
  return amax;
}

void coarse_inverse(HostLevel& L) {
  const int64_t n = L.n();
  std::vector<double> A;
  const double amax = merge_dense(L, A);
  std::vector<int64_t> piv((size_t)n);
  for (int64_t k = 0; k < n; ++k) {
    int64_t p = k;
    double best = std::fabs(A[(size_t)(k * n + k)]);
    for (int64_t i = k + 1; i < n; ++i) {
      double v = std::fabs(A[(size_t)(i * n + k)]);
      if (v > best) {
        best = v;
        p = i;
      }
    }
    if (!(best > 1e-13 * amax)) fail(kErrSingularCoarse, "coarsest merged matrix is singular");
    piv[k] = p;
    if (p != k)
      for (int64_t j = 0; j < n; ++j) std::swap(A[(size_t)(k * n + j)], A[(size_t)(p * n + j)]);
    const double d = A[(size_t)(k * n + k)];
    for (int64_t i = k + 1; i < n; ++i) {
      double l = A[(size_t)(i * n + k)] / d;
      A[(size_t)(i * n + k)] = l;
      if (l != 0.0)
        for (int64_t j = k + 1; j < n; ++j) A[(size_t)(i * n + j)] -= l * A[(size_t)(k * n + j)];
    }
  }
  // inverse: solve A X = I column by column (row-major X)
  L.Ainv.assign((size_t)(n * n), 0.0);
  std::vector<double> x((size_t)n);
  for (int64_t c = 0; c < n; ++c) {
    std::fill(x.begin(), x.end(), 0.0);
    x[c] = 1.0;
    for (int64_t k = 0; k < n; ++k) std::swap(x[k], x[piv[k]]);
    for (int64_t i = 0; i < n; ++i) {
      double s = x[i];
      for (int64_t j = 0; j < i; ++j) s -= A[(size_t)(i * n + j)] * x[j];
      x[i] = s;
    }
    for (int64_t i = n - 1; i >= 0; --i) {
      double s = x[i];
      for (int64_t j = i + 1; j < n; ++j) s -= A[(size_t)(i * n + j)] * x[j];
      x[i] = s / A[(size_t)(i * n + i)];
    }
    for (int64_t i = 0; i < n; ++i) L.Ainv[(size_t)(i * n + c)] = x[i];
  }
}

HostLevel coarsen(HostLevel& L, const SetupOptions& opt) {
  const int bs = L.bs_u;
  const int64_t nn = L.n_u() / bs;
  PhaseTimer pt_all("coarsen (level total)");
  L.dirichlet = find_dirichlet(L.K, L.G);
  std::vector<uint8_t> active((size_t)nn, 0);
  for (int64_t a = 0; a < nn; ++a)
    for (int c = 0; c < bs; ++c)
      if (!L.dirichlet[a * bs + c]) active[a] = 1;
  std::vector<int64_t> gp;
  std::vector<int32_t> gi;
  {
    PhaseTimer pt("node graph + aggregation");
    node_graph(L, gp, gi);
    L.n_agg_u = aggregate_nodes(gp, gi, active, L.agg_u);
    L.n_agg_l = lagmult_aggregation(L, L.agg_l);
  }

  HostLevel Cn;
  std::vector<double> nsc_u, nsc_l;
  tentative(
      L.n_u(), L.n_ns_u, L.ns_u, L.agg_u, L.n_agg_u, [&](int64_t r) { return r / bs; },
      [&](int64_t r) { return L.dirichlet[r] != 0; }, L.P_u, nsc_u);
  tentative(
      L.n_l(), L.n_ns_l, L.ns_l, L.agg_l, L.n_agg_l, [&](int64_t r) { return (int64_t)L.lm_node[r]; },
      [&](int64_t) { return false; }, L.P_l, nsc_l);
  if (opt.prolongator == 1)
    L.P_u = opt.atilde == 2 ? smooth_prolongator_nodal(L.K, L.P_u, opt.sa_omega,
                                                       nodal_lumping_inverse(L.K, L.bs_u, 1.0), L.bs_u)
                            : smooth_prolongator(L.K, L.P_u, opt.sa_omega);
  HostCSR Ru = transpose(L.P_u), Rl = transpose(L.P_l);
  {
    PhaseTimer pt("galerkin");
    Cn.K = galerkin(Ru, L.K, L.P_u);
    // with K = K^T and R = P^T the coarse K is symmetric in exact arithmetic,
    // but its sums reach mirrored entries in different orders: restore the
    // symmetry bit for bit (a change of rounding size), so the coarse level
    // can use the symmetric blocked-ELL storage too
    if (L.k_symmetric) {
      symmetrize_values(Cn.K);
      Cn.k_symmetric = csr_equals_transpose(Cn.K);
    }
    Cn.G = galerkin(Ru, L.G, L.P_l);
    Cn.B = galerkin(Rl, L.B, L.P_u);
    Cn.C = galerkin(Rl, L.C, L.P_l);
  }
  Cn.bs_u = L.n_ns_u;
  Cn.bs_l = L.n_ns_l;
  Cn.n_ns_u = L.n_ns_u;
  Cn.n_ns_l = L.n_ns_l;
  Cn.slave_node.assign((size_t)L.n_agg_u, 0);
  Cn.master_node.assign((size_t)L.n_agg_u, 0);
  for (int64_t a = 0; a < nn; ++a) {
    int32_t g = L.agg_u[a];
    if (g < 0) continue;
    if (L.slave_node[a]) Cn.slave_node[g] = 1;
    if (L.master_node[a]) Cn.master_node[g] = 1;
  }
  Cn.n_nodes_l = L.n_agg_l;
  Cn.lm_node.resize((size_t)(L.n_agg_l * L.n_ns_l));
  for (size_t j = 0; j < Cn.lm_node.size(); ++j) Cn.lm_node[j] = (int32_t)(j / L.n_ns_l);
  Cn.ns_u = std::move(nsc_u);
  Cn.ns_l = std::move(nsc_l);
  return Cn;
}

}  // namespace

HostCSR transpose(const HostCSR& A, std::vector<int32_t>* perm) {
  HostCSR T;
  T.init_empty(A.ncols, A.nrows);
  for (int32_t c : A.ci) T.rp[c + 1]++;
  for (int64_t i = 0; i < A.ncols; ++i) T.rp[i + 1] += T.rp[i];
  T.ci.resize(A.ci.size());
  T.v.resize(A.ci.size());
  if (perm) perm->resize(A.ci.size());
  std::vector<int64_t> pos(T.rp.begin(), T.rp.end() - 1);
  for (int64_t i = 0; i < A.nrows; ++i)
    for (int64_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      int64_t p = pos[A.ci[k]]++;
      T.ci[p] = (int32_t)i;
      T.v[p] = A.v[k];
      if (perm) (*perm)[k] = (int32_t)p;
    }
  return T;
}

void build_hierarchy(std::vector<HostLevel>& levels, const SetupOptions& opt) {
  {
    PhaseTimer pt("symmetry check");
    levels[0].k_symmetric = csr_equals_transpose(levels[0].K);
  }
  while ((int)levels.size() < opt.max_levels && levels.back().n() > opt.max_coarse_rows) {
    HostLevel nxt = coarsen(levels.back(), opt);
    if (nxt.n() >= levels.back().n()) {
      // no coarsening progress: drop the aggregation data of the last level
      HostLevel& L = levels.back();
      L.agg_u.clear();
      L.agg_l.clear();
      L.n_agg_u = L.n_agg_l = 0;
      L.P_u = HostCSR();
      L.P_l = HostCSR();
      break;
    }
    levels.push_back(std::move(nxt));
  }
  const size_t n_smooth = opt.simple_coarse ? levels.size() : levels.size() - 1;
  {
    PhaseTimer pt("smoother data");
    for (size_t l = 0; l < n_smooth; ++l) smoother_data(levels[l], opt);
  }
  PhaseTimer pt("coarsest inverse");
  if (!opt.simple_coarse) {
    if (opt.device_inverse) {
      HostLevel& C = levels.back();
      C.Adense_amax = merge_dense(C, C.Adense);
    } else {
      coarse_inverse(levels.back());
    }
  }
}

}  // namespace camg
