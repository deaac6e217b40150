// Host-side construction of the fully coupled aggregation-AMG hierarchy.
//
// Runs once per amg_setup (outside the timed solve).  Integer work
// (aggregation, multiplier aggregation) is inherently sequential greedy
// graph work; the numeric products are row-parallel-friendly but small
// next to the solve, so both stay on the host here and the results are
// uploaded.
#pragma once

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <exception>
#include <string>
#include <thread>
#include <vector>

namespace camg {

struct HostCSR {
  int64_t nrows = 0, ncols = 0;
  std::vector<int64_t> rp;  // nrows + 1
  std::vector<int32_t> ci;
  std::vector<double> v;
  int64_t nnz() const { return (int64_t)ci.size(); }
  void init_empty(int64_t r, int64_t c) {
    nrows = r;
    ncols = c;
    rp.assign((size_t)r + 1, 0);
    ci.clear();
    v.clear();
  }
};

// Host threads for the row-independent products: OMP_NUM_THREADS when set
// (the process's CPU share), else the hardware count, at most 64.
inline int setup_threads() {
  int n = 0;
  if (const char* e = std::getenv("OMP_NUM_THREADS")) n = std::atoi(e);
  if (n <= 0) n = (int)std::thread::hardware_concurrency();
  return std::max(1, std::min(n, 64));
}

// Runs body(c, t) for every chunk c in [0, n_chunks) on nt threads (t is
// the thread's index in [0, nt), for per-thread scratch), chunks handed out
// in increasing order.  Results must depend only on the chunk, never on the
// thread, so the output is identical for any thread count.  The first
// exception thrown by a body is rethrown after all threads end.
template <typename Body>
void parallel_chunks(int64_t n_chunks, int nt, Body body) {
  if (nt <= 1) {
    for (int64_t c = 0; c < n_chunks; ++c) body(c, 0);
    return;
  }
  std::atomic<int64_t> next{0};
  std::exception_ptr err;
  std::atomic<bool> failed{false};
  auto work = [&](int t) {
    for (;;) {
      const int64_t c = next.fetch_add(1);
      if (c >= n_chunks || failed.load()) return;
      try {
        body(c, t);
      } catch (...) {
        if (!failed.exchange(true)) err = std::current_exception();
        return;
      }
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nt; ++t) pool.emplace_back(work, t);
  work(0);
  for (auto& t : pool) t.join();
  if (err) std::rethrow_exception(err);
}

// body(i0, i1) over [0, n) in chunks of `grain` on the setup threads
// (element-wise loops whose result does not depend on the split).
template <typename Body>
void parallel_for(int64_t n, Body body, int64_t grain = 1 << 16) {
  const int64_t n_chunks = (n + grain - 1) / grain;
  const int nt = (int)std::min<int64_t>(setup_threads(), std::max<int64_t>(n_chunks, 1));
  parallel_chunks(n_chunks, nt, [&](int64_t c, int) { body(c * grain, std::min(n, (c + 1) * grain)); });
}

// Setup phase timing on stderr when CAMG_SETUP_TIMING=1 (diagnostics only).
struct PhaseTimer {
  const char* name;
  std::chrono::steady_clock::time_point t0;
  explicit PhaseTimer(const char* n) : name(n), t0(std::chrono::steady_clock::now()) {}
  ~PhaseTimer() {
    static const bool on = [] {
      const char* e = std::getenv("CAMG_SETUP_TIMING");
      return e && e[0] == '1';
    }();
    if (!on) return;
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    std::fprintf(stderr, "[camg setup] %-28s %8.3f s\n", name, sec);
  }
};

struct HostLevel {
  HostCSR K, G, B, C;
  bool k_symmetric = false;        // K equals its transpose bit for bit
  int bs_u = 0, bs_l = 0;          // dofs per displacement node / multiplier node
  int n_ns_u = 0, n_ns_l = 0;      // null-space columns (next level's block sizes)
  std::vector<uint8_t> slave_node, master_node;  // per displacement node
  std::vector<int32_t> lm_node;    // multiplier dof -> pseudo-node
  int64_t n_nodes_l = 0;
  std::vector<double> ns_u, ns_l;  // column-major null spaces
  std::vector<uint8_t> dirichlet;  // per displacement dof
  std::vector<int32_t> agg_u, agg_l;
  int64_t n_agg_u = 0, n_agg_l = 0;
  HostCSR P_u, P_l;
  std::vector<double> atilde_inv, jac_inv, sd_inv;
  std::vector<double> sblk_inv;    // block Schur option: inverse nodal blocks, bs_l x bs_l row-major each
  std::vector<double> ablk_inv;    // nodal lumping option: inverse blocks, bs_u x bs_u row-major each
  HostCSR S;                       // B Atilde^-1 G - C (only when relaxed by Jacobi sweeps)
  std::vector<double> Ainv;        // coarsest level with the direct solve: dense inverse, row-major
  std::vector<double> Adense;      // ... or the merged dense matrix (row-major), inverted on the device
  double Adense_amax = 0.0;        // max |entry| of Adense (singularity threshold)
  int64_t n_u() const { return K.nrows; }
  int64_t n_l() const { return C.nrows; }
  int64_t n() const { return n_u() + n_l(); }
  int64_t nnz_all() const { return K.nnz() + G.nnz() + B.nnz() + C.nnz(); }
};

struct SetupOptions {
  int max_levels = 4;
  int max_coarse_rows = 1000;
  int atilde = 0;       // 0 row sums of |K|, 1 diag(K), 2 nodal blocks
  int jacobi_diag = 0;  // 0 Atilde, 1 diag(K)
  int prolongator = 0;  // 0 tentative, 1 smoothed (displacement transfers)
  double sa_omega = 4.0 / 3.0;
  int schur = 0;         // 0 diagonal of S, 1 signed l1 row sums of S, 2 nodal blocks of S
  int schur_sweeps = 1;  // > 1: keep S for Jacobi sweeps
  bool simple_coarse = false;  // coarsest level smooths (smoother data, no dense inverse)
  bool device_inverse = false; // coarsest level: keep the merged matrix for the device LU (no host LU)
  // Braess-Sarazin: > 0 scales the lumping to lumping * bs_alpha, which then
  // also serves as the prediction's diagonal (the sweep runs with unit dampings)
  double bs_alpha = 0.0;
};

// Status codes mirror the C-ABI's CAMG_* values.
struct SetupError {
  int code;
  std::string msg;
};

// Transpose keeping explicit zeros; rows of the result are sorted.
// If perm is given, perm[k] = position of input entry k in the output.
HostCSR transpose(const HostCSR& A, std::vector<int32_t>* perm = nullptr);

// Builds all levels.  levels[0] must hold K, G, B, C, bs_u/bs_l, n_ns_*,
// node masks, lm_node, n_nodes_l and the level-0 null spaces.
void build_hierarchy(std::vector<HostLevel>& levels, const SetupOptions& opt);

}  // namespace camg
