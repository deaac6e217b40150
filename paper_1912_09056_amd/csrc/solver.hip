// libcamg: C-ABI, device hierarchy, V-cycle and FGMRES orchestration.
//
// Host code here only sequences kernels; every vector operation of the
// solve phase runs on the GPU.  The only per-iteration device-to-host
// traffic is a 32-byte result block (Hessenberg residual estimate and Arnoldi
// norm), read one Arnoldi step behind the launches so the device never waits
// for the host: when step j-1 meets the tolerance, the already launched step
// j is discarded and never enters the solution.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/camg.h"
#include "common.hpp"
#include "dense_inverse.hpp"
#include "kernels.hpp"
#include "setup.hpp"

namespace camg {

thread_local std::string g_last_error;

struct ApiError {
  int code;
  std::string msg;
};

[[noreturn]] static void api_fail(int code, const std::string& m) { throw ApiError{code, m}; }

// ---------------------------------------------------------------------------
// device matrices

struct DevMat {
  int32_t nrows = 0, ncols = 0;
  int64_t nnz = 0;
  DBuf<int32_t> rp, ci;
  DBuf<double> v64;
  DBuf<float> v32;
  int32_t bs = 0;  // > 0: node-blocked copy present (see DCSR)
  DBuf<int32_t> bptr, bcol;
  DBuf<double> bv64;
  DBuf<float> bv32;
  template <typename T>
  DCSR<T> view() const;
};

template <>
DCSR<double> DevMat::view<double>() const {
  DCSR<double> d;
  d.nrows = nrows;
  d.ncols = ncols;
  d.nnz = nnz;
  d.rp = rp.p;
  d.ci = ci.p;
  d.v = v64.p;
  if (bs > 0 && bv64.p) {
    d.bs = bs;
    d.bptr = bptr.p;
    d.bcol = bcol.p;
    d.bval = bv64.p;
  }
  return d;
}
template <>
DCSR<float> DevMat::view<float>() const {
  DCSR<float> d;
  d.nrows = nrows;
  d.ncols = ncols;
  d.nnz = nnz;
  d.rp = rp.p;
  d.ci = ci.p;
  d.v = v32.p;
  if (bs > 0 && bv32.p) {
    d.bs = bs;
    d.bptr = bptr.p;
    d.bcol = bcol.p;
    d.bval = bv32.p;
  }
  return d;
}

static void upload_mat(DevMat& D, const HostCSR& H, bool f64, bool f32, hipStream_t s) {
  D.nrows = (int32_t)H.nrows;
  D.ncols = (int32_t)H.ncols;
  D.nnz = H.nnz();
  std::vector<int32_t> rp32(H.rp.size());
  for (size_t i = 0; i < H.rp.size(); ++i) rp32[i] = (int32_t)H.rp[i];
  D.rp.upload(rp32, s);
  D.ci.upload(H.ci, s);
  if (f64) D.v64.upload(H.v, s);
  if (f32) {
    std::vector<float> v32(H.v.size());
    parallel_for((int64_t)v32.size(), [&](int64_t i0, int64_t i1) {
      for (int64_t i = i0; i < i1; ++i) v32[(size_t)i] = (float)H.v[(size_t)i];
    });
    D.v32.upload(v32, s);
  }
  CAMG_HIP(hipStreamSynchronize(s));  // host staging vectors go out of scope
}

// Node-blocked copy of a CSR matrix whose rows are unions of full bs x bs
// blocks with the same block columns for all bs rows of a node (the coarse
// Galerkin blocks K_c = R K P have this shape); false otherwise.
static bool upload_rowblock(DevMat& D, const HostCSR& H, int bs, bool f64, bool f32, hipStream_t s) {
  if (bs != 3 && bs != 6) return false;
  if (H.nrows % bs || H.ncols % bs) return false;
  const int64_t nn = H.nrows / bs;
  std::vector<int32_t> bptr((size_t)nn + 1, 0), bcol;
  std::vector<double> val;
  for (int64_t nd = 0; nd < nn; ++nd) {
    const int64_t r0 = nd * bs;
    const int64_t len = H.rp[r0 + 1] - H.rp[r0];
    if (len % bs) return false;
    for (int a = 0; a < bs; ++a) {
      const int64_t ra = r0 + a;
      if (H.rp[ra + 1] - H.rp[ra] != len) return false;
      for (int64_t k = 0; k < len; ++k) {
        const int32_t c = H.ci[H.rp[ra] + k], c0 = H.ci[H.rp[r0] + k];
        if (c != c0) return false;
        if (k % bs == 0 ? c % bs != 0 : c != H.ci[H.rp[ra] + k - 1] + 1) return false;
      }
    }
    const int64_t nb = len / bs;
    for (int64_t q = 0; q < nb; ++q) {
      bcol.push_back(H.ci[H.rp[r0] + q * bs] / bs);
      for (int a = 0; a < bs; ++a)
        for (int b = 0; b < bs; ++b) val.push_back(H.v[H.rp[r0 + a] + q * bs + b]);
    }
    bptr[(size_t)nd + 1] = (int32_t)bcol.size();
  }
  D.bs = bs;
  D.bptr.upload(bptr, s);
  D.bcol.upload(bcol, s);
  if (f64) D.bv64.upload(val, s);
  if (f32) {
    std::vector<float> v32(val.begin(), val.end());
    D.bv32.upload(v32, s);
  }
  CAMG_HIP(hipStreamSynchronize(s));
  return true;
}

// Sliced blocked-ELL copy of a square node-blocked CSR matrix.
struct HostBell {
  int32_t n_nodes = 0, bs = 0, n_slices = 0;
  int64_t n_blocks = 0;
  std::vector<int32_t> slice_ptr, bcol;
  std::vector<int16_t> bdel;  // bcol as deltas from the lane's node, when all fit in 16 bits
  std::vector<double> val;
  std::vector<int64_t> pos;  // CSR entry -> index into val (-1: not stored, symmetric storage)
  // symmetric storage (the DBELL comment in common.hpp): lower positions
  bool sym = false;
  std::vector<int32_t> lptr, lidx;
  int64_t n_lower = 0;     // blocks left of the diagonal (read through their mirrors)
  int64_t nnz_stored = 0;  // CSR entries in the stored blocks
};

// Whether a square CSR matrix equals its transpose exactly (pattern and
// values); At is its transpose with sorted columns.
static bool csr_symmetric(const HostCSR& A, const HostCSR& At) {
  return A.rp == At.rp && A.ci == At.ci && A.v == At.v;
}

static HostBell make_bell(const HostCSR& A, int bs) {
  HostBell B;
  B.bs = bs;
  B.n_nodes = (int32_t)(A.nrows / bs);
  B.n_slices = (B.n_nodes + 63) / 64;
  const int nt = setup_threads();
  // sorted distinct block columns of every node, one slice (64 nodes) per chunk
  std::vector<std::vector<int32_t>> sl_cols((size_t)B.n_slices);
  std::vector<std::vector<int32_t>> sl_cnt((size_t)B.n_slices);
  parallel_chunks(B.n_slices, nt, [&](int64_t sl, int) {
    std::vector<int32_t> tmp;
    auto& cols = sl_cols[(size_t)sl];
    auto& cnt = sl_cnt[(size_t)sl];
    for (int32_t i = (int32_t)sl * 64; i < std::min(B.n_nodes, (int32_t)sl * 64 + 64); ++i) {
      tmp.clear();
      for (int a = 0; a < bs; ++a) {
        const int64_t r = (int64_t)i * bs + a;
        for (int64_t k = A.rp[r]; k < A.rp[r + 1]; ++k) tmp.push_back(A.ci[k] / bs);
      }
      std::sort(tmp.begin(), tmp.end());
      tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
      cols.insert(cols.end(), tmp.begin(), tmp.end());
      cnt.push_back((int32_t)tmp.size());
    }
  });
  B.slice_ptr.assign((size_t)B.n_slices + 1, 0);
  int64_t nblk = 0;
  for (int32_t sl = 0; sl < B.n_slices; ++sl) {
    int32_t w = 0;
    for (int32_t c : sl_cnt[(size_t)sl]) w = std::max(w, c);
    B.slice_ptr[sl + 1] = B.slice_ptr[sl] + w;
    nblk += (int64_t)sl_cols[(size_t)sl].size();
  }
  B.n_blocks = nblk;
  const int64_t npos = B.slice_ptr[B.n_slices];
  B.bcol.assign((size_t)(npos * 64), 0);
  B.val.assign((size_t)(npos * 64 * bs * bs), 0.0);
  B.pos.resize((size_t)A.nnz());
  parallel_chunks(B.n_slices, nt, [&](int64_t sl, int) {
    const auto& cols = sl_cols[(size_t)sl];
    const auto& cnt = sl_cnt[(size_t)sl];
    const int64_t p0 = B.slice_ptr[sl], w = B.slice_ptr[sl + 1] - p0;
    int64_t off = 0;
    for (int32_t lane = 0; lane < (int32_t)cnt.size(); ++lane) {
      const int32_t i = (int32_t)sl * 64 + lane;
      const int32_t* b0 = cols.data() + off;
      const int32_t* b1 = b0 + cnt[(size_t)lane];
      for (int64_t k = 0; k < w; ++k) B.bcol[(size_t)((p0 + k) * 64 + lane)] = k < cnt[(size_t)lane] ? b0[k] : i;
      for (int a = 0; a < bs; ++a) {
        const int64_t r = (int64_t)i * bs + a;
        for (int64_t k = A.rp[r]; k < A.rp[r + 1]; ++k) {
          const int32_t bc = A.ci[k] / bs, b = A.ci[k] % bs;
          const int64_t kk = std::lower_bound(b0, b1, bc) - b0;
          const int64_t idx = ((p0 + kk) * bs * bs + a * bs + b) * 64 + lane;
          B.val[(size_t)idx] = A.v[k];
          B.pos[(size_t)k] = idx;
        }
      }
      off += cnt[(size_t)lane];
    }
  });
  // 16-bit deltas from each lane's node when the band allows (lanes past the
  // last node keep delta 0 and column 0)
  bool fits = true;
  for (int32_t sl = 0; sl < B.n_slices && fits; ++sl)
    for (int64_t p = B.slice_ptr[sl]; p < B.slice_ptr[sl + 1] && fits; ++p)
      for (int32_t lane = 0; lane < 64; ++lane) {
        const int64_t node = (int64_t)sl * 64 + lane;
        if (node >= B.n_nodes) break;
        const int64_t d = (int64_t)B.bcol[(size_t)(p * 64 + lane)] - node;
        if (d < -32767 || d > 32767) {
          fits = false;
          break;
        }
      }
  if (fits) {
    B.bdel.assign(B.bcol.size(), 0);
    for (int32_t sl = 0; sl < B.n_slices; ++sl)
      for (int64_t p = B.slice_ptr[sl]; p < B.slice_ptr[sl + 1]; ++p)
        for (int32_t lane = 0; lane < 64; ++lane) {
          const int64_t node = (int64_t)sl * 64 + lane;
          if (node < B.n_nodes) B.bdel[(size_t)(p * 64 + lane)] = (int16_t)(B.bcol[(size_t)(p * 64 + lane)] - node);
        }
  }
  return B;
}

// Symmetric storage of a square node-blocked CSR matrix that equals its
// transpose: the blocks on and right of the block diagonal in the sliced
// layout (16-bit deltas), the blocks left of it as (delta, mirror position)
// pairs.  Returns a HostBell with sym = false when a delta or a mirror
// offset does not fit 16 bits or a mirror block is missing.
static HostBell make_bell_sym(const HostCSR& A, int bs) {
  HostBell B;
  B.bs = bs;
  B.n_nodes = (int32_t)(A.nrows / bs);
  B.n_slices = (B.n_nodes + 63) / 64;
  const int nt = setup_threads();
  const int bb = bs * bs;
  // sorted distinct block columns per node, the number left of the diagonal,
  // and each lane's offset into its slice's list
  std::vector<std::vector<int32_t>> sl_cols((size_t)B.n_slices);
  std::vector<std::vector<int32_t>> sl_cnt((size_t)B.n_slices), sl_low((size_t)B.n_slices),
      sl_off((size_t)B.n_slices);
  parallel_chunks(B.n_slices, nt, [&](int64_t sl, int) {
    std::vector<int32_t> tmp;
    auto& cols = sl_cols[(size_t)sl];
    for (int32_t i = (int32_t)sl * 64; i < std::min(B.n_nodes, (int32_t)sl * 64 + 64); ++i) {
      tmp.clear();
      for (int a = 0; a < bs; ++a) {
        const int64_t r = (int64_t)i * bs + a;
        for (int64_t k = A.rp[r]; k < A.rp[r + 1]; ++k) tmp.push_back(A.ci[k] / bs);
      }
      std::sort(tmp.begin(), tmp.end());
      tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
      sl_off[(size_t)sl].push_back((int32_t)cols.size());
      cols.insert(cols.end(), tmp.begin(), tmp.end());
      sl_cnt[(size_t)sl].push_back((int32_t)tmp.size());
      sl_low[(size_t)sl].push_back((int32_t)(std::lower_bound(tmp.begin(), tmp.end(), i) - tmp.begin()));
    }
  });
  B.slice_ptr.assign((size_t)B.n_slices + 1, 0);
  B.lptr.assign((size_t)B.n_slices + 1, 0);
  int64_t nblk = 0, nlow = 0;
  for (int32_t sl = 0; sl < B.n_slices; ++sl) {
    int32_t wu = 0, wl = 0;
    for (size_t ln = 0; ln < sl_cnt[(size_t)sl].size(); ++ln) {
      wu = std::max(wu, sl_cnt[(size_t)sl][ln] - sl_low[(size_t)sl][ln]);
      wl = std::max(wl, sl_low[(size_t)sl][ln]);
      nlow += sl_low[(size_t)sl][ln];
    }
    // at least one stored position: a padded mirror entry reads the lane's
    // first stored block (and multiplies it by 0)
    B.slice_ptr[sl + 1] = B.slice_ptr[sl] + std::max(wu, 1);
    B.lptr[sl + 1] = B.lptr[sl] + wl;
    nblk += (int64_t)sl_cols[(size_t)sl].size();
  }
  B.n_blocks = nblk;
  B.n_lower = nlow;
  const int64_t npos = B.slice_ptr[B.n_slices], nlpos = B.lptr[B.n_slices];
  B.bdel.assign((size_t)(npos * 64), 0);
  B.val.assign((size_t)(npos * 64 * bb), 0.0);
  B.pos.assign((size_t)A.nnz(), -1);
  const int32_t pad_word = (int32_t)((uint32_t)(uint16_t)INT16_MIN << 16);  // no block
  B.lidx.assign((size_t)(nlpos * 64), pad_word);
  std::atomic<bool> ok{true};
  std::atomic<int64_t> stored{0};
  parallel_chunks(B.n_slices, nt, [&](int64_t sl, int) {
    const auto& cols = sl_cols[(size_t)sl];
    const int64_t p0 = B.slice_ptr[sl], q0 = B.lptr[sl];
    int64_t nst = 0;
    for (int32_t lane = 0; lane < (int32_t)sl_cnt[(size_t)sl].size(); ++lane) {
      const int32_t i = (int32_t)sl * 64 + lane;
      const int32_t cnt = sl_cnt[(size_t)sl][(size_t)lane], low = sl_low[(size_t)sl][(size_t)lane];
      const int32_t* b0 = cols.data() + sl_off[(size_t)sl][(size_t)lane];
      for (int32_t k = low; k < cnt; ++k) {
        const int64_t d = (int64_t)b0[k] - i;
        if (d > 32767) ok = false;
        else B.bdel[(size_t)((p0 + k - low) * 64 + lane)] = (int16_t)d;
      }
      for (int a = 0; a < bs; ++a) {
        const int64_t r = (int64_t)i * bs + a;
        for (int64_t k = A.rp[r]; k < A.rp[r + 1]; ++k) {
          const int32_t bc = A.ci[k] / bs, b = A.ci[k] % bs;
          if (bc < i) continue;
          const int64_t kk = std::lower_bound(b0 + low, b0 + cnt, bc) - (b0 + low);
          const int64_t idx = ((p0 + kk) * bb + a * bs + b) * 64 + lane;
          B.val[(size_t)idx] = A.v[k];
          B.pos[(size_t)k] = idx;
          ++nst;
        }
      }
      // blocks left of the diagonal: block (i, c) = block (c, i)^T, stored
      // in node c's upper list
      for (int32_t k = 0; k < low; ++k) {
        const int32_t c = b0[k];
        const int64_t d = (int64_t)c - i;
        const int32_t sc = c / 64, lc = c % 64;
        const int32_t* c0 = sl_cols[(size_t)sc].data() + sl_off[(size_t)sc][(size_t)lc];
        const int32_t clow = sl_low[(size_t)sc][(size_t)lc], ccnt = sl_cnt[(size_t)sc][(size_t)lc];
        const int32_t* hit = std::lower_bound(c0 + clow, c0 + ccnt, i);
        if (d < -32767 || hit == c0 + ccnt || *hit != i) {
          ok = false;
          continue;
        }
        const int64_t rel = (int64_t)B.slice_ptr[sc] + (hit - (c0 + clow)) - p0;
        if (rel < -32767 || rel > 32767) {
          ok = false;
          continue;
        }
        B.lidx[(size_t)((q0 + k) * 64 + lane)] =
            (int32_t)(((uint32_t)(uint16_t)(int16_t)rel << 16) | (uint32_t)(uint16_t)(int16_t)d);
      }
    }
    stored += nst;
  });
  B.nnz_stored = stored;
  B.sym = ok;
  if (!B.sym) return HostBell{};
  return B;
}

struct DevBell {
  int32_t n_nodes = 0, bs = 0, n_slices = 0;
  DBuf<int32_t> slice_ptr, bcol;
  DBuf<int16_t> bdel;  // replaces bcol when the column deltas fit in 16 bits
  DBuf<double> v64;
  DBuf<float> v32;
  DBuf<uint16_t> v16;  // bfloat16 words in place of v32 (fine-level K with CAMG_PREC_MIXED_BF16)
  DBuf<int32_t> lptr, lidx;  // symmetric storage: lower positions
  bool npl = false;          // symmetric storage: node-per-lane kernels
  template <typename T>
  DBELL<T> view() const {
    DBELL<T> d;
    d.n_nodes = n_nodes;
    d.bs = bs;
    d.n_slices = n_slices;
    d.slice_ptr = slice_ptr.p;
    d.bcol = bcol.p;
    d.bdel = bdel.p;
    d.lptr = lptr.p;
    d.lidx = lidx.p;
    if constexpr (sizeof(T) == 8) {
      d.val = reinterpret_cast<const T*>(v64.p);
      d.stream = 1;
    } else {
      d.val = reinterpret_cast<const T*>(v32.p);
      d.val16 = v16.p;
      // more than three quarters of the 256 MB last-level cache: the values
      // cannot stay there between passes, so they stream
      const size_t bytes = v16.p ? v16.n * sizeof(uint16_t) : v32.n * sizeof(float);
      d.stream = bytes > (size_t(192) << 20) ? 1 : 0;
    }
    if (lptr.p) d.stream = npl ? 1 : 0;
    return d;
  }
};

// b16: the reduced copy holds bfloat16 words (FP64 -> FP32 -> bfloat16,
// each to nearest even) instead of FP32 values.
static void upload_bell(DevBell& D, const HostBell& H, bool f64, bool f32, hipStream_t s, bool b16 = false) {
  D.n_nodes = H.n_nodes;
  D.bs = H.bs;
  D.n_slices = H.n_slices;
  D.slice_ptr.upload(H.slice_ptr, s);
  if (!H.bdel.empty()) D.bdel.upload(H.bdel, s);
  else D.bcol.upload(H.bcol, s);
  if (H.sym) {
    D.lptr.upload(H.lptr, s);
    D.lidx.upload(H.lidx, s);
  }
  if (f64) D.v64.upload(H.val, s);
  if (f32 && b16) {
    std::vector<uint16_t> v16(H.val.size());
    parallel_for((int64_t)v16.size(), [&](int64_t i0, int64_t i1) {
      for (int64_t i = i0; i < i1; ++i) {
        const float f = (float)H.val[(size_t)i];
        uint32_t u;
        std::memcpy(&u, &f, sizeof(u));
        const uint32_t lower = u & 0xFFFFu, upper = u >> 16;
        const uint32_t up = (lower > 0x8000u || (lower == 0x8000u && (upper & 1u))) ? 1u : 0u;
        v16[(size_t)i] = (uint16_t)(upper + up);
      }
    });
    D.v16.upload(v16, s);
    CAMG_HIP(hipStreamSynchronize(s));
  } else if (f32) {
    std::vector<float> v32(H.val.size());
    parallel_for((int64_t)v32.size(), [&](int64_t i0, int64_t i1) {
      for (int64_t i = i0; i < i1; ++i) v32[(size_t)i] = (float)H.val[(size_t)i];
    });
    D.v32.upload(v32, s);
    CAMG_HIP(hipStreamSynchronize(s));
  }
  CAMG_HIP(hipStreamSynchronize(s));
}

template <typename T>
struct LevelVecs {
  DBuf<T> b, z, zn, r, delta, aux1, aux2, su;
  DBuf<T> delta2, qrhs;  // Schur sweeps: second delta buffer and right-hand side
  DBuf<T> jinv, ainv, sdinv;
  DBuf<T> sblk;  // block Schur option: inverse nodal blocks of S (bs_l x bs_l, row-major)
  DBuf<T> ablk;  // nodal lumping option: inverse lumping blocks (bs_u x bs_u, row-major)
  DBuf<T> Ainv, AinvT;
};

struct DevLevel {
  int64_t n_u = 0, n_l = 0;
  DevMat K, G, B, C, KT, GT, BT, CT, Pu, Pl, Ru, Rl;
  DevMat S, ST;  // Schur matrix B Atilde^-1 G - C and its transpose (Schur sweeps only)
  int sg_S = 8;
  int sblk_bs = 0;     // > 0: the Schur step relaxes with nodal blocks of this size
  int ablk_bs = 0;     // > 0: nodal lumping blocks of this size (the nodal sweep)
  DBuf<int32_t> g_nodes;  // nodal sweep: nodes with a nonempty G row (the back-substitution's support)
  int32_t n_g_nodes = 0;
  bool bell = false;   // K and K^T in sliced blocked-ELL layout
  // sym: K = K^T and Kb holds it in symmetric storage, which also serves
  // the transposed kernels (KTb stays empty).  sym_stale: level 0 after an
  // update of K's values that are no longer symmetric; its FP64 kernels then
  // use the CSR copies (the FP32 hierarchy keeps the values it was built on).
  bool sym = false, sym_stale = false;
  DevBell Kb, KTb;
  int64_t k_blocks = 0, k_slots = 0, k_lower = 0, k_nnz_stored = 0;
  DBuf<int32_t> g_rows;
  int32_t n_g_rows = 0;
  int sg_K = 16, sg_R = 16, sg_P = 8;
  // transfers with the tentative aggregate pattern stored without column
  // indices (agg_ok); otherwise the CSR P / R above
  bool agg_ok = false;
  int ns_u = 0, ns_l = 0, n_agg_u = 0, n_agg_l = 0;
  DBuf<int32_t> base_u, base_l, aptr_u, arows_u, aptr_l, arows_l;
  DBuf<double> pu64, pl64;
  DBuf<float> pu32, pl32;
  template <typename T>
  AggTransferView<T> agg_view() const;
  LevelVecs<double> v64;
  LevelVecs<float> v32;
  int64_t n() const { return n_u + n_l; }
  // whether the kernels of precision T use the blocked-ELL copies of K
  template <typename T>
  bool bell_for() const {
    return bell && !(sizeof(T) == 8 && sym_stale);
  }
  // blocked-ELL view of K or K^T (the symmetric storage serves both)
  template <typename T>
  DBELL<T> kview(bool trans) const {
    return (trans && !sym ? KTb : Kb).template view<T>();
  }
};

template <>
AggTransferView<double> DevLevel::agg_view<double>() const {
  AggTransferView<double> t;
  t.n_u = (int)n_u, t.n_l = (int)n_l, t.ns_u = ns_u, t.ns_l = ns_l, t.n_agg_u = n_agg_u, t.n_agg_l = n_agg_l;
  t.base_u = base_u.p, t.base_l = base_l.p, t.ptr_u = aptr_u.p, t.rows_u = arows_u.p, t.ptr_l = aptr_l.p;
  t.rows_l = arows_l.p, t.pu = pu64.p, t.pl = pl64.p;
  return t;
}
template <>
AggTransferView<float> DevLevel::agg_view<float>() const {
  AggTransferView<float> t;
  t.n_u = (int)n_u, t.n_l = (int)n_l, t.ns_u = ns_u, t.ns_l = ns_l, t.n_agg_u = n_agg_u, t.n_agg_l = n_agg_l;
  t.base_u = base_u.p, t.base_l = base_l.p, t.ptr_u = aptr_u.p, t.rows_u = arows_u.p, t.ptr_l = aptr_l.p;
  t.rows_l = arows_l.p, t.pu = pu32.p, t.pl = pl32.p;
  return t;
}

// Whether P has the tentative aggregate pattern: every row empty or exactly
// the ns consecutive columns of one aggregate (first column a multiple of
// ns).  Fills the per-row base column (-1 for empty rows), dense per-row
// values and each aggregate's ascending fine-row list.
static bool agg_pattern(const HostCSR& P, int ns, std::vector<int32_t>& base, std::vector<double>& vals,
                        std::vector<int32_t>& aptr, std::vector<int32_t>& arows) {
  if (ns <= 0 || P.ncols % ns) return false;
  const int64_t n = P.nrows, n_agg = P.ncols / ns;
  base.assign((size_t)n, -1);
  vals.assign((size_t)(n * ns), 0.0);
  aptr.assign((size_t)n_agg + 1, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t r0 = P.rp[i], len = P.rp[i + 1] - r0;
    if (len == 0) continue;
    if (len != ns) return false;
    const int32_t c0 = P.ci[r0];
    if (c0 % ns) return false;
    for (int k = 0; k < ns; ++k) {
      if (P.ci[r0 + k] != c0 + k) return false;
      vals[(size_t)(i * ns + k)] = P.v[r0 + k];
    }
    base[(size_t)i] = c0;
    ++aptr[(size_t)(c0 / ns) + 1];
  }
  for (int64_t a = 0; a < n_agg; ++a) aptr[(size_t)a + 1] += aptr[(size_t)a];
  arows.assign((size_t)aptr.back(), 0);
  std::vector<int32_t> fill(aptr.begin(), aptr.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    if (base[(size_t)i] >= 0) arows[(size_t)fill[(size_t)(base[(size_t)i] / ns)]++] = (int32_t)i;
  return true;
}

// ---------------------------------------------------------------------------
// profiling (hipEvents around launches of selected kernel classes)

struct Prof {
  int mask = 0;
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  hipEvent_t get() {
    if (pool_used == pool.size()) {
      hipEvent_t e;
      // timing only: skip the system-scope release fence, whose cache
      // write-back would otherwise land inside the bracketed interval
      CAMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
      pool.push_back(e);
    }
    return pool[pool_used++];
  }
  ~Prof() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

struct ProfScope {
  Prof* p;
  int cls;
  hipStream_t s;
  hipEvent_t a = nullptr;
  ProfScope(Prof* prof, int c, hipStream_t st) : p(prof), cls(c), s(st) {
    if (p && (p->mask & cls)) {
      a = p->get();
      CAMG_HIP(hipEventRecord(a, s));
    }
  }
  ~ProfScope() noexcept(false) {
    if (a) {
      hipEvent_t b = p->get();
      CAMG_HIP(hipEventRecord(b, s));
      p->recs.push_back({cls, a, b});
    }
  }
};

}  // namespace camg

using namespace camg;

// Work memory of amg_vcycle_apply_noalloc: the V-cycle vectors of every level
// (right-hand side, iterates, residual, multiplier increments, prediction
// buffers) for callers that cannot allocate.  Each GPU that runs the library
// holds one copy until the process ends; host code reaches it only through
// the per-device address from hipGetSymbolAddress, never through this name.
static constexpr size_t kNoallocScratchBytes = CAMG_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace camg {

static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be current; looked up
// once per device.
static void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) api_fail(CAMG_ERR_INVALID_ARG, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    CAMG_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) api_fail(CAMG_ERR_HIP, "no device address for the no-allocation scratch array");
    g_scratch_addr[device] = p;
  }
  return g_scratch_addr[device];
}

}  // namespace camg

struct amg_handle {
  int device = 0;
  amg_options opts{};
  int dim = 0;
  std::vector<HostLevel> host;
  std::vector<DevLevel> lev;
  std::vector<int32_t> perm_K, perm_G, perm_B, perm_C;
  DBuf<int32_t> d_perm_K, d_perm_G, d_perm_B, d_perm_C;
  DBuf<int64_t> d_bpos_K, d_bpos_KT;  // level-0 K entry -> BELL slot of K / K^T (-1: not stored)
  DBuf<int32_t> d_asym;               // symmetric storage: flag set by the symmetry check of an update
  int64_t n = 0, n_u = 0, n_l = 0;
  // Krylov workspace
  int m_alloc = 0;
  DBuf<double> V, Z, w, r, H, cs, sn, g, h1, h2, hn2, partial, out, y;
  DBuf<double> Gram, gn, cc;  // two-pass CGS2: Gram matrix of the basis, next Gram column, update coefficients
  double* hbuf = nullptr;  // pinned host: [0,4) synchronous reads, then 4 doubles per pipelined slot
  double* hbuf_dev = nullptr;  // the same memory as a device address (kernels write the slots)
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  static constexpr int kSlots = 8;
  hipEvent_t evq[kSlots] = {};
  // V-cycle captured once per direction and replayed (graphs option)
  hipStream_t cap_stream = nullptr;
  hipGraph_t vgraph[2] = {nullptr, nullptr};
  hipGraphExec_t vexec[2] = {nullptr, nullptr};
  void* vout[2] = {nullptr, nullptr};
  Prof prof;
  void* scratch = nullptr;  // this device's no-allocation scratch array (device address)
  ~amg_handle() {
    for (int t = 0; t < 2; ++t) {
      if (vexec[t]) (void)hipGraphExecDestroy(vexec[t]);
      if (vgraph[t]) (void)hipGraphDestroy(vgraph[t]);
    }
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    for (auto e : evq)
      if (e) (void)hipEventDestroy(e);
    if (hbuf) (void)hipHostFree(hbuf);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }
};

namespace camg {

static hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Validates a caller's CSR block: the row pointers first, then the entries
// of the rows in parallel chunks, reporting the error of the first
// offending row (whichever chunk finds its own first).
static void check_csr(const amg_csr& A, int64_t nrows, int64_t ncols, const char* name) {
  const std::string nm(name);
  if (A.nrows != nrows || A.ncols != ncols) api_fail(CAMG_ERR_SHAPE, nm + ": wrong dimensions");
  if (A.nnz < 0 || A.nnz >= (int64_t(1) << 31)) api_fail(CAMG_ERR_SHAPE, nm + ": nnz out of range");
  if (nrows > 0 && !A.rowptr) api_fail(CAMG_ERR_INVALID_ARG, nm + ": rowptr is NULL");
  if (A.nnz > 0 && (!A.col || !A.val)) api_fail(CAMG_ERR_INVALID_ARG, nm + ": col/val is NULL");
  if (nrows == 0) return;
  if (A.rowptr[0] != 0 || A.rowptr[nrows] != A.nnz) api_fail(CAMG_ERR_SHAPE, nm + ": rowptr ends do not match nnz");
  // row pointers first (serially cheap), so the entry scan below stays in range
  for (int64_t i = 0; i < nrows; ++i)
    if (A.rowptr[i + 1] < A.rowptr[i] || A.rowptr[i + 1] > A.nnz)
      api_fail(CAMG_ERR_SHAPE, nm + ": rowptr not monotone");
  constexpr int64_t kGrain = 1 << 14;
  const int64_t n_chunks = (nrows + kGrain - 1) / kGrain;
  struct Bad {
    int64_t row = -1;
    int code = 0;
    const char* what = nullptr;
  };
  std::vector<Bad> bad((size_t)n_chunks);
  parallel_chunks(n_chunks, setup_threads(), [&](int64_t c, int) {
    const int64_t r1 = std::min(nrows, (c + 1) * kGrain);
    for (int64_t i = c * kGrain; i < r1; ++i)
      for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
        if (A.col[k] < 0 || A.col[k] >= ncols) {
          bad[(size_t)c] = {i, CAMG_ERR_SHAPE, ": column index out of range"};
          return;
        }
        if (k > A.rowptr[i] && A.col[k] <= A.col[k - 1]) {
          bad[(size_t)c] = {i, CAMG_ERR_SHAPE, ": columns not sorted/unique"};
          return;
        }
        if (!std::isfinite(A.val[k])) {
          bad[(size_t)c] = {i, CAMG_ERR_NONFINITE, ": non-finite value"};
          return;
        }
      }
  });
  for (const Bad& b : bad)
    if (b.row >= 0) api_fail(b.code, nm + b.what);
}

static HostCSR to_host(const amg_csr& A) {
  HostCSR H;
  H.nrows = A.nrows;
  H.ncols = A.ncols;
  H.rp.assign(A.rowptr, A.rowptr + A.nrows + 1);
  if (A.nnz) {
    H.ci.resize((size_t)A.nnz);
    H.v.resize((size_t)A.nnz);
    parallel_for(A.nnz, [&](int64_t k0, int64_t k1) {
      std::memcpy(H.ci.data() + k0, A.col + k0, (size_t)(k1 - k0) * sizeof(int32_t));
      std::memcpy(H.v.data() + k0, A.val + k0, (size_t)(k1 - k0) * sizeof(double));
    }, int64_t(1) << 22);
  }
  return H;
}

// dense_coarse: the level is the coarsest one and is solved with its dense
// inverse (otherwise it smooths and needs the smoother diagonals).
template <typename T>
static void alloc_vecs(LevelVecs<T>& V, const HostLevel& H, bool dense_coarse, hipStream_t s) {
  const int64_t n = H.n(), nu = H.n_u(), nl = H.n_l();
  for (DBuf<T>* b : {&V.b, &V.z, &V.zn, &V.r}) {
    b->alloc((size_t)n);
    zero_vec<T>(b->p, n, s);
  }
  for (DBuf<T>* b : {&V.delta, &V.delta2, &V.qrhs}) {
    b->alloc((size_t)std::max<int64_t>(nl, 1));
    zero_vec<T>(b->p, std::max<int64_t>(nl, 1), s);
  }
  for (DBuf<T>* b : {&V.aux1, &V.aux2, &V.su}) {
    b->alloc((size_t)std::max<int64_t>(nu, 1));
    zero_vec<T>(b->p, std::max<int64_t>(nu, 1), s);
  }
  auto up = [&](DBuf<T>& d, const std::vector<double>& h) {
    std::vector<T> t(h.begin(), h.end());
    d.upload(t, s);
    CAMG_HIP(hipStreamSynchronize(s));
  };
  if (!dense_coarse) {
    up(V.jinv, H.jac_inv);
    up(V.ainv, H.atilde_inv);
    up(V.sdinv, H.sd_inv);
    if (!H.sblk_inv.empty()) up(V.sblk, H.sblk_inv);
    if (!H.ablk_inv.empty()) up(V.ablk, H.ablk_inv);
  } else if (!H.Ainv.empty()) {
    up(V.Ainv, H.Ainv);
    std::vector<double> t(H.Ainv.size());
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < n; ++j) t[(size_t)(j * n + i)] = H.Ainv[(size_t)(i * n + j)];
    up(V.AinvT, t);
  } else {
    // LU of the merged matrix on the device (FP64), the inverse and its
    // transpose rounded to T
    DBuf<double> a;
    a.upload(H.Adense, s);
    V.Ainv.alloc((size_t)(n * n));
    V.AinvT.alloc((size_t)(n * n));
    if (!dense_inverse<T>(a.p, n, 1e-13 * H.Adense_amax, V.Ainv.p, V.AinvT.p, s))
      throw SetupError{CAMG_ERR_SINGULAR_COARSE, "coarsest merged matrix is singular"};
  }
}

static void upload_hierarchy(amg_handle& h, hipStream_t s) {
  const bool mixed = h.opts.precision != CAMG_PREC_FP64;
  const size_t L = h.host.size();
  h.lev.resize(L);
  for (size_t l = 0; l < L; ++l) {
    HostLevel& H = h.host[l];
    DevLevel& D = h.lev[l];
    const bool coarsest = (l + 1 == L);
    const bool f64 = !mixed || l == 0;  // level 0 in FP64 always (outer operator)
    const bool f32 = mixed;
    D.n_u = H.n_u();
    D.n_l = H.n_l();
    PhaseTimer pt_level(l == 0 ? "upload level 0" : "upload coarse level");
    upload_mat(D.K, H.K, f64, f32, s);
    upload_mat(D.G, H.G, f64, f32, s);
    upload_mat(D.B, H.B, f64, f32, s);
    upload_mat(D.C, H.C, f64, f32, s);
    std::vector<int32_t>* perms[4] = {nullptr, nullptr, nullptr, nullptr};
    if (l == 0) perms[0] = &h.perm_K, perms[1] = &h.perm_G, perms[2] = &h.perm_B, perms[3] = &h.perm_C;
    const HostCSR KT = transpose(H.K, perms[0]);
    upload_mat(D.KT, KT, f64, f32, s);
    upload_mat(D.GT, transpose(H.G, perms[1]), f64, f32, s);
    upload_mat(D.BT, transpose(H.B, perms[2]), f64, f32, s);
    upload_mat(D.CT, transpose(H.C, perms[3]), f64, f32, s);
    D.sg_K = pick_subgroup(H.K.nnz(), H.K.nrows);
    {
      const int64_t nodes = H.n_u() / H.bs_u;
      const int64_t slices = (nodes + 63) / 64;
      const int fmt = h.opts.spmv_format & ~CAMG_SPMV_FULL;
      const bool full = (h.opts.spmv_format & CAMG_SPMV_FULL) != 0;
      D.bell = (fmt == CAMG_SPMV_BELL) || (fmt == CAMG_SPMV_AUTO && slices >= 512);
      if (D.bell && H.bs_u > 0 && H.n_u() % H.bs_u == 0) {
        const bool b16 = l == 0 && h.opts.precision == CAMG_PREC_MIXED_BF16;
        HostBell hb;
        if (!full && csr_symmetric(H.K, KT)) hb = make_bell_sym(H.K, H.bs_u);
        D.sym = hb.sym;
        if (D.sym) {
          if (l == 0) {
            h.d_bpos_K.upload(hb.pos, s);
            h.d_asym.alloc(1);
            CAMG_HIP(hipStreamSynchronize(s));
          }
          upload_bell(D.Kb, hb, f64, f32, s, b16);
          // one wave per slice: only levels with enough slices to fill the
          // chip (8192: 32 waves on each of the 256 compute units), or any
          // level when the blocked-ELL layout is forced
          D.Kb.npl = fmt == CAMG_SPMV_BELL || hb.n_slices >= 8192;
          D.k_lower = hb.n_lower;
          D.k_nnz_stored = hb.nnz_stored;
        } else {
          hb = make_bell(H.K, H.bs_u);
          HostBell hbt = make_bell(KT, H.bs_u);
          if (l == 0) {
            std::vector<int64_t> posT((size_t)H.K.nnz());
            parallel_for(H.K.nnz(), [&](int64_t k0, int64_t k1) {
              for (int64_t k = k0; k < k1; ++k) posT[(size_t)k] = hbt.pos[(size_t)h.perm_K[(size_t)k]];
            });
            h.d_bpos_K.upload(hb.pos, s);
            h.d_bpos_KT.upload(posT, s);
            CAMG_HIP(hipStreamSynchronize(s));
          }
          upload_bell(D.Kb, hb, f64, f32, s, b16);
          upload_bell(D.KTb, hbt, f64, f32, s, b16);
          D.k_nnz_stored = H.K.nnz();
        }
        D.k_blocks = hb.n_blocks;
        D.k_slots = (int64_t)hb.slice_ptr.back() * 64;
      } else {
        D.bell = false;
      }
    }
    // coarse levels: node-blocked copies of K and K^T for the row dots
    if (!D.bell && l > 0 && (h.opts.spmv_format & ~CAMG_SPMV_FULL) == CAMG_SPMV_AUTO &&
        !(coarsest && h.opts.coarse_solver == CAMG_COARSE_LU)) {
      upload_rowblock(D.K, H.K, H.bs_u, f64, f32, s);
      upload_rowblock(D.KT, KT, H.bs_u, f64, f32, s);
    }
    if (!coarsest) {
      const bool t64 = !mixed;
      upload_mat(D.Pu, H.P_u, t64, f32, s);
      upload_mat(D.Pl, H.P_l, t64, f32, s);
      HostCSR Ru = transpose(H.P_u), Rl = transpose(H.P_l);
      upload_mat(D.Ru, Ru, t64, f32, s);
      upload_mat(D.Rl, Rl, t64, f32, s);
      D.sg_R = pick_subgroup(Ru.nnz(), Ru.nrows);
      D.sg_P = pick_subgroup(H.P_u.nnz(), H.P_u.nrows);
      std::vector<int32_t> bu, bl, pu_, ru_, pl_, rl_;
      std::vector<double> vu, vl;
      D.agg_ok = agg_pattern(H.P_u, H.n_ns_u, bu, vu, pu_, ru_) && agg_pattern(H.P_l, H.n_ns_l, bl, vl, pl_, rl_) &&
                 ((H.n_ns_u == 6 && H.n_ns_l == 3) || (H.n_ns_u == 3 && H.n_ns_l == 2));
      if (D.agg_ok) {
        D.ns_u = H.n_ns_u, D.ns_l = H.n_ns_l;
        D.n_agg_u = (int)(pu_.size() - 1), D.n_agg_l = (int)(pl_.size() - 1);
        D.base_u.upload(bu, s);
        D.base_l.upload(bl, s);
        D.aptr_u.upload(pu_, s);
        D.arows_u.upload(ru_, s);
        D.aptr_l.upload(pl_, s);
        D.arows_l.upload(rl_, s);
        if (t64) {
          D.pu64.upload(vu, s);
          D.pl64.upload(vl, s);
        } else {
          std::vector<float> fu(vu.begin(), vu.end()), fl(vl.begin(), vl.end());
          D.pu32.upload(fu, s);
          D.pl32.upload(fl, s);
        }
        CAMG_HIP(hipStreamSynchronize(s));
      }
    }
    const bool dense_coarse = coarsest && h.opts.coarse_solver == CAMG_COARSE_LU;
    if (!dense_coarse) {
      const bool t64 = !mixed;
      if (H.S.nrows > 0) {
        upload_mat(D.S, H.S, t64, f32, s);
        upload_mat(D.ST, transpose(H.S), t64, f32, s);
        D.sg_S = pick_subgroup(H.S.nnz(), H.S.nrows);
      }
      std::vector<int32_t> gr;
      for (int64_t i = 0; i < H.G.nrows; ++i)
        if (H.G.rp[i + 1] > H.G.rp[i]) gr.push_back((int32_t)i);
      D.n_g_rows = (int32_t)gr.size();
      D.g_rows.upload(gr, s);
    }
    D.sblk_bs = (!dense_coarse && !H.sblk_inv.empty()) ? H.bs_l : 0;
    D.ablk_bs = (!dense_coarse && !H.ablk_inv.empty()) ? H.bs_u : 0;
    if (D.ablk_bs > 0) {
      std::vector<int32_t> gn;
      for (int64_t nd = 0; nd < H.n_u() / H.bs_u; ++nd) {
        bool any = false;
        for (int b = 0; b < H.bs_u; ++b) {
          const int64_t i = nd * H.bs_u + b;
          any = any || H.G.rp[i + 1] > H.G.rp[i];
        }
        if (any) gn.push_back((int32_t)nd);
      }
      D.n_g_nodes = (int32_t)gn.size();
      D.g_nodes.upload(gn, s);
    }
    if (mixed) alloc_vecs<float>(D.v32, H, dense_coarse, s);
    else alloc_vecs<double>(D.v64, H, dense_coarse, s);
    if (mixed && l == 0) {
      // FP64 level-0 vectors for operator applies outside the V-cycle
      D.v64.r.alloc((size_t)H.n());
    }
  }
  h.d_perm_K.upload(h.perm_K, s);
  h.d_perm_G.upload(h.perm_G, s);
  h.d_perm_B.upload(h.perm_B, s);
  h.d_perm_C.upload(h.perm_C, s);
  CAMG_HIP(hipStreamSynchronize(s));
}

// ---------------------------------------------------------------------------
// V-cycle

template <typename T>
static LevelVecs<T>& vecs(DevLevel& D);
template <>
LevelVecs<double>& vecs<double>(DevLevel& D) {
  return D.v64;
}
template <>
LevelVecs<float>& vecs<float>(DevLevel& D) {
  return D.v32;
}

// One sweep with the nodal lumping blocks M = Atilde^-1 (the option that
// makes the smoothers covariant under rotations of the node frames).
// Forward (SIMPLE; Uzawa and Braess-Sarazin as in sweep):
//   t = b_u - K z_u - G z_l,  w = J(t) (block Jacobi with M),
//   q = -(b_l - B (z_u + w) - C z_l),  delta = S-relaxation(q),
//   zn_l = z_l + alpha delta,  zn_u = z_u + w - alpha M G delta.
// Adjoint: s_u = b_u - K^T z_u - B^T z_l, q = -(b_l - G^T (z_u + M^T s_u) -
// C^T z_l), delta from S^T, zn_u = z_u + J^T(s_u - alpha B^T delta) with M^T.
// On the level-0 blocked-ELL layout the residual and the block prediction
// are one kernel; the back-substitution runs on the interface nodes only;
// elsewhere the steps are separate products and block applies.  From z = 0
// (first) the forward sweep starts from t = b_u and the adjoint one clears
// the multiplier part of its input buffer (the V-cycle's own work buffer).
template <typename T>
static void sweep_nodal(amg_handle& h, int l, bool transpose, const T* b, const T* z, T* zn, bool first,
                        hipStream_t s) {
  DevLevel& D = h.lev[l];
  LevelVecs<T>& V = vecs<T>(D);
  const int nu = (int)D.n_u, nl = (int)D.n_l, bs = D.ablk_bs;
  const bool uzawa = h.opts.smoother == CAMG_SMOOTHER_UZAWA;
  const bool bsz = h.opts.smoother == CAMG_SMOOTHER_BRAESS_SARAZIN;
  const T om = bsz ? T(1) : (T)h.opts.jacobi_omega;
  const T al = bsz ? T(1) : (T)h.opts.simple_alpha;
  const int nj = bsz ? 1 : std::max(1, h.opts.jacobi_sweeps);
  const int ks = D.S.nrows > 0 ? std::max(1, h.opts.schur_sweeps) - 1 : 0;  // Jacobi sweeps on S after the first
  const bool sblock = D.sblk_bs > 0;
  T* q = V.qrhs.p;
  const T* sdv = sblock ? nullptr : V.sdinv.p;
  const T* bu = b;
  const T* bl = b + nu;
  const T* zu = z;
  const T* zl = z + nu;
  T* znu = zn;
  T* znl = zn + nu;
  const T* M = V.ablk.p;
  DCSR<T> none;
  // delta from q = -(r_l - B w): the multiplier kernel already divided by the
  // diagonal (point options) or only stored q (nodal Schur blocks)
  auto schur = [&](const DevMat& SM, const T* zl_in, bool trans) -> const T* {
    if (sblock)
      return schur_block_steps<T>(SM.view<T>(), q, V.delta.p, V.delta2.p, V.sblk.p, trans, zl_in, al, znl, ks + 1,
                                  nl, D.sblk_bs, s);
    return schur_steps<T>(SM.view<T>(), q, V.delta.p, V.delta2.p, V.sdinv.p, zl_in, al, znl, ks, nl, D.sg_S, s);
  };
  T* wa = V.aux2.p;
  T* wb = V.su.p;
  T* tr = V.r.p;  // r is free during a sweep
  if (!transpose) {
    // prediction: t = b_u - K z_u - G z_l (t = b_u from zero), w = J(t), zn_u = z_u + w
    const T* t = bu;
    bool zn_done = false;
    if (!first && D.bell_for<T>()) {
      smooth_u_bell_nodal<T>(D.kview<T>(false), D.G.view<T>(), zu, zl, bu, M, om, znu, nj > 1 ? V.aux1.p : nullptr, wa,
                             nu, s);
      t = V.aux1.p;
      zn_done = nj == 1;
    } else {
      if (!first) {
        blk_spmv<T>(D.K.view<T>(), D.G.view<T>(), none, none, zu, zl, bu, nullptr, V.aux1.p, nullptr, nu, 0, 1,
                    D.sg_K, s);
        t = V.aux1.p;
      }
      node_apply<T>(M, t, om, nullptr, nullptr, wa, nu, bs, false, s);
    }
    for (int k = 1; k < nj; ++k) {
      if (D.bell_for<T>())
        blk_spmv_bell<T>(D.kview<T>(false), none, none, none, wa, nullptr, t, nullptr, tr, nullptr, nu, 0, 1, s);
      else
        blk_spmv<T>(D.K.view<T>(), none, none, none, wa, nullptr, t, nullptr, tr, nullptr, nu, 0, 1, D.sg_K, s);
      node_apply<T>(M, tr, om, wa, wb, nullptr, nu, bs, false, s);
      std::swap(wa, wb);
    }
    if (!zn_done) uzawa_update<T>(first ? nullptr : zu, wa, T(1), znu, nu, s);
    smooth_l<T>(D.B.view<T>(), D.C.view<T>(), znu, zl, bl, sdv, al, znl, V.delta.p, q, nl, first, s);
    const T* dfin = schur(D.S, first ? nullptr : zl, false);
    if (uzawa)
      uzawa_update<T>(first ? nullptr : zu, wa, al, znu, nu, s);
    else  // back-substitution on the interface nodes: zn_u -= alpha M G delta
      node_correct<T>(D.G.view<T>(), D.g_nodes.p, D.n_g_nodes, dfin, M, -al, znu, bs, s);
  } else {
    // from zero only the multiplier part of z is read (cleared here)
    if (first) zero_vec<T>(const_cast<T*>(zl), nl, s);
    const T* su = bu;
    if (!first) {
      if (D.bell_for<T>())
        tsmooth_u_bell<T>(D.kview<T>(true), D.BT.view<T>(), zu, zl, bu, V.aux1.p, nu, s);
      else
        tsmooth_u<T>(D.KT.view<T>(), D.BT.view<T>(), zu, zl, bu, V.aux1.p, nu, false, D.sg_K, s);
      su = V.aux1.p;
    }
    // q = -(s_l - G^T M^T s_u) = -(b_l - G^T (z_u + M^T s_u) - C^T z_l); G^T reads
    // its argument only on the interface nodes
    const T* y = first ? nullptr : zu;
    if (!uzawa) {
      node_apply<T>(M, su, T(1), first ? nullptr : zu, tr, nullptr, nu, bs, true, s, D.g_nodes.p, D.n_g_nodes);
      y = tr;
    }
    tsmooth_l<T>(D.GT.view<T>(), D.CT.view<T>(), y, zl, bl, su, nullptr, sdv, al, znl, V.delta.p, q, nl, y == nullptr,
                 s);
    const T* dfin = schur(D.ST, zl, true);
    // zn_u = z_u + c J^T(s_u - a B^T delta) with M^T
    const T a_bt = uzawa ? T(1) : al;
    const T c_w = uzawa ? al : T(1);
    T* t = V.r.p;
    tcorrect_nodal<T>(D.BT.view<T>(), su, dfin, M, om, a_bt, c_w, first ? nullptr : zu, znu, nj > 1 ? t : nullptr,
                      nj > 1 ? wa : nullptr, nu, bs, s);
    if (nj > 1) {
      T* tk = V.aux1.p == su ? V.su.p : V.aux1.p;  // s_u is no longer needed
      wb = (tk == V.su.p) ? V.aux1.p : V.su.p;
      for (int k = 1; k < nj; ++k) {
        if (D.bell_for<T>())
          blk_spmv_bell<T>(D.kview<T>(true), none, none, none, wa, nullptr, t, nullptr, tk, nullptr, nu, 0, 1, s);
        else
          blk_spmv<T>(D.KT.view<T>(), none, none, none, wa, nullptr, t, nullptr, tk, nullptr, nu, 0, 1, D.sg_K, s);
        node_apply<T>(M, tk, om, wa, wb, nullptr, nu, bs, true, s);
        std::swap(wa, wb);
      }
      uzawa_update<T>(first ? nullptr : zu, wa, c_w, znu, nu, s);
    }
  }
}

template <typename T>
static void sweep(amg_handle& h, int l, bool transpose, const T* b, const T* z, T* zn, bool first, hipStream_t s) {
  DevLevel& D = h.lev[l];
  if (D.ablk_bs > 0) {
    sweep_nodal<T>(h, l, transpose, b, z, zn, first, s);
    return;
  }
  LevelVecs<T>& V = vecs<T>(D);
  const int nu = (int)D.n_u, nl = (int)D.n_l;
  // Braess-Sarazin runs the CheapSIMPLE kernels on its scaled lumping with
  // unit dampings and one Jacobi step (the setup folded its damping in);
  // Uzawa keeps the prediction w for its damped displacement update and
  // skips the back-substitution
  const bool uzawa = h.opts.smoother == CAMG_SMOOTHER_UZAWA;
  const bool bsz = h.opts.smoother == CAMG_SMOOTHER_BRAESS_SARAZIN;
  const T om = bsz ? T(1) : (T)h.opts.jacobi_omega;
  const T al = bsz ? T(1) : (T)h.opts.simple_alpha;
  const int nj = bsz ? 1 : std::max(1, h.opts.jacobi_sweeps);
  const bool keep_w = nj > 1 || uzawa;
  const int ks = D.S.nrows > 0 ? std::max(1, h.opts.schur_sweeps) - 1 : 0;  // Jacobi sweeps on S after the first
  // block option: the multiplier kernels only write the right-hand side
  // q = -(r_l - B w) and the nodal block steps form delta and zn_l
  const bool sblock = D.sblk_bs > 0;
  T* q = (ks || sblock) ? V.qrhs.p : nullptr;
  const T* sdv = sblock ? nullptr : V.sdinv.p;
  auto schur = [&](const DevMat& SM, const T* zl_in, bool trans) -> const T* {
    if (sblock)
      return schur_block_steps<T>(SM.view<T>(), q, V.delta.p, V.delta2.p, V.sblk.p, trans, zl_in, al, zn + nu, ks + 1,
                                  nl, D.sblk_bs, s);
    return schur_steps<T>(SM.view<T>(), q, V.delta.p, V.delta2.p, V.sdinv.p, zl_in, al, zn + nu, ks, nl, D.sg_S, s);
  };
  const T* bu = b;
  const T* bl = b + nu;
  const T* zu = z;
  const T* zl = z + nu;
  T* znu = zn;
  T* znl = zn + nu;
  Prof* pp = (l == 0) ? &h.prof : nullptr;
  if (!transpose && first && nj == 1) {
    smooth_first_l<T>(D.B.view<T>(), bu, bl, V.jinv.p, sdv, om, al, znl, V.delta.p, q, nl, s);
    const T* dfin = schur(D.S, nullptr, false);
    if (uzawa)  // zn_u = alpha * omega * jinv .* b_u: no back-substitution
      smooth_first_u<T>(DCSR<T>{}, bu, V.jinv.p, V.ainv.p, dfin, al * om, al, znu, nu, s);
    else
      smooth_first_u<T>(D.G.view<T>(), bu, V.jinv.p, V.ainv.p, dfin, om, al, znu, nu, s);
    return;
  }
  if (!transpose) {
    {
      ProfScope ps(first ? nullptr : pp, CAMG_KCLASS_SMOOTH_U, s);
      if (D.bell_for<T>() && !first)
        smooth_u_bell<T>(D.kview<T>(false), D.G.view<T>(), zu, zl, bu, V.jinv.p, om, znu, keep_w ? V.aux1.p : nullptr,
                         keep_w ? V.aux2.p : nullptr, nu, s);
      else
        smooth_u<T>(D.K.view<T>(), D.G.view<T>(), zu, zl, bu, V.jinv.p, om, znu, keep_w ? V.aux1.p : nullptr,
                    keep_w ? V.aux2.p : nullptr, nu, first, D.sg_K, s);
    }
    T* wa = V.aux2.p;
    T* wb = V.su.p;
    for (int k = 1; k < nj; ++k) {
      if (D.bell_for<T>())
        jacobi_extra_bell<T>(D.kview<T>(false), wa, V.aux1.p, V.jinv.p, om, wb, first ? nullptr : zu, znu, k == nj - 1,
                             nu, s);
      else
        jacobi_extra<T>(D.K.view<T>(), wa, V.aux1.p, V.jinv.p, om, wb, first ? nullptr : zu, znu, k == nj - 1, nu,
                        D.sg_K, s);
      std::swap(wa, wb);
    }
    smooth_l<T>(D.B.view<T>(), D.C.view<T>(), znu, zl, bl, sdv, al, znl, V.delta.p, q, nl, first, s);
    const T* dfin = schur(D.S, first ? nullptr : zl, false);
    if (uzawa)
      uzawa_update<T>(first ? nullptr : zu, wa, al, znu, nu, s);
    else
      correct_u<T>(D.G.view<T>(), D.g_rows.p, D.n_g_rows, dfin, V.ainv.p, al, znu, s);
  } else {
    // from z = 0 the adjoint residual is b itself: no first kernel
    const T* su = first ? bu : V.su.p;
    if (!first) {
      ProfScope ps(pp, CAMG_KCLASS_SMOOTH_U, s);
      if (D.bell_for<T>())
        tsmooth_u_bell<T>(D.kview<T>(true), D.BT.view<T>(), zu, zl, bu, V.su.p, nu, s);
      else
        tsmooth_u<T>(D.KT.view<T>(), D.BT.view<T>(), zu, zl, bu, V.su.p, nu, false, D.sg_K, s);
    }
    tsmooth_l<T>(D.GT.view<T>(), D.CT.view<T>(), zu, zl, bl, su, uzawa ? nullptr : V.ainv.p, sdv, al, znl,
                 V.delta.p, q, nl, first, s);
    const T* dfin = schur(D.ST, first ? nullptr : zl, true);
    tcorrect_u<T>(D.BT.view<T>(), su, dfin, V.jinv.p, om, uzawa ? T(1) : al, zu, znu, keep_w ? V.aux1.p : nullptr,
                  keep_w ? V.aux2.p : nullptr, nu, first, s);
    T* wa = V.aux2.p;
    T* wb = V.r.p;  // r is free during a sweep
    for (int k = 1; k < nj; ++k) {
      if (D.bell_for<T>())
        jacobi_extra_bell<T>(D.kview<T>(true), wa, V.aux1.p, V.jinv.p, om, wb, first ? nullptr : zu, znu,
                             k == nj - 1, nu, s);
      else
        jacobi_extra<T>(D.KT.view<T>(), wa, V.aux1.p, V.jinv.p, om, wb, first ? nullptr : zu, znu, k == nj - 1, nu,
                        D.sg_K, s);
      std::swap(wa, wb);
    }
    if (uzawa) uzawa_update<T>(first ? nullptr : zu, wa, al, znu, nu, s);
  }
}

// Runs the cycle from level l on vecs(l).b; returns the buffer holding z.
template <typename T>
static T* vcycle_level(amg_handle& h, int l, bool transpose, hipStream_t s) {
  DevLevel& D = h.lev[l];
  LevelVecs<T>& V = vecs<T>(D);
  const int nu = (int)D.n_u, nl = (int)D.n_l;
  const int last = (int)h.lev.size() - 1;
  if (l == last && h.opts.coarse_solver == CAMG_COARSE_LU) {
    dense_gemv<T>(transpose ? V.AinvT.p : V.Ainv.p, V.b.p, V.z.p, (int)D.n(), s);
    return V.z.p;
  }
  if (l == last) {
    // CheapSIMPLE coarse solver: coarse_sweeps sweeps from zero (adjoint
    // sweeps for the transposed cycle)
    T* zc = V.z.p;
    T* zx = V.zn.p;
    for (int k = 0; k < h.opts.coarse_sweeps; ++k) {
      sweep<T>(h, l, transpose, V.b.p, zc, zx, k == 0, s);
      std::swap(zc, zx);
    }
    return zc;
  }
  const int npre = transpose ? h.opts.nu_post : h.opts.nu_pre;
  const int npost = transpose ? h.opts.nu_pre : h.opts.nu_post;
  T* zc = V.z.p;
  T* zx = V.zn.p;
  bool first = true;
  for (int k = 0; k < npre; ++k) {
    sweep<T>(h, l, transpose, V.b.p, zc, zx, first, s);
    std::swap(zc, zx);
    first = false;
  }
  if (first) zero_vec<T>(zc, D.n(), s);
  {
    ProfScope ps(l == 0 ? &h.prof : nullptr, CAMG_KCLASS_RESIDUAL, s);
    if (D.bell_for<T>()) {
      if (!transpose)
        blk_spmv_bell<T>(D.kview<T>(false), D.G.view<T>(), D.B.view<T>(), D.C.view<T>(), zc, zc + nu, V.b.p, V.b.p + nu,
                         V.r.p, V.r.p + nu, nu, nl, 1, s);
      else
        blk_spmv_bell<T>(D.kview<T>(true), D.BT.view<T>(), D.GT.view<T>(), D.CT.view<T>(), zc, zc + nu, V.b.p,
                         V.b.p + nu, V.r.p, V.r.p + nu, nu, nl, 1, s);
    } else if (!transpose)
      blk_spmv<T>(D.K.view<T>(), D.G.view<T>(), D.B.view<T>(), D.C.view<T>(), zc, zc + nu, V.b.p, V.b.p + nu, V.r.p,
                  V.r.p + nu, nu, nl, 1, D.sg_K, s);
    else
      blk_spmv<T>(D.KT.view<T>(), D.BT.view<T>(), D.GT.view<T>(), D.CT.view<T>(), zc, zc + nu, V.b.p, V.b.p + nu,
                  V.r.p, V.r.p + nu, nu, nl, 1, D.sg_K, s);
  }
  DevLevel& Dc = h.lev[l + 1];
  LevelVecs<T>& Vc = vecs<T>(Dc);
  const int ncu = (int)Dc.n_u, ncl = (int)Dc.n_l;
  DCSR<T> none;
  if (!(D.agg_ok && agg_transfer<T>(D.agg_view<T>(), true, V.r.p, V.r.p + nu, Vc.b.p, Vc.b.p + ncu, s)))
    blk_spmv<T>(D.Ru.view<T>(), none, none, D.Rl.view<T>(), V.r.p, V.r.p + nu, nullptr, nullptr, Vc.b.p,
                Vc.b.p + ncu, ncu, ncl, 0, D.sg_R, s);
  T* zcoarse = vcycle_level<T>(h, l + 1, transpose, s);
  if (!(D.agg_ok && agg_transfer<T>(D.agg_view<T>(), false, zcoarse, zcoarse + ncu, zc, zc + nu, s)))
    blk_spmv<T>(D.Pu.view<T>(), none, none, D.Pl.view<T>(), zcoarse, zcoarse + ncu, nullptr, nullptr, zc, zc + nu,
                nu, nl, 2, D.sg_P, s);
  for (int k = 0; k < npost; ++k) {
    sweep<T>(h, l, transpose, V.b.p, zc, zx, false, s);
    std::swap(zc, zx);
  }
  return zc;
}

static void drop_vcycle_graphs(amg_handle& h) {
  for (int t = 0; t < 2; ++t) {
    if (h.vexec[t]) (void)hipGraphExecDestroy(h.vexec[t]);
    if (h.vgraph[t]) (void)hipGraphDestroy(h.vgraph[t]);
    h.vexec[t] = nullptr;
    h.vgraph[t] = nullptr;
    h.vout[t] = nullptr;
  }
}

// The V-cycle's kernel sequence and buffers are fixed for a handle, so with
// the graphs option it is captured once per direction (on an internal
// stream) and replayed on the caller's stream.  Event-based profiling needs
// the eager path.
template <typename T>
static T* vcycle_run(amg_handle& h, bool transpose, hipStream_t s) {
  if (!h.opts.graphs || h.prof.mask) return vcycle_level<T>(h, 0, transpose, s);
  const int t = transpose ? 1 : 0;
  if (!h.vexec[t]) {
    if (!h.cap_stream) CAMG_HIP(hipStreamCreateWithFlags(&h.cap_stream, hipStreamNonBlocking));
    CAMG_HIP(hipStreamBeginCapture(h.cap_stream, hipStreamCaptureModeThreadLocal));
    T* out = nullptr;
    try {
      out = vcycle_level<T>(h, 0, transpose, h.cap_stream);
    } catch (...) {
      hipGraph_t g = nullptr;
      (void)hipStreamEndCapture(h.cap_stream, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    CAMG_HIP(hipStreamEndCapture(h.cap_stream, &h.vgraph[t]));
    CAMG_HIP(hipGraphInstantiate(&h.vexec[t], h.vgraph[t], nullptr, nullptr, 0));
    h.vout[t] = out;
  }
  CAMG_HIP(hipGraphLaunch(h.vexec[t], s));
  return reinterpret_cast<T*>(h.vout[t]);
}

static void vcycle_to(amg_handle& h, bool transpose, double* z, hipStream_t s) {
  const int64_t n = h.lev[0].n();
  if (h.opts.precision != CAMG_PREC_FP64) {
    float* out = vcycle_run<float>(h, transpose, s);
    cast_f2d(out, z, n, s);
  } else {
    double* out = vcycle_run<double>(h, transpose, s);
    copy_vec<double>(out, z, n, s);
  }
}

// z = M^{-1} r (or M^{-T} r) on FP64 device vectors.
static void precondition(amg_handle& h, bool transpose, const double* r, double* z, hipStream_t s) {
  DevLevel& D0 = h.lev[0];
  const int64_t n = D0.n();
  if (h.opts.precision != CAMG_PREC_FP64) cast_d2f(r, D0.v32.b.p, n, s);
  else copy_vec<double>(r, D0.v64.b.p, n, s);
  vcycle_to(h, transpose, z, s);
}

// The work vectors of one level, in the order they are laid out in scratch.
template <typename T>
static std::vector<std::pair<DBuf<T>*, int64_t>> work_vectors(DevLevel& D) {
  LevelVecs<T>& V = vecs<T>(D);
  const int64_t n = D.n(), nu = std::max<int64_t>(D.n_u, 1), nl = std::max<int64_t>(D.n_l, 1);
  return {{&V.b, n},      {&V.z, n},       {&V.zn, n},     {&V.r, n},    {&V.delta, nl},
          {&V.delta2, nl}, {&V.qrhs, nl},   {&V.aux1, nu},  {&V.aux2, nu}, {&V.su, nu}};
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Bytes of scratch that one V-cycle of this handle needs.
template <typename T>
static size_t noalloc_bytes(amg_handle& h) {
  size_t total = 0;
  for (DevLevel& D : h.lev)
    for (auto& wv : work_vectors<T>(D)) total += align256((size_t)wv.second * sizeof(T));
  return total;
}

// One eager V-cycle whose work vectors live in this device's scratch array:
// the level buffers of the handle are pointed at carve-outs of it for the
// duration of the launches (restored on every exit path), the carved region
// is cleared first with a fill kernel, and neither graph capture nor event
// profiling runs, so nothing is allocated.  The kernels are the ones of
// amg_vcycle_apply in the same order.
template <typename T>
static void vcycle_noalloc(amg_handle& h, bool transpose, const double* r, double* z, hipStream_t s) {
  const size_t need = noalloc_bytes<T>(h);
  if (need > kNoallocScratchBytes)
    api_fail(CAMG_ERR_TOO_LARGE, "V-cycle work vectors need " + std::to_string(need) +
                                     " bytes; the no-allocation scratch holds " +
                                     std::to_string(kNoallocScratchBytes));
  struct Restore {
    std::vector<std::pair<DBuf<T>*, T*>> saved;
    Prof& prof;
    int mask;
    ~Restore() {
      for (auto& sv : saved) sv.first->p = sv.second;
      prof.mask = mask;
    }
  } restore{{}, h.prof, h.prof.mask};
  h.prof.mask = 0;
  unsigned char* base = static_cast<unsigned char*>(h.scratch);
  size_t off = 0;
  for (DevLevel& D : h.lev)
    for (auto& wv : work_vectors<T>(D)) {
      restore.saved.emplace_back(wv.first, wv.first->p);
      wv.first->p = reinterpret_cast<T*>(base + off);
      off += align256((size_t)wv.second * sizeof(T));
    }
  zero_vec<float>(reinterpret_cast<float*>(base), (int64_t)(off / sizeof(float)), s);
  const int64_t n = h.lev[0].n();
  LevelVecs<T>& V0 = vecs<T>(h.lev[0]);
  if constexpr (std::is_same<T, float>::value) {
    cast_d2f(r, V0.b.p, n, s);
    cast_f2d(vcycle_level<float>(h, 0, transpose, s), z, n, s);
  } else {
    copy_vec<double>(r, V0.b.p, n, s);
    copy_vec<double>(vcycle_level<double>(h, 0, transpose, s), z, n, s);
  }
}

// Runs the V-cycle on the level-0 input already in vecs(0).b and writes the
// FP64 result to z.
// y = A x, or y = b - A x when b is given (FP64 level-0 operator).
static void apply_op(amg_handle& h, bool transpose, const double* x, const double* b, double* y, hipStream_t s) {
  DevLevel& D = h.lev[0];
  const int nu = (int)D.n_u, nl = (int)D.n_l;
  ProfScope ps(&h.prof, CAMG_KCLASS_OPERATOR, s);
  const int mode = b ? 1 : 0;
  if (D.bell_for<double>()) {
    if (!transpose)
      blk_spmv_bell<double>(D.kview<double>(false), D.G.view<double>(), D.B.view<double>(), D.C.view<double>(), x,
                            x + nu, b, b ? b + nu : nullptr, y, y + nu, nu, nl, mode, s);
    else
      blk_spmv_bell<double>(D.kview<double>(true), D.BT.view<double>(), D.GT.view<double>(), D.CT.view<double>(), x,
                            x + nu, b, b ? b + nu : nullptr, y, y + nu, nu, nl, mode, s);
  } else if (!transpose)
    blk_spmv<double>(D.K.view<double>(), D.G.view<double>(), D.B.view<double>(), D.C.view<double>(), x, x + nu, b,
                     b ? b + nu : nullptr, y, y + nu, nu, nl, mode, D.sg_K, s);
  else
    blk_spmv<double>(D.KT.view<double>(), D.BT.view<double>(), D.GT.view<double>(), D.CT.view<double>(), x, x + nu, b,
                     b ? b + nu : nullptr, y, y + nu, nu, nl, mode, D.sg_K, s);
}

static void ensure_krylov(amg_handle& h, int m) {
  if (h.m_alloc >= m) return;
  const int64_t n = h.n;
  h.V.alloc((size_t)(n * (m + 1)));
  h.Z.alloc((size_t)(n * m));
  h.w.alloc((size_t)n);
  h.r.alloc((size_t)n);
  h.H.alloc((size_t)((m + 1) * m));
  h.cs.alloc((size_t)m);
  h.sn.alloc((size_t)m);
  h.g.alloc((size_t)(m + 1));
  h.h1.alloc((size_t)(m + 1));
  h.h2.alloc((size_t)(m + 1));
  h.hn2.alloc(1);
  h.partial.alloc((size_t)((m + 1) * std::max(mdot_blocks(n), cgs_blocks(n))));
  h.out.alloc(4);
  h.y.alloc((size_t)m);
  h.Gram.alloc(64 * 64);
  h.gn.alloc(65);
  h.cc.alloc(64);
  h.m_alloc = m;
}

static void read_out(amg_handle& h, hipStream_t s) {
  CAMG_HIP(hipMemcpyAsync(h.hbuf, h.out.p, 4 * sizeof(double), hipMemcpyDeviceToHost, s));
  CAMG_HIP(hipStreamSynchronize(s));
}

static int gmres(amg_handle& h, bool transpose, const double* b, double* x, const amg_gmres_options& o,
                 amg_gmres_result* res, hipStream_t s) {
  const int m = o.m;
  const int64_t n = h.n;
  ensure_krylov(h, m);
  const bool fixed = o.fixed_iters > 0;
  const int limit = fixed ? o.fixed_iters : o.max_iters;
  const double o_rtol = o.rtol;
  const int lag = std::min(std::max(1, o.lookahead), amg_handle::kSlots - 1);
  CAMG_HIP(hipEventRecord(h.ev0, s));
  // r0 = b - A x0, beta = ||r0||
  apply_op(h, transpose, x, b, h.r.p, s);
  mdot(h.r.p, n, 1, h.r.p, n, h.partial.p, h.hn2.p, s);
  restart_init(h.r.p, h.hn2.p, h.V.p, h.g.p, m + 1, h.out.p, n, s);
  read_out(h, s);
  const double r0 = h.hbuf[0];
  if (!std::isfinite(r0)) api_fail(CAMG_ERR_NONFINITE, "non-finite initial residual");
  int total = 0, restarts = 0;
  double est = 1.0, true_rel = 1.0;
  int status = CAMG_NOT_CONVERGED;
  if (r0 == 0.0) {
    est = true_rel = 0.0;
    status = CAMG_OK;
  } else {
    const bool fused = (m + 1 <= 64);
    const bool mixed = h.opts.precision != CAMG_PREC_FP64;
    DevLevel& D0 = h.lev[0];
    // Launches Arnoldi step j: v_j, z_j = M^-1 v_j, w = A z_j, CGS2, Givens;
    // leaves w / ||w|| scaling for the next step's prep and copies the
    // 4-double result block to pinned slot j % 2.
    auto launch_iter = [&](int j) {
      double* vj = h.V.p + (int64_t)j * n;
      double* zj = h.Z.p + (int64_t)j * n;
      const double* scale = j ? h.out.p + 2 : nullptr;
      if (mixed) arnoldi_prep<float>(h.w.p, scale, vj, D0.v32.b.p, n, s);
      else arnoldi_prep<double>(h.w.p, scale, vj, D0.v64.b.p, n, s);
      if (D0.bell_for<double>()) {
        // the FP64 operator reads the V-cycle output directly and stores z_j
        const int nu0 = (int)D0.n_u, nl0 = (int)D0.n_l;
        const DBELL<double> Kx = D0.kview<double>(transpose);
        const DCSR<double> A12 = transpose ? D0.BT.view<double>() : D0.G.view<double>();
        const DCSR<double> A21 = transpose ? D0.GT.view<double>() : D0.B.view<double>();
        const DCSR<double> A22 = transpose ? D0.CT.view<double>() : D0.C.view<double>();
        if (mixed) {
          float* out = vcycle_run<float>(h, transpose, s);
          ProfScope ps(&h.prof, CAMG_KCLASS_OPERATOR, s);
          op_apply_from_f32(Kx, A12, A21, A22, out, h.w.p, zj, nu0, nl0, s);
        } else {
          double* out = vcycle_run<double>(h, transpose, s);
          ProfScope ps(&h.prof, CAMG_KCLASS_OPERATOR, s);
          op_apply_copy(Kx, A12, A21, A22, out, h.w.p, zj, nu0, nl0, s);
        }
      } else {
        vcycle_to(h, transpose, zj, s);
        apply_op(h, transpose, zj, nullptr, h.w.p, s);
      }
      {
        ProfScope ps(&h.prof, CAMG_KCLASS_ORTHO, s);
        if (fused && o.ortho == 1) {
          cgs2_gram(h.V.p, n, j + 1, h.w.p, n, h.partial.p, h.h1.p, h.h2.p, h.cc.p, h.Gram.p, h.gn.p,
                    j ? h.out.p + 2 : nullptr, h.H.p, m + 1, h.cs.p, h.sn.p, h.g.p, h.out.p,
                    h.hbuf_dev + 4 + 4 * (j % amg_handle::kSlots), s);
        } else if (fused) {
          cgs_pass1(h.V.p, n, j + 1, h.w.p, n, h.partial.p, h.h1.p, s);
          cgs_pass2(h.V.p, n, j + 1, h.w.p, n, h.h1.p, h.partial.p, h.h2.p, s);
          cgs_pass3(h.V.p, n, j + 1, h.w.p, n, h.h1.p, h.h2.p, h.partial.p, h.H.p, m + 1, h.cs.p, h.sn.p, h.g.p,
                    h.out.p, h.hbuf_dev + 4 + 4 * (j % amg_handle::kSlots), s);
        } else {
          mdot(h.V.p, n, j + 1, h.w.p, n, h.partial.p, h.h1.p, s);
          gemv_acc(h.V.p, n, j + 1, h.h1.p, -1.0, h.w.p, n, s);
          mdot(h.V.p, n, j + 1, h.w.p, n, h.partial.p, h.h2.p, s);
          gemv_acc(h.V.p, n, j + 1, h.h2.p, -1.0, h.w.p, n, s);
          mdot(h.w.p, n, 1, h.w.p, n, h.partial.p, h.hn2.p, s);
          arnoldi_update(h.H.p, m + 1, h.cs.p, h.sn.p, h.g.p, h.h1.p, h.h2.p, h.hn2.p, j, h.out.p,
                         h.hbuf_dev + 4 + 4 * (j % amg_handle::kSlots), s);
        }
      }
      // the finish kernel wrote the step's result block into pinned slot j % kSlots
      CAMG_HIP(hipEventRecord(h.evq[j % amg_handle::kSlots], s));
    };
    // Reads step j's result (`lag` steps behind the launches); true = stop.
    auto check = [&](int j) -> bool {
      const int sl = j % amg_handle::kSlots;
      CAMG_HIP(hipEventSynchronize(h.evq[sl]));
      const double* o = h.hbuf + 4 + 4 * sl;
      est = o[0] / r0;
      if (!std::isfinite(est)) api_fail(CAMG_ERR_NONFINITE, "non-finite residual estimate");
      // happy breakdown: the new Arnoldi vector vanishes relative to the
      // Hessenberg column, h_{j+1,j} <= 1e-300 ||H(:, j)||
      if (o[1] <= 1e-300 * o[3]) return true;
      return !fixed && est <= o_rtol;
    };
    for (;;) {
      int k = 0;
      bool stopped = false;
      int launched = 0;
      int checked = 0;  // steps of this cycle whose result has been read
      for (int j = 0; j < m; ++j) {
        if (total >= limit) break;
        launch_iter(j);
        ++total;
        launched = j + 1;
        if (j - lag >= 0) {
          ++checked;
          if (check(j - lag)) {
            // steps j-lag+1 .. j were launched speculatively: they never
            // enter the solution
            total -= lag;
            k = j - lag + 1;
            stopped = true;
            break;
          }
        }
      }
      if (!stopped) {
        k = launched;
        for (int q = checked; q < launched; ++q) {
          if (check(q)) {
            total -= launched - (q + 1);
            k = q + 1;
            break;
          }
        }
      }
      hess_solve(h.H.p, m + 1, h.g.p, h.y.p, k, s);
      gemv_acc(h.Z.p, n, k, h.y.p, 1.0, x, n, s);
      apply_op(h, transpose, x, b, h.r.p, s);
      mdot(h.r.p, n, 1, h.r.p, n, h.partial.p, h.hn2.p, s);
      restart_init(h.r.p, h.hn2.p, h.V.p, h.g.p, m + 1, h.out.p, n, s);
      read_out(h, s);
      true_rel = h.hbuf[0] / r0;
      if (!std::isfinite(true_rel)) api_fail(CAMG_ERR_NONFINITE, "non-finite residual");
      if (fixed) {
        if (total >= limit) {
          status = CAMG_OK;
          break;
        }
      } else {
        if (true_rel <= o.rtol) {
          status = CAMG_OK;
          break;
        }
        if (total >= limit) break;
      }
      if (h.hbuf[0] == 0.0) {
        status = CAMG_OK;
        break;
      }
      ++restarts;
    }
  }
  CAMG_HIP(hipEventRecord(h.ev1, s));
  CAMG_HIP(hipEventSynchronize(h.ev1));
  float ms = 0.f;
  CAMG_HIP(hipEventElapsedTime(&ms, h.ev0, h.ev1));
  if (res) {
    res->iters = total;
    res->restarts = restarts;
    res->status = status;
    res->rel_res_est = est;
    res->rel_res_true = true_rel;
    res->seconds = ms * 1e-3;
  }
  return status;
}

template <typename F>
static int guarded(F&& f) {
  try {
    return f();
  } catch (const ApiError& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const SetupError& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const HipError& e) {
    g_last_error = std::string("HIP error ") + hipGetErrorString(e.err) + " in " + e.where;
    return CAMG_ERR_HIP;
  } catch (const OomError& e) {
    g_last_error = "device allocation of " + std::to_string(e.bytes) + " bytes failed";
    return CAMG_ERR_OOM;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return CAMG_ERR_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return CAMG_ERR_INVALID_ARG;
  }
}

}  // namespace camg

// ---------------------------------------------------------------------------
// C-ABI

extern "C" {

void amg_default_options(amg_options* o) {
  if (!o) return;
  o->max_levels = 4;
  o->max_coarse_rows = 1000;
  o->nu_pre = 2;
  o->nu_post = 2;
  o->jacobi_sweeps = 1;
  o->atilde = CAMG_ATILDE_ROWSUM_ABS;
  o->jacobi_diag = CAMG_JACOBI_ATILDE;
  o->precision = CAMG_PREC_FP64;
  o->spmv_format = CAMG_SPMV_AUTO;
  o->graphs = 1;
  o->jacobi_omega = 0.8;
  o->simple_alpha = 0.8;
  o->prolongator = CAMG_PROLONG_TENTATIVE;
  o->schur = CAMG_SCHUR_DIAG;
  o->schur_sweeps = 1;
  o->sa_omega = 4.0 / 3.0;
  o->coarse_solver = CAMG_COARSE_LU;
  o->coarse_sweeps = 2;
  o->smoother = CAMG_SMOOTHER_SIMPLE;
}

void amg_default_gmres_options(amg_gmres_options* o) {
  if (!o) return;
  o->m = 50;
  o->max_iters = 1000;
  o->fixed_iters = 0;
  o->lookahead = 1;
  o->rtol = 1e-8;
  o->ortho = 1;
}

}  // extern "C"

namespace camg {

// device_inverse: keep the coarsest merged matrix for the device LU
// (amg_setup) instead of factorising it on the host (amg_setup_host).
static std::unique_ptr<amg_handle> build_host(const amg_problem* p, const amg_options* opts, bool device_inverse) {
  if (!p) api_fail(CAMG_ERR_INVALID_ARG, "NULL problem");
  amg_options o;
  amg_default_options(&o);
  if (opts) o = *opts;
  if (p->dim < 1 || p->dim > 3) api_fail(CAMG_ERR_INVALID_ARG, "dim must be 1..3");
  if (o.max_levels < 1 || o.nu_pre < 0 || o.nu_post < 0 || o.jacobi_sweeps < 1 ||
      o.precision < CAMG_PREC_FP64 || o.precision > CAMG_PREC_MIXED_BF16 || o.atilde < 0 || o.atilde > 2 ||
      (o.atilde == CAMG_ATILDE_NODAL && o.jacobi_diag != CAMG_JACOBI_ATILDE) ||
      o.jacobi_diag < 0 || o.jacobi_diag > 1 || o.spmv_format < 0 || o.spmv_format > 6 ||
      (o.spmv_format & 3) == 3 || o.spmv_format == (CAMG_SPMV_CSR | CAMG_SPMV_FULL) || o.graphs < 0 ||
      o.graphs > 1 || o.prolongator < 0 || o.prolongator > 1 || o.schur < 0 || o.schur > 2 || o.schur_sweeps < 1 ||
      o.schur_sweeps > 64 || !(o.sa_omega > 0.0) || !std::isfinite(o.sa_omega) || o.coarse_solver < 0 ||
      o.coarse_solver > 1 || o.coarse_sweeps < 1 || o.coarse_sweeps > 64 || o.smoother < 0 || o.smoother > 2 ||
      !(o.simple_alpha > 0.0) || !std::isfinite(o.simple_alpha))
    api_fail(CAMG_ERR_INVALID_ARG, "invalid options");
  const int64_t nu = p->K.nrows, nl = p->C.nrows;
  if (nu <= 0 || nu % p->dim) api_fail(CAMG_ERR_SHAPE, "n_u must be a positive multiple of dim");
  if (nl < 0 || nu + nl >= (int64_t(1) << 31)) api_fail(CAMG_ERR_SHAPE, "system too large");
  {
    PhaseTimer pt("input checks");
    check_csr(p->K, nu, nu, "K");
    check_csr(p->G, nu, nl, "G");
    check_csr(p->B, nl, nu, "B");
    check_csr(p->C, nl, nl, "C");
  }
  if ((p->n_slave > 0 && !p->slave_dofs) || (p->n_master > 0 && !p->master_dofs) || p->n_slave < 0 ||
      p->n_master < 0)
    api_fail(CAMG_ERR_INVALID_ARG, "interface dof lists");
  auto h = std::make_unique<amg_handle>();
  h->opts = o;
  h->dim = p->dim;
  h->n_u = nu;
  h->n_l = nl;
  h->n = nu + nl;

  HostLevel L0;
  {
    PhaseTimer pt("input copies");
    L0.K = to_host(p->K);
    L0.G = to_host(p->G);
    L0.B = to_host(p->B);
    L0.C = to_host(p->C);
  }
  L0.bs_u = p->dim;
  L0.bs_l = p->dim;
  const int64_t nn = nu / p->dim;
  L0.slave_node.assign((size_t)nn, 0);
  L0.master_node.assign((size_t)nn, 0);
  for (int32_t i = 0; i < p->n_slave; ++i) {
    if (p->slave_dofs[i] < 0 || p->slave_dofs[i] >= nu) api_fail(CAMG_ERR_SHAPE, "slave dof out of range");
    L0.slave_node[p->slave_dofs[i] / p->dim] = 1;
  }
  for (int32_t i = 0; i < p->n_master; ++i) {
    if (p->master_dofs[i] < 0 || p->master_dofs[i] >= nu) api_fail(CAMG_ERR_SHAPE, "master dof out of range");
    L0.master_node[p->master_dofs[i] / p->dim] = 1;
  }
  L0.lm_node.resize((size_t)nl);
  int64_t maxnode = -1;
  for (int64_t j = 0; j < nl; ++j) {
    int32_t v = p->lm_node ? p->lm_node[j] : (int32_t)(j / p->dim);
    if (v < 0) api_fail(CAMG_ERR_SHAPE, "negative multiplier pseudo-node");
    L0.lm_node[j] = v;
    maxnode = std::max<int64_t>(maxnode, v);
  }
  L0.n_nodes_l = maxnode + 1;
  if (p->nullspace && p->n_ns > 0) {
    L0.n_ns_u = p->n_ns;
    L0.ns_u.assign(p->nullspace, p->nullspace + (size_t)nu * p->n_ns);
    for (double v : L0.ns_u)
      if (!std::isfinite(v)) api_fail(CAMG_ERR_NONFINITE, "non-finite null space");
  } else {
    L0.n_ns_u = p->dim;
    L0.ns_u.assign((size_t)nu * p->dim, 0.0);
    for (int64_t i = 0; i < nu; ++i) L0.ns_u[(size_t)(i % p->dim) * nu + i] = 1.0;
  }
  L0.n_ns_l = p->dim;
  L0.ns_l.assign((size_t)nl * p->dim, 0.0);
  for (int64_t j = 0; j < nl; ++j) L0.ns_l[(size_t)(j % p->dim) * nl + j] = 1.0;
  h->host.push_back(std::move(L0));

  SetupOptions so;
  so.max_levels = o.max_levels;
  so.max_coarse_rows = o.max_coarse_rows;
  so.atilde = o.atilde;
  so.jacobi_diag = o.jacobi_diag;
  so.prolongator = o.prolongator;
  so.sa_omega = o.sa_omega;
  so.schur = o.schur;
  so.schur_sweeps = o.schur_sweeps;
  so.simple_coarse = o.coarse_solver == CAMG_COARSE_SIMPLE;
  so.bs_alpha = o.smoother == CAMG_SMOOTHER_BRAESS_SARAZIN ? o.simple_alpha : 0.0;
  so.device_inverse = device_inverse;
  build_hierarchy(h->host, so);
  return h;
}

// Host copies of a problem statement whose arrays are device pointers
// (device_ptrs = 1).  The hierarchy is built on the host, so the arrays are
// copied down once; sizes come from the (host) structure itself.
struct StagedProblem {
  amg_problem p{};
  std::vector<int64_t> rp[4];
  std::vector<int32_t> ci[4];
  std::vector<double> v[4];
  std::vector<int32_t> sd, md, ln;
  std::vector<double> ns;
};

template <typename T>
static void stage_array(std::vector<T>& dst, const T* src, int64_t count, const char* what) {
  if (count < 0) api_fail(CAMG_ERR_SHAPE, std::string(what) + ": negative length");
  dst.resize((size_t)count);
  if (count == 0) return;
  if (!src) api_fail(CAMG_ERR_INVALID_ARG, std::string(what) + " is NULL");
  CAMG_HIP(hipMemcpy(dst.data(), src, (size_t)count * sizeof(T), hipMemcpyDeviceToHost));
}

static void stage_problem(const amg_problem& in, StagedProblem& out) {
  out.p = in;
  out.p.device_ptrs = 0;
  amg_csr* blocks[4] = {&out.p.K, &out.p.G, &out.p.B, &out.p.C};
  const char* names[4] = {"K", "G", "B", "C"};
  for (int b = 0; b < 4; ++b) {
    amg_csr& A = *blocks[b];
    if (A.nrows < 0 || A.nnz < 0 || A.nnz >= (int64_t(1) << 31)) api_fail(CAMG_ERR_SHAPE, std::string(names[b]) + ": sizes");
    stage_array(out.rp[b], A.rowptr, A.nrows + 1, names[b]);
    stage_array(out.ci[b], A.col, A.nnz, names[b]);
    stage_array(out.v[b], A.val, A.nnz, names[b]);
    A.rowptr = out.rp[b].data();
    A.col = A.nnz ? out.ci[b].data() : nullptr;
    A.val = A.nnz ? out.v[b].data() : nullptr;
  }
  stage_array(out.sd, in.slave_dofs, in.n_slave, "slave_dofs");
  stage_array(out.md, in.master_dofs, in.n_master, "master_dofs");
  out.p.slave_dofs = in.n_slave ? out.sd.data() : nullptr;
  out.p.master_dofs = in.n_master ? out.md.data() : nullptr;
  if (in.lm_node) {
    stage_array(out.ln, in.lm_node, in.C.nrows, "lm_node");
    out.p.lm_node = out.ln.data();
  }
  if (in.nullspace && in.n_ns > 0) {
    stage_array(out.ns, in.nullspace, in.K.nrows * (int64_t)in.n_ns, "nullspace");
    out.p.nullspace = out.ns.data();
  }
}

static void need_device(const amg_handle* h) {
  if (h->lev.empty()) api_fail(CAMG_ERR_INVALID_ARG, "handle was built by amg_setup_host and has no device data");
}

}  // namespace camg

extern "C" {

int amg_setup(const amg_problem* p, const amg_options* opts, void* stream, amg_handle** out) {
  return guarded([&]() -> int {
    if (!out) api_fail(CAMG_ERR_INVALID_ARG, "NULL output handle");
    *out = nullptr;
    PhaseTimer pt_all("amg_setup total");
    StagedProblem staged;
    if (p && p->device_ptrs) {
      PhaseTimer pt("device-to-host staging");
      stage_problem(*p, staged);
      p = &staged.p;
    }
    auto h = [&] {
      PhaseTimer pt("host import + hierarchy");
      return build_host(p, opts, true);
    }();
    hipStream_t s = as_stream(stream);
    CAMG_HIP(hipGetDevice(&h->device));
    h->scratch = scratch_address(h->device);
    CAMG_HIP(hipEventCreate(&h->ev0));
    CAMG_HIP(hipEventCreate(&h->ev1));
    CAMG_HIP(hipHostMalloc((void**)&h->hbuf, (4 + 4 * amg_handle::kSlots) * sizeof(double),
                           hipHostMallocMapped | hipHostMallocCoherent));
    CAMG_HIP(hipHostGetDevicePointer((void**)&h->hbuf_dev, h->hbuf, 0));
    for (auto& e : h->evq) CAMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    {
      PhaseTimer pt("device upload");
      upload_hierarchy(*h, s);
    }
    *out = h.release();
    return CAMG_OK;
  });
}

int amg_setup_host(const amg_problem* p, const amg_options* opts, amg_handle** out) {
  return guarded([&]() -> int {
    if (!out) api_fail(CAMG_ERR_INVALID_ARG, "NULL output handle");
    *out = nullptr;
    if (p && p->device_ptrs) api_fail(CAMG_ERR_INVALID_ARG, "amg_setup_host takes host pointers only");
    *out = build_host(p, opts, false).release();
    return CAMG_OK;
  });
}

int amg_num_levels(const amg_handle* h) { return h ? (int)h->host.size() : CAMG_ERR_INVALID_ARG; }

int amg_level_info_get(const amg_handle* h, int level, amg_level_info* out) {
  return guarded([&]() -> int {
    if (!h || !out || level < 0 || level >= (int)h->host.size()) api_fail(CAMG_ERR_INVALID_ARG, "level");
    const HostLevel& L = h->host[level];
    out->n_u = L.n_u();
    out->n_l = L.n_l();
    out->nnz_K = L.K.nnz();
    out->nnz_G = L.G.nnz();
    out->nnz_B = L.B.nnz();
    out->nnz_C = L.C.nnz();
    out->bs_u = L.bs_u;
    out->bs_l = L.bs_l;
    out->n_nodes_u = L.n_u() / std::max(1, L.bs_u);
    out->n_nodes_l = L.n_nodes_l;
    out->n_agg_u = L.n_agg_u;
    out->n_agg_l = L.n_agg_l;
    double tot = 0.0;
    for (const auto& X : h->host) tot += (double)X.nnz_all();
    out->op_complexity = tot / (double)h->host[0].nnz_all();
    out->k_layout = -1;
    out->k_bs = L.bs_u;
    out->k_blocks = 0;
    out->k_slots = 0;
    out->transfer_layout = -1;
    out->k_index_bytes = 0;
    out->k_lower_blocks = 0;
    out->k_nnz_stored = 0;
    out->k_sym_stale = 0;
    if (!h->lev.empty()) {
      const DevLevel& D = h->lev[level];
      out->k_layout = D.bell ? (D.sym ? 3 : 1) : (D.K.bs > 0 ? 2 : 0);
      out->k_index_bytes = D.bell ? (D.Kb.bdel.p ? 2 : 4) : (D.K.bs > 0 ? 4 : 0);
      out->k_blocks = D.bell ? D.k_blocks : (D.K.bs > 0 ? (int64_t)D.K.bcol.n : 0);
      out->k_slots = D.k_slots;
      out->k_lower_blocks = D.k_lower;
      out->k_nnz_stored = D.bell ? D.k_nnz_stored : 0;
      out->k_sym_stale = D.sym_stale ? 1 : 0;
      if (level + 1 < (int)h->lev.size()) out->transfer_layout = D.agg_ok ? 1 : 0;
    }
    return CAMG_OK;
  });
}

int amg_get_aggregates(const amg_handle* h, int level, int32_t* disp_agg, int32_t* lm_agg) {
  return guarded([&]() -> int {
    if (!h || level < 0 || level + 1 >= (int)h->host.size()) api_fail(CAMG_ERR_INVALID_ARG, "level");
    const HostLevel& L = h->host[level];
    if (disp_agg) std::copy(L.agg_u.begin(), L.agg_u.end(), disp_agg);
    if (lm_agg) std::copy(L.agg_l.begin(), L.agg_l.end(), lm_agg);
    return CAMG_OK;
  });
}

int amg_get_level_matrix(const amg_handle* h, int level, int which, int64_t* nrows, int64_t* ncols, int64_t* nnz,
                         int64_t* rowptr, int32_t* col, double* val) {
  return guarded([&]() -> int {
    if (!h || level < 0 || level >= (int)h->host.size() || which < 0 || which > 8)
      api_fail(CAMG_ERR_INVALID_ARG, "level/which");
    const HostLevel& L = h->host[level];
    // which = 7 / 8: the inverse nodal Schur / lumping blocks as a block-diagonal matrix
    auto block_diag = [](const std::vector<double>& v, int bs, int64_t n) {
      HostCSR blk;
      if (v.empty()) return blk;
      blk.nrows = blk.ncols = n;
      blk.rp.resize((size_t)n + 1);
      for (int64_t j = 0; j <= n; ++j) blk.rp[(size_t)j] = j * bs;
      blk.ci.resize((size_t)(n * bs));
      for (int64_t j = 0; j < n; ++j)
        for (int c = 0; c < bs; ++c) blk.ci[(size_t)(j * bs + c)] = (int32_t)((j / bs) * bs + c);
      blk.v = v;
      return blk;
    };
    HostCSR blk;
    if (which == 7) blk = block_diag(L.sblk_inv, L.bs_l, L.n_l());
    if (which == 8) blk = block_diag(L.ablk_inv, L.bs_u, L.n_u());
    const HostCSR* M[9] = {&L.K, &L.G, &L.B, &L.C, &L.P_u, &L.P_l, &L.S, &blk, &blk};
    if ((which == 4 || which == 5) && level + 1 >= (int)h->host.size())
      api_fail(CAMG_ERR_INVALID_ARG, "no transfer on coarsest");
    const HostCSR& A = *M[which];
    if (nrows) *nrows = A.nrows;
    if (ncols) *ncols = A.ncols;
    if (nnz) *nnz = A.nnz();
    if (rowptr) {
      if (A.rp.empty()) rowptr[0] = 0;
      else std::copy(A.rp.begin(), A.rp.end(), rowptr);
    }
    if (col) std::copy(A.ci.begin(), A.ci.end(), col);
    if (val) std::copy(A.v.begin(), A.v.end(), val);
    return CAMG_OK;
  });
}

int amg_update_fine_values(amg_handle* h, const double* K_val, const double* G_val, const double* B_val,
                           const double* C_val, void* stream) {
  return guarded([&]() -> int {
    if (!h) api_fail(CAMG_ERR_INVALID_ARG, "NULL handle");
    need_device(h);
    CAMG_HIP(hipSetDevice(h->device));
    hipStream_t s = as_stream(stream);
    DevLevel& D = h->lev[0];
    struct Item {
      const double* src;
      DevMat* M;
      DevMat* MT;
      DBuf<int32_t>* perm;
    } items[4] = {{K_val, &D.K, &D.KT, &h->d_perm_K},
                  {G_val, &D.G, &D.GT, &h->d_perm_G},
                  {B_val, &D.B, &D.BT, &h->d_perm_B},
                  {C_val, &D.C, &D.CT, &h->d_perm_C}};
    for (auto& it : items) {
      if (!it.src || it.M->nnz == 0) continue;
      CAMG_HIP(hipMemcpyAsync(it.M->v64.p, it.src, it.M->nnz * sizeof(double), hipMemcpyDeviceToDevice, s));
      scatter_perm<double>(it.src, it.perm->p, it.MT->v64.p, it.M->nnz, s);
    }
    if (K_val && D.bell && D.K.nnz) {
      if (D.sym) {
        // the symmetric storage keeps one block of each mirror pair: it stays
        // in use only while the new values are symmetric too
        CAMG_HIP(hipMemsetAsync(h->d_asym.p, 0, sizeof(int32_t), s));
        check_symmetric(K_val, h->d_perm_K.p, D.K.nnz, h->d_asym.p, s);
        int32_t asym = 0;
        CAMG_HIP(hipMemcpyAsync(&asym, h->d_asym.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        CAMG_HIP(hipStreamSynchronize(s));
        const bool stale = asym != 0;
        if (!stale) scatter_pos64(K_val, h->d_bpos_K.p, D.Kb.v64.p, D.K.nnz, s);
        // an FP64 V-cycle switches its level-0 kernels: capture it again
        if (stale != D.sym_stale && h->opts.precision == CAMG_PREC_FP64) drop_vcycle_graphs(*h);
        D.sym_stale = stale;
      } else {
        scatter_pos64(K_val, h->d_bpos_K.p, D.Kb.v64.p, D.K.nnz, s);
        scatter_pos64(K_val, h->d_bpos_KT.p, D.KTb.v64.p, D.K.nnz, s);
      }
    }
    return CAMG_OK;
  });
}

int amg_apply_operator(amg_handle* h, int transpose, const double* x, double* y, void* stream) {
  return guarded([&]() -> int {
    if (!h || !x || !y) api_fail(CAMG_ERR_INVALID_ARG, "NULL argument");
    need_device(h);
    CAMG_HIP(hipSetDevice(h->device));
    apply_op(*h, transpose != 0, x, nullptr, y, as_stream(stream));
    return CAMG_OK;
  });
}

int amg_vcycle_apply(amg_handle* h, int transpose, const double* r, double* z, void* stream) {
  return guarded([&]() -> int {
    if (!h || !r || !z) api_fail(CAMG_ERR_INVALID_ARG, "NULL argument");
    if (r == z) api_fail(CAMG_ERR_INVALID_ARG, "r and z must not overlap");
    need_device(h);
    CAMG_HIP(hipSetDevice(h->device));
    precondition(*h, transpose != 0, r, z, as_stream(stream));
    return CAMG_OK;
  });
}

int amg_vcycle_apply_noalloc(amg_handle* h, int transpose, const double* r, double* z, void* stream) {
  return guarded([&]() -> int {
    if (!h || !r || !z) api_fail(CAMG_ERR_INVALID_ARG, "NULL argument");
    if (r == z) api_fail(CAMG_ERR_INVALID_ARG, "r and z must not overlap");
    need_device(h);
    if (!h->scratch) api_fail(CAMG_ERR_INVALID_ARG, "handle has no scratch address");
    CAMG_HIP(hipSetDevice(h->device));
    if (h->opts.precision != CAMG_PREC_FP64) vcycle_noalloc<float>(*h, transpose != 0, r, z, as_stream(stream));
    else vcycle_noalloc<double>(*h, transpose != 0, r, z, as_stream(stream));
    return CAMG_OK;
  });
}

int fgmres_solve(amg_handle* h, int transpose, const double* b, double* x, const amg_gmres_options* gopts,
                 amg_gmres_result* res, void* stream) {
  return guarded([&]() -> int {
    if (!h || !b || !x) api_fail(CAMG_ERR_INVALID_ARG, "NULL argument");
    amg_gmres_options o;
    amg_default_gmres_options(&o);
    if (gopts) o = *gopts;
    if (o.m < 1 || o.m > 512 || o.max_iters < 0 || o.fixed_iters < 0 || !(o.rtol >= 0.0) || o.ortho < 0 ||
        o.ortho > 1)
      api_fail(CAMG_ERR_INVALID_ARG, "invalid FGMRES options");
    need_device(h);
    CAMG_HIP(hipSetDevice(h->device));
    return gmres(*h, transpose != 0, b, x, o, res, as_stream(stream));
  });
}

int amg_grad_K(amg_handle* h, const double* lam, const double* x, double* dK, void* stream) {
  return guarded([&]() -> int {
    if (!h || !lam || !x || !dK) api_fail(CAMG_ERR_INVALID_ARG, "NULL argument");
    need_device(h);
    CAMG_HIP(hipSetDevice(h->device));
    grad_K(h->lev[0].K.view<double>(), lam, x, dK, as_stream(stream));
    return CAMG_OK;
  });
}

int amg_dense_inverse(const double* A, double* Ainv, int64_t n, void* stream) {
  return guarded([&]() -> int {
    if (!A || !Ainv || n <= 0) api_fail(CAMG_ERR_INVALID_ARG, "NULL argument or n <= 0");
    if (A == Ainv) api_fail(CAMG_ERR_INVALID_ARG, "A and Ainv must not overlap");
    if (n > 46000) api_fail(CAMG_ERR_INVALID_ARG, "n too large for the dense inverse");
    hipStream_t s = as_stream(stream);
    // the singularity threshold of the coarsest solve: 1e-13 max |A_ij|
    DBuf<double> amax(1);
    max_abs(A, n * n, amax.p, s);
    double am = 0.0;
    CAMG_HIP(hipMemcpyAsync(&am, amax.p, sizeof(double), hipMemcpyDeviceToHost, s));
    CAMG_HIP(hipStreamSynchronize(s));
    if (!std::isfinite(am)) api_fail(CAMG_ERR_NONFINITE, "non-finite matrix entry");
    if (!dense_inverse<double>(A, n, 1e-13 * am, Ainv, nullptr, s))
      api_fail(CAMG_ERR_SINGULAR_COARSE, "matrix is singular (pivot below 1e-13 max|A_ij|)");
    return CAMG_OK;
  });
}

int amg_grad_A(amg_handle* h, const double* lam, const double* x, double* dK, double* dG, double* dB, double* dC,
               void* stream) {
  return guarded([&]() -> int {
    if (!h || !lam || !x) api_fail(CAMG_ERR_INVALID_ARG, "NULL argument");
    need_device(h);
    CAMG_HIP(hipSetDevice(h->device));
    const DevLevel& D = h->lev[0];
    const int64_t nu = D.n_u;
    hipStream_t s = as_stream(stream);
    // block (rows, columns) = (u, u), (u, l), (l, u), (l, l) of [u; l]
    if (dK) grad_K(D.K.view<double>(), lam, x, dK, s);
    if (dG) grad_K(D.G.view<double>(), lam, x + nu, dG, s);
    if (dB) grad_K(D.B.view<double>(), lam + nu, x, dB, s);
    if (dC) grad_K(D.C.view<double>(), lam + nu, x + nu, dC, s);
    return CAMG_OK;
  });
}

int amg_profile_enable(amg_handle* h, int mask) {
  if (!h) return CAMG_ERR_INVALID_ARG;
  h->prof.mask = mask;
  return CAMG_OK;
}

int amg_profile_read(amg_handle* h, int kclass, int64_t* launches, double* total_ms) {
  return guarded([&]() -> int {
    if (!h) api_fail(CAMG_ERR_INVALID_ARG, "NULL handle");
    int64_t cnt = 0;
    double tot = 0.0;
    for (auto& r : h->prof.recs) {
      if (r.cls != kclass) continue;
      CAMG_HIP(hipEventSynchronize(r.b));
      float ms = 0.f;
      CAMG_HIP(hipEventElapsedTime(&ms, r.a, r.b));
      tot += ms;
      ++cnt;
    }
    if (launches) *launches = cnt;
    if (total_ms) *total_ms = tot;
    return CAMG_OK;
  });
}

void amg_destroy(amg_handle* h) { delete h; }

const char* amg_strerror(int code) {
  switch (code) {
    case CAMG_OK: return "ok";
    case CAMG_NOT_CONVERGED: return "not converged";
    case CAMG_ERR_INVALID_ARG: return "invalid argument";
    case CAMG_ERR_SHAPE: return "shape or structure error";
    case CAMG_ERR_NONFINITE: return "non-finite value";
    case CAMG_ERR_ZERO_DIAG: return "zero diagonal";
    case CAMG_ERR_RANK_DEFICIENT_AGG: return "rank-deficient aggregate";
    case CAMG_ERR_SINGULAR_COARSE: return "singular coarsest matrix";
    case CAMG_ERR_HIP: return "HIP error";
    case CAMG_ERR_OOM: return "out of memory";
    case CAMG_ERR_UNMAPPED_MULTIPLIER: return "multiplier without slave coupling";
    case CAMG_ERR_TOO_LARGE: return "problem exceeds the no-allocation scratch";
    default: return "unknown status";
  }
}

const char* amg_last_error(void) { return camg::g_last_error.c_str(); }

}  // extern "C"
