// Shared HIP plumbing for libcamg: error propagation and device buffers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace camg {

struct HipError {
  hipError_t err;
  std::string where;
};

#define CAMG_HIP(call)                                                             \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) throw ::camg::HipError{e_, std::string(#call) + " @ " + __FILE__ + ":" + std::to_string(__LINE__)}; \
  } while (0)

// Check for launch errors right after a kernel launch.
#define CAMG_LAUNCHED() CAMG_HIP(hipGetLastError())

struct OomError {
  size_t bytes;
};

// Owning device allocation of n elements of T.
template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  DBuf() = default;
  explicit DBuf(size_t count) { alloc(count); }
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), n(o.n) {
    o.p = nullptr;
    o.n = 0;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      n = o.n;
      o.p = nullptr;
      o.n = 0;
    }
    return *this;
  }
  ~DBuf() { release(); }
  void alloc(size_t count) {
    release();
    n = count;
    if (count == 0) return;
    hipError_t e = hipMalloc((void**)&p, count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      throw OomError{count * sizeof(T)};
    }
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  void upload(const T* host, size_t count, hipStream_t s) {
    if (count) CAMG_HIP(hipMemcpyAsync(p, host, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  void upload(const std::vector<T>& host, hipStream_t s) {
    alloc(host.size());
    upload(host.data(), host.size(), s);
  }
};

// Device CSR view (int32 row pointers: nnz < 2^31 is checked at setup).
template <typename T>
struct DCSR {
  int32_t nrows = 0, ncols = 0;
  int64_t nnz = 0;
  const int32_t* rp = nullptr;
  const int32_t* ci = nullptr;
  const T* v = nullptr;
  // Optional node-blocked copy of the same matrix (bs > 0): the bs rows of a
  // node share block columns bcol[bptr[node] .. bptr[node+1]) and block p
  // holds its values row-major at bval[p bs^2 ...]; the row dots use it when
  // present (one column index per bs^2 values instead of one per value).
  int32_t bs = 0;
  const int32_t* bptr = nullptr;
  const int32_t* bcol = nullptr;
  const T* bval = nullptr;
};

// Device sliced blocked-ELL view of a square node-blocked matrix (bs x bs
// blocks, node-major dofs).  Slice s holds nodes [64 s, 64 s + 64); its
// block columns run over positions p in [slice_ptr[s], slice_ptr[s+1]):
//   bcol[p * 64 + lane]                       block column of node 64 s + lane
//   val[(p * bs * bs + a * bs + b) * 64 + lane] entry (a, b) of that block
// Short rows are padded with zero blocks pointing at a valid node.
// When every block column lies within +-32767 nodes of its row's node (a
// banded node numbering, as on structured meshes), bdel replaces bcol:
//   bdel[p * 64 + lane] = block column - (64 s + lane),
// two bytes per block instead of four.
//
// Symmetric storage (lptr set; K = K^T exactly): the positions above hold
// only the blocks on or right of the block diagonal (column node >= row
// node, always as 16-bit deltas).  The blocks left of it are not stored:
// lower position q in [lptr[s], lptr[s+1]) of lane `lane` holds the word
// w = lidx[q * 64 + lane], whose low 16 bits (signed) are the column node's
// delta, j = 64 s + lane + delta (< the row's node), and whose high 16 bits
// (signed) give the position of block (j, row node) in j's own slice as
// slice_ptr[s] + (w >> 16); the kernel reads that block transposed from
// lane j % 64 there.  Padding: high half INT16_MIN (no block).
template <typename T>
struct DBELL {
  int32_t n_nodes = 0, bs = 0, n_slices = 0;
  int32_t stream = 0;  // 1: load the values nontemporally (they are read once per pass);
                       // symmetric storage: 1 selects the node-per-lane kernels
  const int32_t* slice_ptr = nullptr;
  const int32_t* bcol = nullptr;
  const int16_t* bdel = nullptr;
  const T* val = nullptr;
  // FP32 views only: the values as bfloat16 words (the upper halves of the
  // FP32 words, rounded to nearest even) in place of val, same layout
  const uint16_t* val16 = nullptr;
  const int32_t* lptr = nullptr;  // symmetric storage: lower positions per slice
  const int32_t* lidx = nullptr;  // ... and their (delta, mirror position) words
};

}  // namespace camg
