// Device kernels of libcamg for gfx950 (CDNA4, wave64).
//
// Sparse work is row-parallel CSR: a subgroup of SG lanes owns one row and
// walks its column-index and value streams with unit stride, so the SG
// lanes of a subgroup read contiguous bytes and neighbouring subgroups read
// neighbouring rows.  Row sums are reduced inside the subgroup with
// cross-lane shuffles.  No atomics anywhere: every output element has one
// writer and every reduction has a fixed order, so results repeat bit for
// bit from run to run.
#include "kernels.hpp"

#include <algorithm>
#include <stdexcept>

namespace camg {

namespace {

constexpr int kBlock = 256;
// Levels with more rows than this run the elementwise correction kernels one
// thread per row; smaller ones give each row a 4-lane subgroup.
constexpr int kWideRows = 131072;

template <typename T, int SG>
__device__ __forceinline__ T sg_reduce(T v) {
#pragma unroll
  for (int off = SG / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, SG);
  return v;
}

__device__ __forceinline__ double block_sum(double v, double* lds) {
  v = sg_reduce<double, 64>(v);
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlock / 64; ++w) t += lds[w];
  return t;  // valid in thread 0
}

// Row dot over the node-blocked copy (A.bs > 0): lane-strided over the
// node's blocks, each block's bs values of this row against bs consecutive x.
template <typename T, int SG, int BS>
__device__ __forceinline__ T block_row_dot(const DCSR<T>& A, const T* __restrict__ x, int row, int lane) {
  const int node = row / BS, a = row % BS;
  const int e = A.bptr[node + 1];
  T s = T(0);
  for (int p = A.bptr[node] + lane; p < e; p += SG) {
    const T* __restrict__ v = A.bval + ((size_t)p * BS + a) * BS;
    const T* __restrict__ xc = x + (size_t)A.bcol[p] * BS;
#pragma unroll
    for (int b = 0; b < BS; ++b) s += v[b] * xc[b];
  }
  return s;
}

template <typename T, int SG>
__device__ __forceinline__ T row_dot(const DCSR<T>& A, const T* __restrict__ x, int row, int lane) {
  if (A.bs == 6) return block_row_dot<T, SG, 6>(A, x, row, lane);
  if (A.bs == 3) return block_row_dot<T, SG, 3>(A, x, row, lane);
  T s = T(0);
  const int e = A.rp[row + 1];
#pragma unroll 4
  for (int k = A.rp[row] + lane; k < e; k += SG) s += A.v[k] * x[A.ci[k]];
  return s;
}

// Two products over one row with the same column stream: sum a_ij x_j and
// sum a_ij (d_j * y_j).
template <typename T, int SG>
__device__ __forceinline__ void row_dot2(const DCSR<T>& A, const T* __restrict__ x, const T* __restrict__ d,
                                         const T* __restrict__ y, int row, int lane, T& s1, T& s2) {
  s1 = T(0);
  s2 = T(0);
  const int e = A.rp[row + 1];
#pragma unroll 4
  for (int k = A.rp[row] + lane; k < e; k += SG) {
    const int c = A.ci[k];
    const T a = A.v[k];
    s1 += a * x[c];
    s2 += a * (d[c] * y[c]);
  }
}

// One thread's dot of a short CSR row with x (x converted to T on load).
// The row is taken in chunks of 8: the chunk's column and value loads are
// issued together, then its x gathers, then the products are added in
// entry order -- the same sum as a plain loop, with a dependent-load chain
// of 2 per chunk instead of 2 per entry.
template <typename T, typename XT>
__device__ __forceinline__ T csr_row_serial_x(const DCSR<T>& A, const XT* __restrict__ x, int row) {
  if (A.bs > 0) {  // node-blocked copy: one thread walks the row's blocks
    const int bs = A.bs, node = row / bs, a = row % bs;
    T s = T(0);
    for (int p = A.bptr[node]; p < A.bptr[node + 1]; ++p) {
      const T* v = A.bval + ((size_t)p * bs + a) * bs;
      const XT* xc = x + (size_t)A.bcol[p] * bs;
      for (int b = 0; b < bs; ++b) s += v[b] * (T)xc[b];
    }
    return s;
  }
  constexpr int U = 8;
  const int e = A.rp[row + 1];
  T s = T(0);
  for (int k0 = A.rp[row]; k0 < e; k0 += U) {
    int c[U];
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool in = k0 + u < e;
      c[u] = in ? A.ci[k0 + u] : 0;
      v[u] = in ? A.v[k0 + u] : T(0);
    }
    T xv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) xv[u] = (k0 + u < e) ? (T)x[c[u]] : T(0);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (k0 + u < e) s += v[u] * xv[u];
  }
  return s;
}

template <typename T>
__device__ __forceinline__ T csr_row_serial(const DCSR<T>& A, const T* __restrict__ x, int row) {
  return csr_row_serial_x<T, T>(A, x, row);
}

template <typename T, int SG, int MODE>
__global__ void __launch_bounds__(kBlock) k_blk_spmv(DCSR<T> A11, DCSR<T> A12, DCSR<T> A21, DCSR<T> A22,
                                                     const T* __restrict__ x1, const T* __restrict__ x2,
                                                     const T* __restrict__ b1, const T* __restrict__ b2,
                                                     T* __restrict__ y1, T* __restrict__ y2, int n1, int n) {
  const int row = blockIdx.x * (kBlock / SG) + threadIdx.x / SG;
  const int lane = threadIdx.x % SG;
  if (row >= n) return;  // uniform across the subgroup
  T s = T(0);
  if (row < n1) {
    if (A11.nnz) s = row_dot<T, SG>(A11, x1, row, lane);
    if (A12.nnz) s += row_dot<T, SG>(A12, x2, row, lane);
  } else {
    const int j = row - n1;
    if (A21.nnz) s = row_dot<T, SG>(A21, x1, j, lane);
    if (A22.nnz) s += row_dot<T, SG>(A22, x2, j, lane);
  }
  s = sg_reduce<T, SG>(s);
  if (lane == 0) {
    if (row < n1) {
      if (MODE == 0) y1[row] = s;
      else if (MODE == 1) y1[row] = b1[row] - s;
      else y1[row] += s;
    } else {
      const int j = row - n1;
      if (MODE == 0) y2[j] = s;
      else if (MODE == 1) y2[j] = b2[j] - s;
      else y2[j] += s;
    }
  }
}

template <typename T, int SG>
__global__ void __launch_bounds__(kBlock) k_smooth_u(DCSR<T> K, DCSR<T> G, const T* __restrict__ zu,
                                                     const T* __restrict__ zl, const T* __restrict__ bu,
                                                     const T* __restrict__ jinv, T omega, T* __restrict__ znu,
                                                     T* __restrict__ r_out, T* __restrict__ w_out, int n_u) {
  const int row = blockIdx.x * (kBlock / SG) + threadIdx.x / SG;
  const int lane = threadIdx.x % SG;
  if (row >= n_u) return;
  T s = row_dot<T, SG>(K, zu, row, lane);
  if (G.nnz) s += row_dot<T, SG>(G, zl, row, lane);
  s = sg_reduce<T, SG>(s);
  if (lane == 0) {
    const T r = bu[row] - s;
    const T w = omega * jinv[row] * r;
    znu[row] = zu[row] + w;
    if (r_out) {
      r_out[row] = r;
      w_out[row] = w;
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_smooth_u_first(const T* __restrict__ bu, const T* __restrict__ jinv,
                                                           T omega, T* __restrict__ znu, T* __restrict__ r_out,
                                                           T* __restrict__ w_out, int n_u) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_u) return;
  const T r = bu[i];
  const T w = omega * jinv[i] * r;
  znu[i] = w;
  if (r_out) {
    r_out[i] = r;
    w_out[i] = w;
  }
}

template <typename T, int SG>
__global__ void __launch_bounds__(kBlock) k_jacobi_extra(DCSR<T> M, const T* __restrict__ w, const T* __restrict__ r,
                                                         const T* __restrict__ jinv, T omega, T* __restrict__ w_out,
                                                         const T* __restrict__ zu, T* __restrict__ znu, int last,
                                                         int n_u) {
  const int row = blockIdx.x * (kBlock / SG) + threadIdx.x / SG;
  const int lane = threadIdx.x % SG;
  if (row >= n_u) return;
  T s = row_dot<T, SG>(M, w, row, lane);
  s = sg_reduce<T, SG>(s);
  if (lane == 0) {
    const T wn = w[row] + omega * jinv[row] * (r[row] - s);
    w_out[row] = wn;
    if (last) znu[row] = (zu ? zu[row] : T(0)) + wn;
  }
}

template <typename T, int SG, bool FIRST>
__global__ void __launch_bounds__(kBlock) k_smooth_l(DCSR<T> B, DCSR<T> C, const T* __restrict__ znu,
                                                     const T* __restrict__ zl, const T* __restrict__ bl,
                                                     const T* __restrict__ sdinv, T alpha, T* __restrict__ znl,
                                                     T* __restrict__ delta, T* __restrict__ rhs_out, int n_l) {
  const int row = blockIdx.x * (kBlock / SG) + threadIdx.x / SG;
  const int lane = threadIdx.x % SG;
  if (row >= n_l) return;
  T s = T(0);
  if (B.nnz) s = row_dot<T, SG>(B, znu, row, lane);
  if (!FIRST && C.nnz) s += row_dot<T, SG>(C, zl, row, lane);
  s = sg_reduce<T, SG>(s);
  if (lane == 0) {
    const T q = -(bl[row] - s);
    if (rhs_out) rhs_out[row] = q;
    if (!sdinv) return;  // block option: the nodal step divides
    const T d = q * sdinv[row];
    delta[row] = d;
    znl[row] = (FIRST ? T(0) : zl[row]) + alpha * d;
  }
}

template <typename T, int SG>
__global__ void __launch_bounds__(kBlock) k_correct_u(DCSR<T> G, const int32_t* __restrict__ rows, int n_rows,
                                                      const T* __restrict__ delta, const T* __restrict__ ainv,
                                                      T alpha, T* __restrict__ znu) {
  const int idx = blockIdx.x * (kBlock / SG) + threadIdx.x / SG;
  const int lane = threadIdx.x % SG;
  if (idx >= n_rows) return;
  const int i = rows[idx];
  T s = row_dot<T, SG>(G, delta, i, lane);
  s = sg_reduce<T, SG>(s);
  if (lane == 0) znu[i] -= alpha * ainv[i] * s;
}

template <typename T, int SG, bool FIRST>
__global__ void __launch_bounds__(kBlock) k_tsmooth_u(DCSR<T> KT, DCSR<T> BT, const T* __restrict__ zu,
                                                      const T* __restrict__ zl, const T* __restrict__ bu,
                                                      T* __restrict__ su, int n_u) {
  const int row = blockIdx.x * (kBlock / SG) + threadIdx.x / SG;
  const int lane = threadIdx.x % SG;
  if (row >= n_u) return;
  if (FIRST) {
    if (lane == 0) su[row] = bu[row];
    return;
  }
  T s = row_dot<T, SG>(KT, zu, row, lane);
  if (BT.nnz) s += row_dot<T, SG>(BT, zl, row, lane);
  s = sg_reduce<T, SG>(s);
  if (lane == 0) su[row] = bu[row] - s;
}

template <typename T, int SG, bool FIRST>
__global__ void __launch_bounds__(kBlock) k_tsmooth_l(DCSR<T> GT, DCSR<T> CT, const T* __restrict__ zu,
                                                      const T* __restrict__ zl, const T* __restrict__ bl,
                                                      const T* __restrict__ su, const T* __restrict__ ainv,
                                                      const T* __restrict__ sdinv, T alpha, T* __restrict__ znl,
                                                      T* __restrict__ delta, T* __restrict__ rhs_out, int n_l) {
  const int row = blockIdx.x * (kBlock / SG) + threadIdx.x / SG;
  const int lane = threadIdx.x % SG;
  if (row >= n_l) return;
  T gz = T(0), gs = T(0), cz = T(0);
  if (GT.nnz) {
    if (ainv) row_dot2<T, SG>(GT, zu, ainv, su, row, lane, gz, gs);
    else if (!FIRST) gz = row_dot<T, SG>(GT, zu, row, lane);
  }
  if (!FIRST && CT.nnz) cz = row_dot<T, SG>(CT, zl, row, lane);
  gz = sg_reduce<T, SG>(gz);
  gs = sg_reduce<T, SG>(gs);
  cz = sg_reduce<T, SG>(cz);
  if (lane == 0) {
    const T sl = FIRST ? bl[row] : bl[row] - gz - cz;
    const T q = -(sl - gs);
    if (rhs_out) rhs_out[row] = q;
    if (!sdinv) return;
    const T d = q * sdinv[row];
    delta[row] = d;
    znl[row] = (FIRST ? T(0) : zl[row]) + alpha * d;
  }
}

// Row dot of a short interface row: one thread (SG = 1, chunked loads) or
// SG lanes reduced across the subgroup (every lane gets the sum).
template <typename T, int SG>
__device__ __forceinline__ T short_row_dot(const DCSR<T>& A, const T* __restrict__ x, int row, int lane) {
  if (SG == 1) return csr_row_serial<T>(A, x, row);
  return sg_reduce<T, SG>(row_dot<T, SG>(A, x, row, lane));
}

// SG = 1 on large levels keeps the elementwise streams of one thread per row
// coalesced; small levels use SG lanes per row so the interface rows' dots do
// not serialise on one thread.
template <typename T, int SG>
__global__ void __launch_bounds__(kBlock) k_tcorrect_u(DCSR<T> BT, const T* __restrict__ su,
                                                       const T* __restrict__ delta, const T* __restrict__ jinv,
                                                       T omega, T alpha, const T* __restrict__ zu,
                                                       T* __restrict__ znu, T* __restrict__ t_out,
                                                       T* __restrict__ w_out, int n_u) {
  const int i = blockIdx.x * (kBlock / SG) + threadIdx.x / SG;
  const int lane = threadIdx.x % SG;
  if (i >= n_u) return;
  const T bd = BT.nnz ? short_row_dot<T, SG>(BT, delta, i, lane) : T(0);
  if (lane != 0) return;
  const T t = su[i] - alpha * bd;
  const T w = omega * jinv[i] * t;
  znu[i] = (zu ? zu[i] : T(0)) + w;
  if (t_out) {
    t_out[i] = t;
    w_out[i] = w;
  }
}

// Uzawa update of the displacements: zn_u = z_u + alpha w (z_u null: zero).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_uzawa_update(const T* __restrict__ zu, const T* __restrict__ w, T alpha,
                                                         T* __restrict__ znu, int n_u) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= n_u) return;
  znu[i] = (zu ? zu[i] : T(0)) + alpha * w[i];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_dense_gemv(const T* __restrict__ M, const T* __restrict__ x,
                                                       T* __restrict__ y, int n) {
  const int row = blockIdx.x * (kBlock / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (row >= n) return;
  const T* m = M + (int64_t)row * n;
  T s = T(0);
  for (int c = lane; c < n; c += 64) s += m[c] * x[c];
  s = sg_reduce<T, 64>(s);
  if (lane == 0) y[row] = s;
}

__global__ void k_cast_d2f(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}
__global__ void k_cast_f2d(const float* __restrict__ x, double* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = (double)x[i];
}
template <typename T>
__global__ void k_copy(const T* __restrict__ x, T* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = x[i];
}
template <typename T>
__global__ void k_zero(T* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) y[i] = T(0);
}




// First forward sweep from z = 0 in two kernels: the multiplier rows form
// the prediction w = omega * jinv .* b_u on the fly, then the displacement
// rows apply prediction and correction together.
template <typename T, int SG>
__global__ void __launch_bounds__(kBlock) k_smooth_l_first(DCSR<T> B, const T* __restrict__ bu,
                                                           const T* __restrict__ jinv, T omega,
                                                           const T* __restrict__ bl, const T* __restrict__ sdinv,
                                                           T alpha, T* __restrict__ znl, T* __restrict__ delta,
                                                           T* __restrict__ rhs_out, int n_l) {
  const int row = blockIdx.x * (kBlock / SG) + threadIdx.x / SG;
  const int lane = threadIdx.x % SG;
  if (row >= n_l) return;
  T s = T(0);
  if (B.nnz) {
    const int e = B.rp[row + 1];
#pragma unroll 4
    for (int k = B.rp[row] + lane; k < e; k += SG) {
      const int c = B.ci[k];
      s += B.v[k] * (omega * jinv[c] * bu[c]);
    }
  }
  s = sg_reduce<T, SG>(s);
  if (lane == 0) {
    const T q = -(bl[row] - s);
    if (rhs_out) rhs_out[row] = q;
    if (!sdinv) return;
    const T d = q * sdinv[row];
    delta[row] = d;
    znl[row] = alpha * d;
  }
}

// One undamped Jacobi sweep on the Schur system S delta = q:
// d_out = d_in + sdinv .* (q - S d_in); on the last sweep also
// zn_l = z_l + alpha * d_out (z_l null: zero).
template <typename T, int SG>
__global__ void __launch_bounds__(kBlock) k_schur_jacobi(DCSR<T> S, const T* __restrict__ q,
                                                         const T* __restrict__ d_in, const T* __restrict__ sdinv,
                                                         T* __restrict__ d_out, const T* __restrict__ zl, T alpha,
                                                         T* __restrict__ znl, int last, int n_l) {
  const int row = blockIdx.x * (kBlock / SG) + threadIdx.x / SG;
  const int lane = threadIdx.x % SG;
  if (row >= n_l) return;
  T s = row_dot<T, SG>(S, d_in, row, lane);
  s = sg_reduce<T, SG>(s);
  if (lane == 0) {
    const T dn = d_in[row] + sdinv[row] * (q[row] - s);
    d_out[row] = dn;
    if (last) znl[row] = (zl ? zl[row] : T(0)) + alpha * dn;
  }
}

// One step of nodal block Jacobi on the Schur system S delta = q (block
// option), one thread per multiplier node j (BS consecutive rows):
//   d_out_j = d_in_j + M_j (q_j - (S d_in)_j),   d_in null: d_out_j = M_j q_j,
// M_j the inverse of S's j-th diagonal block (row-major), applied transposed
// with TRANS for the S^T system (S passed as S^T then).  On the last step
// also zn_l = z_l + alpha * d_out (z_l null: zero).
template <typename T, int BS, bool TRANS>
__global__ void __launch_bounds__(kBlock) k_schur_block(DCSR<T> S, const T* __restrict__ q,
                                                        const T* __restrict__ d_in, const T* __restrict__ blk,
                                                        T* __restrict__ d_out, const T* __restrict__ zl, T alpha,
                                                        T* __restrict__ znl, int last, int n_nodes) {
  const int j = blockIdx.x * kBlock + threadIdx.x;
  if (j >= n_nodes) return;
  T r[BS];
#pragma unroll
  for (int a = 0; a < BS; ++a) {
    const int row = j * BS + a;
    r[a] = q[row];
    if (d_in) r[a] -= csr_row_serial<T>(S, d_in, row);
  }
  const T* M = blk + (size_t)j * (BS * BS);
#pragma unroll
  for (int a = 0; a < BS; ++a) {
    const int row = j * BS + a;
    T d = d_in ? d_in[row] : T(0);
#pragma unroll
    for (int b = 0; b < BS; ++b) d += (TRANS ? M[b * BS + a] : M[a * BS + b]) * r[b];
    d_out[row] = d;
    if (last) znl[row] = (zl ? zl[row] : T(0)) + alpha * d;
  }
}

// Nodal lumping option, one thread per node j (BS consecutive dofs):
//   v_j = scale * M_j x_j   (M_j^T x_j with TRANS; M row-major per node),
//   w_out_j = v_j, y_out_j = y_in_j + v_j (y_in null: zero).
// y_in may alias y_out (each thread reads its own rows first).  With list,
// only the listed nodes (n_nodes of them).
template <typename T, int BS, bool TRANS>
__global__ void __launch_bounds__(kBlock) k_node_apply(const T* __restrict__ M, const T* __restrict__ x, T scale,
                                                       const T* y_in, T* y_out, T* __restrict__ w_out, int n_nodes,
                                                       const int32_t* __restrict__ list) {
  const int idx = blockIdx.x * kBlock + threadIdx.x;
  if (idx >= n_nodes) return;
  const int j = list ? list[idx] : idx;
  const T* Mj = M + (size_t)j * (BS * BS);
  T xv[BS], v[BS];
#pragma unroll
  for (int b = 0; b < BS; ++b) xv[b] = x[(size_t)j * BS + b];
#pragma unroll
  for (int a = 0; a < BS; ++a) {
    T acc = T(0);
#pragma unroll
    for (int b = 0; b < BS; ++b) acc += (TRANS ? Mj[b * BS + a] : Mj[a * BS + b]) * xv[b];
    v[a] = scale * acc;
  }
#pragma unroll
  for (int a = 0; a < BS; ++a) {
    const size_t row = (size_t)j * BS + a;
    if (w_out) w_out[row] = v[a];
    if (y_out) y_out[row] = (y_in ? y_in[row] : T(0)) + v[a];
  }
}

template <typename T, int SG>
__global__ void __launch_bounds__(kBlock) k_smooth_u_first_corr(DCSR<T> G, const T* __restrict__ bu,
                                                                const T* __restrict__ jinv, T omega,
                                                                const T* __restrict__ delta,
                                                                const T* __restrict__ ainv, T alpha,
                                                                T* __restrict__ znu, int n_u) {
  const int i = blockIdx.x * (kBlock / SG) + threadIdx.x / SG;
  const int lane = threadIdx.x % SG;
  if (i >= n_u) return;
  const T gd = G.nnz ? short_row_dot<T, SG>(G, delta, i, lane) : T(0);
  if (lane != 0) return;
  T v = omega * jinv[i] * bu[i];
  if (G.nnz) v -= alpha * ainv[i] * gd;
  znu[i] = v;
}

// ---- fused CGS2 passes -------------------------------------------------------

constexpr int kCgsBlock = 256;

// Butterfly reduce-scatter across a wave: every lane holds KMAX (a power of
// two <= 64) values a[0..KMAX); afterwards lane l holds the wave total of
// coefficient l >> (6 - log2 KMAX).  At the stage with lane offset o each lane
// keeps one half of its values (the upper half when bit o of its lane id is
// set), sends the other half to lane l ^ o and adds what it receives: KMAX-1
// shuffles instead of 6 KMAX for separate trees.  Addition order is fixed.
// One butterfly stage on the first M entries of a (lane offset O), then the
// next stage on the half that was kept; unrolled at compile time so the
// array stays in registers.
template <int KMAX, int M, int O>
__device__ __forceinline__ void reduce_scatter_stage(double (&a)[KMAX], int lane) {
  if constexpr (M > 1) {
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < M / 2; ++i) {
      const double send = up ? a[i] : a[i + M / 2];
      const double keep = up ? a[i + M / 2] : a[i];
      a[i] = keep + __shfl_xor(send, O, 64);
    }
    reduce_scatter_stage<KMAX, M / 2, O / 2>(a, lane);
  }
}

template <int KMAX>
__device__ __forceinline__ double wave_reduce_scatter(double (&a)[KMAX]) {
  const int lane = threadIdx.x % 64;
  reduce_scatter_stage<KMAX, KMAX, 32>(a, lane);
  double v = a[0];
  // lanes that share a coefficient (low lane bits) still hold partial sums
#pragma unroll
  for (int o = 64 / KMAX / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// One Krylov row per thread: the thread keeps its kk basis entries in
// registers, so pass 2 reads V once for both the update and the new dots.
// Each workgroup writes partial[k * gridDim.x + blockIdx.x] for its 256 rows
// (wave shuffle trees, then the four waves in order).
template <int KMAX, int PASS>
__global__ void __launch_bounds__(kCgsBlock) k_cgs(const double* __restrict__ V, int64_t ld, int kk,
                                                   double* __restrict__ w, int64_t n,
                                                   const double* __restrict__ coef_in, double* __restrict__ partial) {
  constexpr int NW = kCgsBlock / 64;
  __shared__ double lds[(KMAX + 1) * NW];
  __shared__ double coef[KMAX];
  if (PASS >= 2) {
    for (int k = threadIdx.x; k < kk; k += kCgsBlock) coef[k] = coef_in[k];
    __syncthreads();
  }
  const int64_t i = (int64_t)blockIdx.x * kCgsBlock + threadIdx.x;
  const bool valid = i < n;
  // the basis columns stream past the caches (nontemporal), which keeps the
  // V-cycle's level-0 matrix resident in the last-level cache between steps
  double v[KMAX];
#pragma unroll
  for (int k = 0; k < KMAX; ++k) v[k] = (valid && k < kk) ? __builtin_nontemporal_load(V + (int64_t)k * ld + i) : 0.0;
  double wi = valid ? w[i] : 0.0;
  if (PASS >= 2) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < KMAX; ++k)
      if (k < kk) s += v[k] * coef[k];
    wi -= s;
    if (valid) w[i] = wi;
  }
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (PASS == 3) {
    const double t = sg_reduce<double, 64>(wi * wi);
    if (lane == 0) lds[wave] = t;
  } else {
    if (PASS == 5) {  // the squared norm of the updated w goes after the kk dots
      const double t2 = sg_reduce<double, 64>(wi * wi);
      if (lane == 0) lds[KMAX * NW + wave] = t2;
    }
#pragma unroll
    for (int k = 0; k < KMAX; ++k) v[k] *= wi;
    const double t = wave_reduce_scatter<KMAX>(v);
    constexpr int SHIFT = (KMAX == 64) ? 0 : (KMAX == 32) ? 1 : (KMAX == 16) ? 2 : 3;
    if ((lane & ((1 << SHIFT) - 1)) == 0) lds[(lane >> SHIFT) * NW + wave] = t;
  }
  __syncthreads();
  const int nk = (PASS == 3) ? 1 : kk;
  for (int k = threadIdx.x; k < nk; k += kCgsBlock) {
    double t = 0.0;
    for (int q = 0; q < NW; ++q) t += lds[k * NW + q];
    partial[(int64_t)k * gridDim.x + blockIdx.x] = t;
  }
  if (PASS == 5 && threadIdx.x == 0) {
    double t = 0.0;
    for (int q = 0; q < NW; ++q) t += lds[KMAX * NW + q];
    partial[(int64_t)kk * gridDim.x + blockIdx.x] = t;
  }
}

// Sum of the nb partials of ||w||^2, then Hessenberg column j = kk - 1 from
// h1 + h2 and ||w||, its Givens rotation and g (one workgroup, kk <= 64).
// The column and the previous rotations are staged in LDS by all threads, so
// the serial rotation sweep of thread 0 reads no global memory.
__global__ void __launch_bounds__(kBlock) k_cgs_finish(const double* __restrict__ partial, int nb, int kk,
                                                       const double* __restrict__ h1, const double* __restrict__ h2,
                                                       double* __restrict__ H, int ldh, double* __restrict__ cs,
                                                       double* __restrict__ sn, double* __restrict__ g,
                                                       double* __restrict__ res, double* __restrict__ res_host) {
  __shared__ double lds[kBlock / 64];
  __shared__ double col[65], cl[64], sl[64];
  const int j = kk - 1;
  for (int i = threadIdx.x; i <= j; i += kBlock) {
    col[i] = h1[i] + h2[i];
    if (i < j) {
      cl[i] = cs[i];
      sl[i] = sn[i];
    }
  }
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) acc += partial[b];
  const double hn2 = block_sum(acc, lds);  // its barriers also publish the staged column
  if (threadIdx.x == 0) {
    const double hn = sqrt(hn2);
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
      const double a = col[i], b = col[i + 1];
      col[i] = cl[i] * a + sl[i] * b;
      col[i + 1] = -sl[i] * a + cl[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double d = hypot(a, b);
    double c = 1.0, sv = 0.0;
    if (d != 0.0) {
      c = a / d;
      sv = b / d;
    }
    cs[j] = c;
    sn[j] = sv;
    col[j] = d;
    col[j + 1] = 0.0;
    const double gj = g[j];
    g[j + 1] = -sv * gj;
    g[j] = c * gj;
    // norm of the Hessenberg column (= ||A z_j|| in exact arithmetic; the
    // rotations keep it): the scale of the relative breakdown test
    double cn2 = 0.0;
    for (int i = 0; i <= j; ++i) cn2 += col[i] * col[i];
    res[0] = fabs(g[j + 1]);
    res[1] = hn;
    res[2] = hn > 0.0 ? 1.0 / hn : 0.0;
    res[3] = sqrt(cn2);
    if (res_host) {  // the host's copy (pinned memory), read after the step's event
      res_host[0] = res[0];
      res_host[1] = res[1];
      res_host[2] = res[2];
      res_host[3] = res[3];
    }
  }
  __syncthreads();
  double* hc = H + (int64_t)j * ldh;
  for (int i = threadIdx.x; i <= j + 1; i += kBlock) hc[i] = col[i];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_arnoldi_prep(const double* __restrict__ w,
                                                         const double* __restrict__ scale, double* __restrict__ vj,
                                                         T* __restrict__ b_out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double v;
  if (scale) {
    v = w[i] * scale[0];
    vj[i] = v;
  } else {
    v = vj[i];
  }
  b_out[i] = (T)v;
}

// ---- sliced blocked-ELL kernels ---------------------------------------------

// A blocked-ELL value, read once per launch.  FP64 values are always loaded
// nontemporally: they are 8/9 of an FP64 pass's bytes, and streaming them
// past the caches leaves the x-gathers and, in the mixed solve, a small FP32
// level-0 copy of K resident in the 256 MB last-level cache across the FP64
// operator applies.  FP32 values stream nontemporally too when the matrix
// cannot stay in that cache anyway (A.stream, set at upload); below that
// they load normally and are reused from it across the cycle's passes
// (nontemporal FP32 loads were 2 % slower on the 40^3 workload's 152 MB K,
// 4 % faster on the 100^3 workload's 2.3 GB).
template <typename T, bool NT>
__device__ __forceinline__ T bell_val(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}

// A bfloat16 value widened to FP32 (exact: the word's upper half).
template <bool NT>
__device__ __forceinline__ float bell_val16(const uint16_t* p) {
  uint32_t u;
  if constexpr (NT) u = __builtin_nontemporal_load(p);
  else u = *p;
  return __uint_as_float(u << 16);
}

// Block column of position p for lane `lane` of slice `slice`: a 16-bit
// delta from the lane's node (DEL) or the full index.
// base: the lane's node, or 0 for the lanes past the last node (their
// deltas are 0, so they gather x[0] like the padded full indices do).
template <typename T, bool DEL>
__device__ __forceinline__ int bell_col(const DBELL<T>& A, int64_t p, int base, int lane) {
  if constexpr (DEL) return base + (int)A.bdel[p * 64 + lane];
  else return A.bcol[p * 64 + lane];
}

// Row (node 64*slice + lane, component a) of a BELL matrix times x (x
// converted to T on load).  BS > 0 is the compile-time block size; BS == 0
// reads it at run time.  DEL: 16-bit column deltas; NT: nontemporal value
// loads; B16: bfloat16 values widened to FP32 (all three chosen per matrix
// outside the loop, so each loop has one kind of load).
template <typename T, typename XT, int BS, bool DEL, bool NT, bool B16>
__device__ __forceinline__ T bell_row_impl(const DBELL<T>& A, const XT* __restrict__ x, int slice, int lane, int a) {
  const int bs = BS > 0 ? BS : A.bs;
  const int p0 = A.slice_ptr[slice], p1 = A.slice_ptr[slice + 1];
  const int node = slice * 64 + lane;
  const int base = node < A.n_nodes ? node : 0;
  T acc = T(0);
#pragma unroll 2
  for (int p = p0; p < p1; ++p) {
    const int c = bell_col<T, DEL>(A, p, base, lane);
    const int64_t off = ((int64_t)p * (bs * bs) + a * bs) * 64 + lane;
    const XT* __restrict__ xc = x + (int64_t)c * bs;
    if constexpr (B16) {
      const uint16_t* __restrict__ v = A.val16 + off;
      if (BS > 0) {
#pragma unroll
        for (int b = 0; b < BS; ++b) acc += (T)bell_val16<NT>(v + b * 64) * (T)xc[b];
      } else {
        for (int b = 0; b < bs; ++b) acc += (T)bell_val16<NT>(v + b * 64) * (T)xc[b];
      }
    } else {
      const T* __restrict__ v = A.val + off;
      if (BS > 0) {
#pragma unroll
        for (int b = 0; b < BS; ++b) acc += bell_val<T, NT>(v + b * 64) * (T)xc[b];
      } else {
        for (int b = 0; b < bs; ++b) acc += bell_val<T, NT>(v + b * 64) * (T)xc[b];
      }
    }
  }
  return acc;
}

// The same row with symmetric storage: the blocks left of the diagonal read
// transposed from their mirror slots (column a of block (j, node) in lane
// j % 64 of j's slice), then the stored blocks on and right of it.  The
// lanes' blocks are visited in ascending column order, as in the full
// layout, so both give the same sums.  Every value loads normally: a pass
// reads each stored block a second time as a mirror block, a few thousand
// slices later, from the caches.  The mirror loop has no branch (a padded
// entry reads the lane's own first stored block and multiplies it by 0), so
// the loads of successive positions overlap.
template <typename T, typename XT, int BS, bool B16>
__device__ __forceinline__ T bell_row_sym(const DBELL<T>& A, const XT* __restrict__ x, int slice, int lane, int a) {
  const int bs = BS > 0 ? BS : A.bs;
  const int bb = bs * bs;
  const int p0 = A.slice_ptr[slice], p1 = A.slice_ptr[slice + 1];
  const int q0 = A.lptr[slice], q1 = A.lptr[slice + 1];
  const int node = slice * 64 + lane;
  const int base = node < A.n_nodes ? node : 0;
  T acc = T(0);
  // the index words of kChunk positions first (independent loads), then
  // their mirror blocks; positions past q1 act as padding
  constexpr int kChunk = 8;
  constexpr int kPad = (int)0x80000000u;
  for (int q = q0; q < q1; q += kChunk) {
    int wd[kChunk];
#pragma unroll
    for (int t = 0; t < kChunk; ++t) wd[t] = q + t < q1 ? A.lidx[(int64_t)(q + t) * 64 + lane] : kPad;
#pragma unroll
    for (int t = 0; t < kChunk; ++t) {
      const int rel = wd[t] >> 16;
      const bool ok = rel != -32768;
      const int j = ok ? base + (int)(int16_t)(wd[t] & 0xFFFF) : base;
      const T m = ok ? T(1) : T(0);
      const int64_t off = ((int64_t)(p0 + (ok ? rel : 0)) * bb + a) * 64 + (j & 63);
      const XT* __restrict__ xc = x + (int64_t)j * bs;
      if constexpr (B16) {
        const uint16_t* __restrict__ v = A.val16 + off;
        if (BS > 0) {
#pragma unroll
          for (int b = 0; b < BS; ++b) acc += ((T)bell_val16<false>(v + b * BS * 64) * m) * (T)xc[b];
        } else {
          for (int b = 0; b < bs; ++b) acc += ((T)bell_val16<false>(v + b * bs * 64) * m) * (T)xc[b];
        }
      } else {
        const T* __restrict__ v = A.val + off;
        if (BS > 0) {
#pragma unroll
          for (int b = 0; b < BS; ++b) acc += (bell_val<T, false>(v + b * BS * 64) * m) * (T)xc[b];
        } else {
          for (int b = 0; b < bs; ++b) acc += (bell_val<T, false>(v + b * bs * 64) * m) * (T)xc[b];
        }
      }
    }
  }
#pragma unroll 2
  for (int p = p0; p < p1; ++p) {
    const int c = base + (int)A.bdel[(int64_t)p * 64 + lane];
    const int64_t off = ((int64_t)p * bb + a * bs) * 64 + lane;
    const XT* __restrict__ xc = x + (int64_t)c * bs;
    if constexpr (B16) {
      const uint16_t* __restrict__ v = A.val16 + off;
      if (BS > 0) {
#pragma unroll
        for (int b = 0; b < BS; ++b) acc += (T)bell_val16<false>(v + b * 64) * (T)xc[b];
      } else {
        for (int b = 0; b < bs; ++b) acc += (T)bell_val16<false>(v + b * 64) * (T)xc[b];
      }
    } else {
      const T* __restrict__ v = A.val + off;
      if (BS > 0) {
#pragma unroll
        for (int b = 0; b < BS; ++b) acc += bell_val<T, false>(v + b * 64) * (T)xc[b];
      } else {
        for (int b = 0; b < bs; ++b) acc += bell_val<T, false>(v + b * 64) * (T)xc[b];
      }
    }
  }
  return acc;
}

// Symmetric storage, one node per lane: a thread accumulates all BS rows of
// its node, so a slice's x entries, index words and mirror blocks are loaded
// once instead of once per row wave.  Per row the same products in the same
// order as bell_row_sym.
template <typename T, typename XT, int BS, bool B16>
__device__ __forceinline__ void bell_node_sym_impl(const DBELL<T>& A, const XT* __restrict__ x, int slice, int lane,
                                                   T (&acc)[BS]) {
  constexpr int bb = BS * BS;
  const int p0 = A.slice_ptr[slice], p1 = A.slice_ptr[slice + 1];
  const int q0 = A.lptr[slice], q1 = A.lptr[slice + 1];
  const int node = slice * 64 + lane;
  const int base = node < A.n_nodes ? node : 0;
#pragma unroll
  for (int a = 0; a < BS; ++a) acc[a] = T(0);
  constexpr int kChunk = 4;
  constexpr int kPad = (int)0x80000000u;
  for (int q = q0; q < q1; q += kChunk) {
    int wd[kChunk];
#pragma unroll
    for (int t = 0; t < kChunk; ++t) wd[t] = q + t < q1 ? A.lidx[(int64_t)(q + t) * 64 + lane] : kPad;
#pragma unroll
    for (int t = 0; t < kChunk; ++t) {
      const int rel = wd[t] >> 16;
      const bool ok = rel != -32768;
      const int j = ok ? base + (int)(int16_t)(wd[t] & 0xFFFF) : base;
      const T m = ok ? T(1) : T(0);
      const int64_t off = (int64_t)(p0 + (ok ? rel : 0)) * bb * 64 + (j & 63);
      T xv[BS];
#pragma unroll
      for (int b = 0; b < BS; ++b) xv[b] = (T)x[(int64_t)j * BS + b];
#pragma unroll
      for (int a = 0; a < BS; ++a)
#pragma unroll
        for (int b = 0; b < BS; ++b) {
          T v;
          if constexpr (B16) v = (T)bell_val16<false>(A.val16 + off + (b * BS + a) * 64);
          else v = bell_val<T, false>(A.val + off + (b * BS + a) * 64);
          acc[a] += (v * m) * xv[b];
        }
    }
  }
#pragma unroll 2
  for (int p = p0; p < p1; ++p) {
    const int c = base + (int)A.bdel[(int64_t)p * 64 + lane];
    const int64_t off = (int64_t)p * bb * 64 + lane;
    T xv[BS];
#pragma unroll
    for (int b = 0; b < BS; ++b) xv[b] = (T)x[(int64_t)c * BS + b];
#pragma unroll
    for (int a = 0; a < BS; ++a)
#pragma unroll
      for (int b = 0; b < BS; ++b) {
        T v;
        if constexpr (B16) v = (T)bell_val16<false>(A.val16 + off + (a * BS + b) * 64);
        else v = bell_val<T, false>(A.val + off + (a * BS + b) * 64);
        acc[a] += v * xv[b];
      }
  }
}

template <typename T, typename XT, int BS>
__device__ __forceinline__ void bell_node_sym(const DBELL<T>& A, const XT* __restrict__ x, int slice, int lane,
                                              T (&acc)[BS]) {
  if constexpr (sizeof(T) == 4) {
    if (A.val16) return bell_node_sym_impl<T, XT, BS, true>(A, x, slice, lane, acc);
  }
  bell_node_sym_impl<T, XT, BS, false>(A, x, slice, lane, acc);
}

template <typename T, typename XT, int BS, bool B16>
__device__ __forceinline__ T bell_row_vals(const DBELL<T>& A, const XT* __restrict__ x, int slice, int lane, int a) {
  if (A.lptr) return bell_row_sym<T, XT, BS, B16>(A, x, slice, lane, a);
  if (A.bdel) {
    if (A.stream) return bell_row_impl<T, XT, BS, true, true, B16>(A, x, slice, lane, a);
    return bell_row_impl<T, XT, BS, true, false, B16>(A, x, slice, lane, a);
  }
  if (A.stream) return bell_row_impl<T, XT, BS, false, true, B16>(A, x, slice, lane, a);
  return bell_row_impl<T, XT, BS, false, false, B16>(A, x, slice, lane, a);
}

template <typename T, typename XT, int BS>
__device__ __forceinline__ T bell_row_any(const DBELL<T>& A, const XT* __restrict__ x, int slice, int lane, int a) {
  if constexpr (sizeof(T) == 4) {
    if (A.val16) return bell_row_vals<T, XT, BS, true>(A, x, slice, lane, a);
  }
  return bell_row_vals<T, XT, BS, false>(A, x, slice, lane, a);
}

template <typename T, int BS>
__device__ __forceinline__ T bell_row(const DBELL<T>& A, const T* __restrict__ x, int slice, int lane, int a) {
  return bell_row_any<T, T, BS>(A, x, slice, lane, a);
}

// XCD-aware slice order for the blocked-ELL kernels: the dispatcher hands
// consecutive workgroups to the 8 XCDs in turn, so workgroup g runs on XCD
// g % 8.  Mapping g to slice start(g % 8) + g / 8 gives each XCD one
// contiguous range of slices (nodes), and the x-gathers of neighbouring
// slices hit that XCD's own L2 instead of being fetched once per XCD.  A
// bijection on [0, n): XCD x owns n / 8 slices, plus one when x < n % 8.
__device__ __forceinline__ int xcd_slice(int g, int n) {
  constexpr int kXcd = 8;
  const int x = g % kXcd, q = n / kXcd, rem = n % kXcd;
  return x * q + min(x, rem) + g / kXcd;
}

// Row of a BELL matrix times a vector of another precision (converted on
// load).
template <typename T, typename XT, int BS>
__device__ __forceinline__ T bell_row_x(const DBELL<T>& A, const XT* __restrict__ x, int slice, int lane, int a) {
  return bell_row_any<T, XT, BS>(A, x, slice, lane, a);
}

// Block operator apply with x of type XT (x1 = x, x2 = x + n1).  When xcopy
// is given, every row also stores its own x entry there in T (a widened
// copy of x made in the same pass).
template <typename T, typename XT, int BS, int MODE>
__global__ void k_blk_spmv_bell(DBELL<T> K, DCSR<T> A12, DCSR<T> A21, DCSR<T> A22, const XT* __restrict__ x1,
                                const XT* __restrict__ x2, const T* __restrict__ b1, const T* __restrict__ b2,
                                T* __restrict__ y1, T* __restrict__ y2, int n1, int n2, T* __restrict__ xcopy) {
  const int bs = BS > 0 ? BS : K.bs;
  if ((int)blockIdx.x < K.n_slices) {
    const int lane = threadIdx.x & 63, a = threadIdx.x >> 6;
    const int slice = xcd_slice((int)blockIdx.x, K.n_slices);
    T s = bell_row_x<T, XT, BS>(K, x1, slice, lane, a);
    const int node = slice * 64 + lane;
    if (node >= K.n_nodes) return;
    const int row = node * bs + a;
    if (A12.nnz) s += csr_row_serial_x<T, XT>(A12, x2, row);
    if (MODE == 0) y1[row] = s;
    else if (MODE == 1) y1[row] = b1[row] - s;
    else y1[row] += s;
    if (xcopy) xcopy[row] = (T)x1[row];
  } else {
    const int j = ((int)blockIdx.x - K.n_slices) * (int)blockDim.x + threadIdx.x;
    if (j >= n2) return;
    T s = T(0);
    if (A21.nnz) s = csr_row_serial_x<T, XT>(A21, x1, j);
    if (A22.nnz) s += csr_row_serial_x<T, XT>(A22, x2, j);
    if (MODE == 0) y2[j] = s;
    else if (MODE == 1) y2[j] = b2[j] - s;
    else y2[j] += s;
    if (xcopy) xcopy[n1 + j] = (T)x2[j];
  }
}

template <typename T, int BS>
__global__ void k_smooth_u_bell(DBELL<T> K, DCSR<T> G, const T* __restrict__ zu, const T* __restrict__ zl,
                                const T* __restrict__ bu, const T* __restrict__ jinv, T omega, T* __restrict__ znu,
                                T* __restrict__ r_out, T* __restrict__ w_out) {
  const int bs = BS > 0 ? BS : K.bs;
  const int lane = threadIdx.x & 63, a = threadIdx.x >> 6;
  const int slice = xcd_slice((int)blockIdx.x, (int)gridDim.x);
  T s = bell_row<T, BS>(K, zu, slice, lane, a);
  const int node = slice * 64 + lane;
  if (node >= K.n_nodes) return;
  const int row = node * bs + a;
  if (G.nnz) s += csr_row_serial<T>(G, zl, row);
  const T r = bu[row] - s;
  const T w = omega * jinv[row] * r;
  znu[row] = zu[row] + w;
  if (r_out) {
    r_out[row] = r;
    w_out[row] = w;
  }
}

template <typename T, int BS>
__global__ void k_tsmooth_u_bell(DBELL<T> KT, DCSR<T> BT, const T* __restrict__ zu, const T* __restrict__ zl,
                                 const T* __restrict__ bu, T* __restrict__ su) {
  const int bs = BS > 0 ? BS : KT.bs;
  const int lane = threadIdx.x & 63, a = threadIdx.x >> 6;
  const int slice = xcd_slice((int)blockIdx.x, (int)gridDim.x);
  T s = bell_row<T, BS>(KT, zu, slice, lane, a);
  const int node = slice * 64 + lane;
  if (node >= KT.n_nodes) return;
  const int row = node * bs + a;
  if (BT.nnz) s += csr_row_serial<T>(BT, zl, row);
  su[row] = bu[row] - s;
}

// Node-per-lane forms of the three hot blocked-ELL kernels for symmetric
// storage with 3x3 blocks (the fine level): 256 threads = 4 slices per
// workgroup, the groups of 4 slices in the XCD-contiguous order.  With the
// layout's loads through the caches (not memory) the limit, one thread per
// node loads each x entry, index word and mirror block once where a wave
// per block row loads them three times: 7-8 % faster passes than the
// row-wave form on the 100^3 workload.  A view selects them with `stream`
// (set for large levels: a third of the waves must still fill the chip).
constexpr int kNplBlock = 256;

template <typename T, typename XT, int BS, int MODE>
__global__ void __launch_bounds__(kNplBlock) k_blk_spmv_bell_npl(DBELL<T> K, DCSR<T> A12, DCSR<T> A21, DCSR<T> A22,
                                                                 const XT* __restrict__ x1, const XT* __restrict__ x2,
                                                                 const T* __restrict__ b1, const T* __restrict__ b2,
                                                                 T* __restrict__ y1, T* __restrict__ y2, int n1, int n2,
                                                                 T* __restrict__ xcopy) {
  const int ng = (K.n_slices + 3) / 4;
  if ((int)blockIdx.x < ng) {
    const int lane = threadIdx.x & 63;
    const int slice = xcd_slice((int)blockIdx.x, ng) * 4 + (int)(threadIdx.x >> 6);
    if (slice >= K.n_slices) return;
    T acc[BS];
    bell_node_sym<T, XT, BS>(K, x1, slice, lane, acc);
    const int node = slice * 64 + lane;
    if (node >= K.n_nodes) return;
#pragma unroll
    for (int a = 0; a < BS; ++a) {
      const int row = node * BS + a;
      T s = acc[a];
      if (A12.nnz) s += csr_row_serial_x<T, XT>(A12, x2, row);
      if (MODE == 0) y1[row] = s;
      else if (MODE == 1) y1[row] = b1[row] - s;
      else y1[row] += s;
      if (xcopy) xcopy[row] = (T)x1[row];
    }
  } else {
    const int j = ((int)blockIdx.x - ng) * kNplBlock + threadIdx.x;
    if (j >= n2) return;
    T s = T(0);
    if (A21.nnz) s = csr_row_serial_x<T, XT>(A21, x1, j);
    if (A22.nnz) s += csr_row_serial_x<T, XT>(A22, x2, j);
    if (MODE == 0) y2[j] = s;
    else if (MODE == 1) y2[j] = b2[j] - s;
    else y2[j] += s;
    if (xcopy) xcopy[n1 + j] = (T)x2[j];
  }
}

template <typename T, int BS>
__global__ void __launch_bounds__(kNplBlock) k_smooth_u_bell_npl(DBELL<T> K, DCSR<T> G, const T* __restrict__ zu,
                                                                 const T* __restrict__ zl, const T* __restrict__ bu,
                                                                 const T* __restrict__ jinv, T omega,
                                                                 T* __restrict__ znu, T* __restrict__ r_out,
                                                                 T* __restrict__ w_out) {
  const int ng = (K.n_slices + 3) / 4;
  const int lane = threadIdx.x & 63;
  const int slice = xcd_slice((int)blockIdx.x, ng) * 4 + (int)(threadIdx.x >> 6);
  if (slice >= K.n_slices) return;
  T acc[BS];
  bell_node_sym<T, T, BS>(K, zu, slice, lane, acc);
  const int node = slice * 64 + lane;
  if (node >= K.n_nodes) return;
#pragma unroll
  for (int a = 0; a < BS; ++a) {
    const int row = node * BS + a;
    T s = acc[a];
    if (G.nnz) s += csr_row_serial<T>(G, zl, row);
    const T r = bu[row] - s;
    const T w = omega * jinv[row] * r;
    znu[row] = zu[row] + w;
    if (r_out) {
      r_out[row] = r;
      w_out[row] = w;
    }
  }
}

template <typename T, int BS>
__global__ void __launch_bounds__(kNplBlock) k_tsmooth_u_bell_npl(DBELL<T> KT, DCSR<T> BT, const T* __restrict__ zu,
                                                                  const T* __restrict__ zl, const T* __restrict__ bu,
                                                                  T* __restrict__ su) {
  const int ng = (KT.n_slices + 3) / 4;
  const int lane = threadIdx.x & 63;
  const int slice = xcd_slice((int)blockIdx.x, ng) * 4 + (int)(threadIdx.x >> 6);
  if (slice >= KT.n_slices) return;
  T acc[BS];
  bell_node_sym<T, T, BS>(KT, zu, slice, lane, acc);
  const int node = slice * 64 + lane;
  if (node >= KT.n_nodes) return;
#pragma unroll
  for (int a = 0; a < BS; ++a) {
    const int row = node * BS + a;
    T s = acc[a];
    if (BT.nnz) s += csr_row_serial<T>(BT, zl, row);
    su[row] = bu[row] - s;
  }
}

template <typename T, int BS>
__global__ void k_jacobi_extra_bell(DBELL<T> M, const T* __restrict__ w, const T* __restrict__ r,
                                    const T* __restrict__ jinv, T omega, T* __restrict__ w_out,
                                    const T* __restrict__ zu, T* __restrict__ znu, int last) {
  const int bs = BS > 0 ? BS : M.bs;
  const int lane = threadIdx.x & 63, a = threadIdx.x >> 6;
  const int slice = xcd_slice((int)blockIdx.x, (int)gridDim.x);
  T s = bell_row<T, BS>(M, w, slice, lane, a);
  const int node = slice * 64 + lane;
  if (node >= M.n_nodes) return;
  const int row = node * bs + a;
  const T wn = w[row] + omega * jinv[row] * (r[row] - s);
  w_out[row] = wn;
  if (last) znu[row] = (zu ? zu[row] : T(0)) + wn;
}

// Nodal lumping option, level-0 layout: residual and block Jacobi prediction
// in one pass.  The BS rows of a node sit in the BS waves of the workgroup
// (lane = node in the slice, wave = row in the node); their residuals meet in
// LDS and each row applies its row of the node's inverse lumping block M:
//   t = b_u - K z_u - G z_l,  w = omega M t,  zn_u = z_u + w,
// t_out / w_out optional.
template <typename T, int BS>
__global__ void k_smooth_u_bell_nodal(DBELL<T> K, DCSR<T> G, const T* __restrict__ zu, const T* __restrict__ zl,
                                      const T* __restrict__ bu, const T* __restrict__ M, T omega,
                                      T* __restrict__ znu, T* __restrict__ t_out, T* __restrict__ w_out) {
  __shared__ T tl[BS][64];
  const int lane = threadIdx.x & 63, a = threadIdx.x >> 6;
  const int slice = xcd_slice((int)blockIdx.x, (int)gridDim.x);
  T s = bell_row<T, BS>(K, zu, slice, lane, a);
  const int node = slice * 64 + lane;
  const bool live = node < K.n_nodes;
  const int row = node * BS + a;
  T t = T(0);
  if (live) {
    if (G.nnz) s += csr_row_serial<T>(G, zl, row);
    t = bu[row] - s;
  }
  tl[a][lane] = t;
  __syncthreads();
  if (!live) return;
  const T* Mn = M + (size_t)node * (BS * BS) + a * BS;
  T acc = T(0);
#pragma unroll
  for (int b = 0; b < BS; ++b) acc += Mn[b] * tl[b][lane];
  const T w = omega * acc;
  znu[row] = zu[row] + w;
  if (t_out) t_out[row] = t;
  if (w_out) w_out[row] = w;
}

// Nodal lumping option: back-substitution on the listed (interface) nodes,
// zn_u += scale * M (G delta) per node.  One wave per node: row b of the node
// takes lanes [b SGB, (b+1) SGB) for its G row dot (the interface rows are
// short and their loads chain, so they are spread over lanes), then lanes
// a < BS apply row a of M to the node's BS dots.
template <typename T, int BS>
__global__ void __launch_bounds__(kBlock) k_node_correct(DCSR<T> G, const int32_t* __restrict__ nodes, int n_list,
                                                         const T* __restrict__ delta, const T* __restrict__ M,
                                                         T scale, T* __restrict__ znu) {
  constexpr int SGB = BS <= 2 ? 32 : (BS <= 4 ? 16 : 8);
  static_assert(BS * SGB <= 64, "one wave per node");
  const int wave = (int)((blockIdx.x * kBlock + threadIdx.x) >> 6);
  const int lane = threadIdx.x & 63;
  if (wave >= n_list) return;  // uniform across the wave
  const int nd = nodes[wave];
  const int b = lane / SGB, sl = lane % SGB;
  T g = T(0);
  if (b < BS) {
    const int row = nd * BS + b;
    const int e = G.rp[row + 1];
    for (int k = G.rp[row] + sl; k < e; k += SGB) g += G.v[k] * delta[G.ci[k]];
  }
  g = sg_reduce<T, SGB>(g);
  T gb[BS];
#pragma unroll
  for (int q = 0; q < BS; ++q) gb[q] = __shfl(g, q * SGB, 64);
  if (lane < BS) {
    const T* Mn = M + (size_t)nd * (BS * BS) + lane * BS;
    T acc = T(0);
#pragma unroll
    for (int q = 0; q < BS; ++q) acc += Mn[q] * gb[q];
    znu[(size_t)nd * BS + lane] += scale * acc;
  }
}

// Nodal lumping option, adjoint update per node:
//   t = s_u - a B^T delta,  w = omega M^T t,  zn_u = z_u + c w   (z_u null: zero)
// t_out / w_out optional (extra Jacobi sweeps).
template <typename T, int BS>
__global__ void __launch_bounds__(kBlock) k_tcorrect_nodal(DCSR<T> BT, const T* __restrict__ su,
                                                           const T* __restrict__ delta, const T* __restrict__ M,
                                                           T omega, T a_bt, T c_w, const T* __restrict__ zu,
                                                           T* __restrict__ znu, T* __restrict__ t_out,
                                                           T* __restrict__ w_out, int n_nodes) {
  const int nd = blockIdx.x * kBlock + threadIdx.x;
  if (nd >= n_nodes) return;
  T t[BS];
#pragma unroll
  for (int b = 0; b < BS; ++b) {
    const int row = nd * BS + b;
    t[b] = su[row];
    if (BT.nnz) t[b] -= a_bt * csr_row_serial<T>(BT, delta, row);
  }
  const T* Mn = M + (size_t)nd * (BS * BS);
#pragma unroll
  for (int a = 0; a < BS; ++a) {
    T acc = T(0);
#pragma unroll
    for (int b = 0; b < BS; ++b) acc += Mn[b * BS + a] * t[b];
    const T w = omega * acc;
    const size_t row = (size_t)nd * BS + a;
    znu[row] = (zu ? zu[row] : T(0)) + c_w * w;
    if (t_out) t_out[row] = t[a];
    if (w_out) w_out[row] = w;
  }
}

// Aggregation transfers with the tentative pattern (plain aggregation): fine
// row i holds exactly its aggregate's NS coarse columns base[i] ..
// base[i] + NS - 1 (base -1: a zeroed row), its values dense per row, so no
// column indices are stored.  Prolongation y += P x, one thread per fine row
// (displacement rows, then multiplier rows).
template <typename T, int NSU, int NSL>
__global__ void __launch_bounds__(kBlock) k_prolong_agg(const int32_t* __restrict__ base_u, const T* __restrict__ pu,
                                                        const int32_t* __restrict__ base_l, const T* __restrict__ pl,
                                                        const T* __restrict__ xu, const T* __restrict__ xl,
                                                        T* __restrict__ yu, T* __restrict__ yl, int nu, int nl) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i < nu) {
    const int c = base_u[i];
    if (c < 0) return;
    T s = T(0);
#pragma unroll
    for (int k = 0; k < NSU; ++k) s += pu[(size_t)i * NSU + k] * xu[c + k];
    yu[i] += s;
  } else if (i < nu + nl) {
    const int j = i - nu;
    const int c = base_l[j];
    if (c < 0) return;
    T s = T(0);
#pragma unroll
    for (int k = 0; k < NSL; ++k) s += pl[(size_t)j * NSL + k] * xl[c + k];
    yl[j] += s;
  }
}

// Restriction y = P^T r with the same storage, one SG-lane subgroup per
// aggregate: its fine rows (ascending, from the aggregate's row list) are
// read once and the NS coarse sums accumulate together.
template <typename T, int NS, int SG>
__device__ __forceinline__ void restrict_one(const int32_t* __restrict__ ptr, const int32_t* __restrict__ rows,
                                             const T* __restrict__ pv, const T* __restrict__ r, T* __restrict__ y,
                                             int a, int lane) {
  T acc[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) acc[k] = T(0);
  const int e = ptr[a + 1];
  for (int p = ptr[a] + lane; p < e; p += SG) {
    const int i = rows[p];
    const T ri = r[i];
#pragma unroll
    for (int k = 0; k < NS; ++k) acc[k] += pv[(size_t)i * NS + k] * ri;
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const T t = sg_reduce<T, SG>(acc[k]);
    if (lane == k) y[(size_t)a * NS + k] = t;
  }
}

template <typename T, int NSU, int NSL, int SG>
__global__ void __launch_bounds__(kBlock) k_restrict_agg(const int32_t* __restrict__ ptr_u,
                                                         const int32_t* __restrict__ rows_u, const T* __restrict__ pu,
                                                         const int32_t* __restrict__ ptr_l,
                                                         const int32_t* __restrict__ rows_l, const T* __restrict__ pl,
                                                         const T* __restrict__ ru, const T* __restrict__ rl,
                                                         T* __restrict__ yu, T* __restrict__ yl, int n_agg_u,
                                                         int n_agg_l) {
  static_assert(NSU <= SG && NSL <= SG, "one lane per coarse row of an aggregate");
  const int a = blockIdx.x * (kBlock / SG) + threadIdx.x / SG;
  const int lane = threadIdx.x % SG;
  if (a < n_agg_u)
    restrict_one<T, NSU, SG>(ptr_u, rows_u, pu, ru, yu, a, lane);
  else if (a < n_agg_u + n_agg_l)
    restrict_one<T, NSL, SG>(ptr_l, rows_l, pl, rl, yl, a - n_agg_u, lane);
}

// ---- Krylov -----------------------------------------------------------------

constexpr int kDotGroup = 8;


__global__ void __launch_bounds__(kBlock) k_mdot_partial(const double* __restrict__ V, int64_t ld, int kk,
                                                         const double* __restrict__ w, int64_t n, int64_t chunk,
                                                         double* __restrict__ partial, int nb) {
  __shared__ double lds[kBlock / 64];
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = min(n, beg + chunk);
  for (int k0 = 0; k0 < kk; k0 += kDotGroup) {
    double acc[kDotGroup];
#pragma unroll
    for (int q = 0; q < kDotGroup; ++q) acc[q] = 0.0;
    for (int64_t i = beg + threadIdx.x; i < end; i += kBlock) {
      const double wi = w[i];
#pragma unroll
      for (int q = 0; q < kDotGroup; ++q)
        if (k0 + q < kk) acc[q] += V[(int64_t)(k0 + q) * ld + i] * wi;
    }
#pragma unroll
    for (int q = 0; q < kDotGroup; ++q) {
      if (k0 + q < kk) {
        const double t = block_sum(acc[q], lds);
        if (threadIdx.x == 0) partial[(int64_t)(k0 + q) * nb + blockIdx.x] = t;
      }
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_mdot_reduce(const double* __restrict__ partial, int nb,
                                                        double* __restrict__ h) {
  // fixed order: thread t adds entries t, t + 256, ... ; then a fixed tree
  __shared__ double lds[kBlock / 64];
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) acc += partial[(int64_t)k * nb + b];
  const double t = block_sum(acc, lds);
  if (threadIdx.x == 0) h[k] = t;
}

// Second projection of CGS2 from the Gram matrix of the basis (two-pass
// variant): column j of G = V^T V arrives as the previous step's dots of V
// with the updated w, times 1/||w|| (its diagonal entry is 1); then
// h2 = h1 - G h1 -- what a second pass over V would measure, up to rounding
// of the first update -- and c = h1 + h2, the update's coefficients.
// G is KMAX x KMAX column-major (kk <= 64), one workgroup.
__global__ void __launch_bounds__(256) k_gram_step(double* __restrict__ G, int j, const double* __restrict__ gprev,
                                                   const double* __restrict__ scale, const double* __restrict__ h1,
                                                   double* __restrict__ h2, double* __restrict__ c) {
  constexpr int L = 64, P = 4;  // 4 partial sums per row k, over q in [16 p, 16 p + 16)
  __shared__ double hs[L];
  __shared__ double part[P][L];
  const int k = threadIdx.x % L, p = threadIdx.x / L;
  if (p == 0) {
    if (k < j) {
      const double gk = gprev[k] * scale[0];
      G[(int64_t)j * L + k] = gk;
      G[(int64_t)k * L + j] = gk;
    }
    if (k == j) G[(int64_t)j * L + j] = 1.0;
    hs[k] = k <= j ? h1[k] : 0.0;
  }
  __syncthreads();
  double t = 0.0;
  if (k <= j) {
#pragma unroll
    for (int u = 0; u < L / P; ++u) {
      const int q = p * (L / P) + u;
      if (q <= j) t += G[(int64_t)q * L + k] * hs[q];
    }
  }
  part[p][k] = t;
  __syncthreads();
  if (p == 0 && k <= j) {
    const double gh = (part[0][k] + part[1][k]) + (part[2][k] + part[3][k]);
    const double d = hs[k] - gh;
    h2[k] = d;
    c[k] = hs[k] + d;
  }
}

__global__ void __launch_bounds__(kBlock) k_gemv_acc(const double* __restrict__ M, int64_t ld, int kk,
                                                     const double* __restrict__ c, double sign,
                                                     double* __restrict__ y, int64_t n) {
  __shared__ double cs[512];
  for (int k = threadIdx.x; k < kk; k += kBlock) cs[k] = c[k];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < kk; ++k) s += M[(int64_t)k * ld + i] * cs[k];
  y[i] += sign * s;
}

__global__ void k_arnoldi_update(double* __restrict__ H, int ldh, double* __restrict__ cs, double* __restrict__ sn,
                                 double* __restrict__ g, const double* __restrict__ h1,
                                 const double* __restrict__ h2, const double* __restrict__ hn2, int j,
                                 double* __restrict__ out, double* __restrict__ out_host) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double* col = H + (int64_t)j * ldh;
  for (int i = 0; i <= j; ++i) col[i] = h1[i] + h2[i];
  const double hn = sqrt(hn2[0]);
  col[j + 1] = hn;
  for (int i = 0; i < j; ++i) {
    const double a = col[i], b = col[i + 1];
    col[i] = cs[i] * a + sn[i] * b;
    col[i + 1] = -sn[i] * a + cs[i] * b;
  }
  const double a = col[j], b = col[j + 1];
  const double d = hypot(a, b);
  double c = 1.0, s = 0.0;
  if (d != 0.0) {
    c = a / d;
    s = b / d;
  }
  cs[j] = c;
  sn[j] = s;
  col[j] = d;
  col[j + 1] = 0.0;
  g[j + 1] = -s * g[j];
  g[j] = c * g[j];
  double cn2 = 0.0;
  for (int i = 0; i <= j; ++i) cn2 += col[i] * col[i];
  out[0] = fabs(g[j + 1]);
  out[1] = hn;
  out[2] = hn > 0.0 ? 1.0 / hn : 0.0;
  out[3] = sqrt(cn2);
  if (out_host) {
    out_host[0] = out[0];
    out_host[1] = out[1];
    out_host[2] = out[2];
    out_host[3] = out[3];
  }
}

__global__ void __launch_bounds__(kBlock) k_restart_init(const double* __restrict__ r,
                                                         const double* __restrict__ beta2, double* __restrict__ V0,
                                                         double* __restrict__ g, int gl, double* __restrict__ out,
                                                         int64_t n) {
  const double beta = sqrt(beta2[0]);
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < n) V0[i] = r[i] * inv;
  if (i < gl) g[i] = (i == 0) ? beta : 0.0;
  if (i == 0) out[0] = beta;
}

__global__ void k_hess_solve(const double* __restrict__ H, int ldh, const double* __restrict__ g,
                             double* __restrict__ y, int k) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int l = i + 1; l < k; ++l) s -= H[(int64_t)l * ldh + i] * y[l];
    y[i] = s / H[(int64_t)i * ldh + i];
  }
}

// SG lanes per row, so the column reads and gradient writes of a row are
// contiguous across the subgroup.
template <int SG>
__global__ void __launch_bounds__(kBlock) k_grad_K(DCSR<double> K, const double* __restrict__ lam,
                                                   const double* __restrict__ x, double* __restrict__ dK) {
  const int i = blockIdx.x * (kBlock / SG) + threadIdx.x / SG;
  const int lane = threadIdx.x % SG;
  if (i >= K.nrows) return;
  const double li = lam[i];
  const int e = K.rp[i + 1];
  for (int k = K.rp[i] + lane; k < e; k += SG) dK[k] = -li * x[K.ci[k]];
}

template <typename T>
__global__ void k_scatter_perm(const double* __restrict__ src, const int32_t* __restrict__ perm, T* __restrict__ dst,
                               int64_t nnz) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < nnz) dst[perm[e]] = (T)src[e];
}

__global__ void k_scatter_pos64(const double* __restrict__ src, const int64_t* __restrict__ pos,
                                double* __restrict__ dst, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e >= n) return;
  const int64_t p = pos[e];
  if (p >= 0) dst[p] = src[e];
}

// flag = 1 if some entry differs from its transpose partner (perm: entry ->
// position of the mirrored entry in the same, symmetric, pattern)
__global__ void k_check_symmetric(const double* __restrict__ v, const int32_t* __restrict__ perm, int64_t n,
                                  int32_t* __restrict__ flag) {
  const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (e < n && !(v[e] == v[perm[e]])) *flag = 1;
}

inline unsigned grid_for(int64_t rows, int rows_per_block) {
  return (unsigned)((rows + rows_per_block - 1) / rows_per_block);
}

}  // namespace

// Lanes per row from the mean row length (measured on the contact
// hierarchies: long coarse rows prefer many lanes for parallel gathers;
// rows of at most 8 entries, e.g. tentative prolongators, one thread each).
// Measured on the 40^3 workload's hierarchy: with the unrolled row loop,
// 16 lanes per row beat 32 and 64 even for rows of 80-160 entries (more
// rows in flight per wave hide the gather latency better).
int pick_subgroup(int64_t nnz, int64_t nrows) {
  const double avg = nrows ? (double)nnz / (double)nrows : 0.0;
  if (avg > 14.0) return 16;
  if (avg > 8.0) return 8;
  return 1;
}

#define CAMG_SG_DISPATCH(sg, ...) \
  switch (sg) {                           \
    case 1: {                             \
      constexpr int SG = 1;               \
      __VA_ARGS__;                        \
    } break;                              \
    case 2: {                             \
      constexpr int SG = 2;               \
      __VA_ARGS__;                        \
    } break;                              \
    case 4: {                             \
      constexpr int SG = 4;               \
      __VA_ARGS__;                        \
    } break;                              \
    case 8: {                             \
      constexpr int SG = 8;               \
      __VA_ARGS__;                        \
    } break;                              \
    case 16: {                            \
      constexpr int SG = 16;              \
      __VA_ARGS__;                        \
    } break;                              \
    case 32: {                            \
      constexpr int SG = 32;              \
      __VA_ARGS__;                        \
    } break;                              \
    default: {                            \
      constexpr int SG = 64;              \
      __VA_ARGS__;                        \
    } break;                              \
  }

template <typename T>
void blk_spmv(const DCSR<T>& A11, const DCSR<T>& A12, const DCSR<T>& A21, const DCSR<T>& A22, const T* x1,
              const T* x2, const T* b1, const T* b2, T* y1, T* y2, int n1, int n2, int mode, int sg,
              hipStream_t s) {
  const int n = n1 + n2;
  if (n <= 0) return;
  CAMG_SG_DISPATCH(sg, {
    dim3 grid(grid_for(n, kBlock / SG));
    if (mode == 0)
      k_blk_spmv<T, SG, 0><<<grid, kBlock, 0, s>>>(A11, A12, A21, A22, x1, x2, b1, b2, y1, y2, n1, n);
    else if (mode == 1)
      k_blk_spmv<T, SG, 1><<<grid, kBlock, 0, s>>>(A11, A12, A21, A22, x1, x2, b1, b2, y1, y2, n1, n);
    else
      k_blk_spmv<T, SG, 2><<<grid, kBlock, 0, s>>>(A11, A12, A21, A22, x1, x2, b1, b2, y1, y2, n1, n);
  });
  CAMG_LAUNCHED();
}

template <typename T>
void smooth_u(const DCSR<T>& K, const DCSR<T>& G, const T* zu, const T* zl, const T* bu, const T* jinv, T omega,
              T* znu, T* r_out, T* w_out, int n_u, bool first, int sg, hipStream_t s) {
  if (n_u <= 0) return;
  if (first) {
    k_smooth_u_first<T><<<grid_for(n_u, kBlock), kBlock, 0, s>>>(bu, jinv, omega, znu, r_out, w_out, n_u);
  } else {
    CAMG_SG_DISPATCH(sg, {
      k_smooth_u<T, SG><<<grid_for(n_u, kBlock / SG), kBlock, 0, s>>>(K, G, zu, zl, bu, jinv, omega, znu, r_out,
                                                                      w_out, n_u);
    });
  }
  CAMG_LAUNCHED();
}

template <typename T>
void jacobi_extra(const DCSR<T>& M, const T* w, const T* r, const T* jinv, T omega, T* w_out, const T* zu, T* znu,
                  bool last, int n_u, int sg, hipStream_t s) {
  if (n_u <= 0) return;
  CAMG_SG_DISPATCH(sg, {
    k_jacobi_extra<T, SG><<<grid_for(n_u, kBlock / SG), kBlock, 0, s>>>(M, w, r, jinv, omega, w_out, zu, znu,
                                                                         last ? 1 : 0, n_u);
  });
  CAMG_LAUNCHED();
}

// Lanes per row of the multiplier-row kernels: the mean row length rule,
// at least 4.
static int rows_sg(int64_t nnz, int64_t rows) { return std::max(4, pick_subgroup(nnz, rows)); }

template <typename T>
void smooth_l(const DCSR<T>& B, const DCSR<T>& C, const T* znu, const T* zl, const T* bl, const T* sdinv, T alpha,
              T* znl, T* delta, T* rhs_out, int n_l, bool first, hipStream_t s) {
  if (n_l <= 0) return;
  CAMG_SG_DISPATCH(rows_sg(B.nnz + C.nnz, n_l), {
    dim3 grid(grid_for(n_l, kBlock / SG));
    if (first)
      k_smooth_l<T, SG, true><<<grid, kBlock, 0, s>>>(B, C, znu, zl, bl, sdinv, alpha, znl, delta, rhs_out, n_l);
    else
      k_smooth_l<T, SG, false><<<grid, kBlock, 0, s>>>(B, C, znu, zl, bl, sdinv, alpha, znl, delta, rhs_out, n_l);
  });
  CAMG_LAUNCHED();
}

template <typename T>
T* schur_steps(const DCSR<T>& S, const T* q, T* d_a, T* d_b, const T* sdinv, const T* zl, T alpha, T* znl,
               int steps, int n_l, int sg, hipStream_t s) {
  if (n_l <= 0 || steps <= 0) return d_a;
  for (int k = 0; k < steps; ++k) {
    const int last = (k == steps - 1) ? 1 : 0;
    CAMG_SG_DISPATCH(sg, {
      k_schur_jacobi<T, SG><<<grid_for(n_l, kBlock / SG), kBlock, 0, s>>>(S, q, d_a, sdinv, d_b, zl, alpha, znl,
                                                                           last, n_l);
    });
    CAMG_LAUNCHED();
    std::swap(d_a, d_b);
  }
  return d_a;
}

template <typename T>
T* schur_block_steps(const DCSR<T>& S, const T* q, T* d_a, T* d_b, const T* blk, bool trans, const T* zl, T alpha,
                     T* znl, int steps, int n_l, int bs, hipStream_t s) {
  if (n_l <= 0 || steps <= 0) return d_a;
  if (bs < 1 || bs > 3 || n_l % bs) throw std::runtime_error("block Schur step: node block size must be 1..3");
  const int nn = n_l / bs;
  const T* din = nullptr;
  T* dout = d_a;
  for (int k = 0; k < steps; ++k) {
    const int last = (k == steps - 1) ? 1 : 0;
    const unsigned g = grid_for(nn, kBlock);
#define CAMG_SCHUR_BLOCK_LAUNCH(BSV)                                                                          \
  if (trans)                                                                                                  \
    k_schur_block<T, BSV, true><<<g, kBlock, 0, s>>>(S, q, din, blk, dout, zl, alpha, znl, last, nn);          \
  else                                                                                                        \
    k_schur_block<T, BSV, false><<<g, kBlock, 0, s>>>(S, q, din, blk, dout, zl, alpha, znl, last, nn);
    if (bs == 3) {
      CAMG_SCHUR_BLOCK_LAUNCH(3)
    } else if (bs == 2) {
      CAMG_SCHUR_BLOCK_LAUNCH(2)
    } else {
      CAMG_SCHUR_BLOCK_LAUNCH(1)
    }
#undef CAMG_SCHUR_BLOCK_LAUNCH
    CAMG_LAUNCHED();
    din = dout;
    dout = (dout == d_a) ? d_b : d_a;
  }
  return const_cast<T*>(din);
}

template <typename T>
void node_apply(const T* M, const T* x, T scale, const T* y_in, T* y_out, T* w_out, int n, int bs, bool trans,
                hipStream_t s, const int32_t* list, int n_list) {
  if (n <= 0) return;
  if (bs < 1 || bs > 6 || n % bs) throw std::runtime_error("node_apply: node block size must be 1..6 and divide n");
  const int nn = list ? n_list : n / bs;
  if (nn <= 0) return;
  const unsigned g = grid_for(nn, kBlock);
#define CAMG_NODE_APPLY_LAUNCH(BSV)                                                                     \
  if (trans)                                                                                            \
    k_node_apply<T, BSV, true><<<g, kBlock, 0, s>>>(M, x, scale, y_in, y_out, w_out, nn, list);          \
  else                                                                                                  \
    k_node_apply<T, BSV, false><<<g, kBlock, 0, s>>>(M, x, scale, y_in, y_out, w_out, nn, list);
  switch (bs) {
    case 1: CAMG_NODE_APPLY_LAUNCH(1) break;
    case 2: CAMG_NODE_APPLY_LAUNCH(2) break;
    case 3: CAMG_NODE_APPLY_LAUNCH(3) break;
    case 4: CAMG_NODE_APPLY_LAUNCH(4) break;
    case 5: CAMG_NODE_APPLY_LAUNCH(5) break;
    default: CAMG_NODE_APPLY_LAUNCH(6) break;
  }
#undef CAMG_NODE_APPLY_LAUNCH
  CAMG_LAUNCHED();
}

template <typename T>
void correct_u(const DCSR<T>& G, const int32_t* rows, int n_rows, const T* delta, const T* ainv, T alpha, T* znu,
               hipStream_t s) {
  if (n_rows <= 0) return;
  CAMG_SG_DISPATCH(rows_sg(G.nnz, n_rows), {
    k_correct_u<T, SG><<<grid_for(n_rows, kBlock / SG), kBlock, 0, s>>>(G, rows, n_rows, delta, ainv, alpha, znu);
  });
  CAMG_LAUNCHED();
}

template <typename T>
void tsmooth_u(const DCSR<T>& KT, const DCSR<T>& BT, const T* zu, const T* zl, const T* bu, T* su, int n_u,
               bool first, int sg, hipStream_t s) {
  if (n_u <= 0) return;
  if (first) {
    k_copy<T><<<grid_for(n_u, kBlock), kBlock, 0, s>>>(bu, su, n_u);
  } else {
    CAMG_SG_DISPATCH(sg, {
      k_tsmooth_u<T, SG, false><<<grid_for(n_u, kBlock / SG), kBlock, 0, s>>>(KT, BT, zu, zl, bu, su, n_u);
    });
  }
  CAMG_LAUNCHED();
}

template <typename T>
void tsmooth_l(const DCSR<T>& GT, const DCSR<T>& CT, const T* zu, const T* zl, const T* bl, const T* su,
               const T* ainv, const T* sdinv, T alpha, T* znl, T* delta, T* rhs_out, int n_l, bool first,
               hipStream_t s) {
  if (n_l <= 0) return;
  CAMG_SG_DISPATCH(rows_sg(GT.nnz + CT.nnz, n_l), {
    dim3 grid(grid_for(n_l, kBlock / SG));
    if (first)
      k_tsmooth_l<T, SG, true><<<grid, kBlock, 0, s>>>(GT, CT, zu, zl, bl, su, ainv, sdinv, alpha, znl, delta,
                                                       rhs_out, n_l);
    else
      k_tsmooth_l<T, SG, false><<<grid, kBlock, 0, s>>>(GT, CT, zu, zl, bl, su, ainv, sdinv, alpha, znl, delta,
                                                        rhs_out, n_l);
  });
  CAMG_LAUNCHED();
}

template <typename T>
void tcorrect_u(const DCSR<T>& BT, const T* su, const T* delta, const T* jinv, T omega, T alpha, const T* zu,
                T* znu, T* t_out, T* w_out, int n_u, bool first, hipStream_t s) {
  if (n_u <= 0) return;
  if (n_u > kWideRows)
    k_tcorrect_u<T, 1><<<grid_for(n_u, kBlock), kBlock, 0, s>>>(BT, su, delta, jinv, omega, alpha,
                                                                first ? nullptr : zu, znu, t_out, w_out, n_u);
  else
    k_tcorrect_u<T, 4><<<grid_for(n_u, kBlock / 4), kBlock, 0, s>>>(BT, su, delta, jinv, omega, alpha,
                                                                    first ? nullptr : zu, znu, t_out, w_out, n_u);
  CAMG_LAUNCHED();
}

template <typename T>
void uzawa_update(const T* zu, const T* w, T alpha, T* znu, int n_u, hipStream_t s) {
  if (n_u <= 0) return;
  k_uzawa_update<T><<<grid_for(n_u, kBlock), kBlock, 0, s>>>(zu, w, alpha, znu, n_u);
  CAMG_LAUNCHED();
}

template <typename T>
void dense_gemv(const T* M, const T* x, T* y, int n, hipStream_t s) {
  if (n <= 0) return;
  k_dense_gemv<T><<<grid_for(n, kBlock / 64), kBlock, 0, s>>>(M, x, y, n);
  CAMG_LAUNCHED();
}

void cast_d2f(const double* x, float* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_cast_d2f<<<grid_for(n, kBlock), kBlock, 0, s>>>(x, y, n);
  CAMG_LAUNCHED();
}
void cast_f2d(const float* x, double* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_cast_f2d<<<grid_for(n, kBlock), kBlock, 0, s>>>(x, y, n);
  CAMG_LAUNCHED();
}
template <typename T>
void copy_vec(const T* x, T* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_copy<T><<<grid_for(n, kBlock), kBlock, 0, s>>>(x, y, n);
  CAMG_LAUNCHED();
}
template <typename T>
void zero_vec(T* y, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_zero<T><<<grid_for(n, kBlock), kBlock, 0, s>>>(y, n);
  CAMG_LAUNCHED();
}


#define CAMG_BS_DISPATCH(bs, ...) \
  switch (bs) {                   \
    case 2: {                     \
      constexpr int BS = 2;       \
      __VA_ARGS__;                \
    } break;                      \
    case 3: {                     \
      constexpr int BS = 3;       \
      __VA_ARGS__;                \
    } break;                      \
    case 6: {                     \
      constexpr int BS = 6;       \
      __VA_ARGS__;                \
    } break;                      \
    default: {                    \
      constexpr int BS = 0;       \
      __VA_ARGS__;                \
    } break;                      \
  }

template <typename T, typename XT>
static void blk_spmv_bell_impl(const DBELL<T>& K, const DCSR<T>& A12, const DCSR<T>& A21, const DCSR<T>& A22,
                               const XT* x1, const XT* x2, const T* b1, const T* b2, T* y1, T* y2, int n1, int n2,
                               int mode, T* xcopy, hipStream_t s) {
  if (K.lptr && K.stream && K.bs == 3) {  // symmetric storage, 3x3 blocks: node per lane
    constexpr int BS = 3;
    dim3 gridn((K.n_slices + 3) / 4 + (n2 + kNplBlock - 1) / kNplBlock);
    if (gridn.x == 0) return;
    if (mode == 0)
      k_blk_spmv_bell_npl<T, XT, BS, 0><<<gridn, kNplBlock, 0, s>>>(K, A12, A21, A22, x1, x2, b1, b2, y1, y2, n1, n2,
                                                                    xcopy);
    else if (mode == 1)
      k_blk_spmv_bell_npl<T, XT, BS, 1><<<gridn, kNplBlock, 0, s>>>(K, A12, A21, A22, x1, x2, b1, b2, y1, y2, n1, n2,
                                                                    xcopy);
    else
      k_blk_spmv_bell_npl<T, XT, BS, 2><<<gridn, kNplBlock, 0, s>>>(K, A12, A21, A22, x1, x2, b1, b2, y1, y2, n1, n2,
                                                                    xcopy);
    CAMG_LAUNCHED();
    return;
  }
  const int threads = 64 * K.bs;
  const int nb_l = (n2 + threads - 1) / threads;
  dim3 grid(K.n_slices + nb_l);
  if (grid.x == 0) return;
  CAMG_BS_DISPATCH(K.bs, {
    if (mode == 0)
      k_blk_spmv_bell<T, XT, BS, 0><<<grid, threads, 0, s>>>(K, A12, A21, A22, x1, x2, b1, b2, y1, y2, n1, n2,
                                                              xcopy);
    else if (mode == 1)
      k_blk_spmv_bell<T, XT, BS, 1><<<grid, threads, 0, s>>>(K, A12, A21, A22, x1, x2, b1, b2, y1, y2, n1, n2,
                                                              xcopy);
    else
      k_blk_spmv_bell<T, XT, BS, 2><<<grid, threads, 0, s>>>(K, A12, A21, A22, x1, x2, b1, b2, y1, y2, n1, n2,
                                                              xcopy);
  });
  CAMG_LAUNCHED();
}

template <typename T>
void blk_spmv_bell(const DBELL<T>& K, const DCSR<T>& A12, const DCSR<T>& A21, const DCSR<T>& A22, const T* x1,
                   const T* x2, const T* b1, const T* b2, T* y1, T* y2, int n1, int n2, int mode, hipStream_t s) {
  blk_spmv_bell_impl<T, T>(K, A12, A21, A22, x1, x2, b1, b2, y1, y2, n1, n2, mode, nullptr, s);
}

void op_apply_from_f32(const DBELL<double>& K, const DCSR<double>& A12, const DCSR<double>& A21,
                       const DCSR<double>& A22, const float* x, double* y, double* xcopy, int n1, int n2,
                       hipStream_t s) {
  blk_spmv_bell_impl<double, float>(K, A12, A21, A22, x, x + n1, nullptr, nullptr, y, y + n1, n1, n2, 0, xcopy, s);
}

void op_apply_copy(const DBELL<double>& K, const DCSR<double>& A12, const DCSR<double>& A21,
                   const DCSR<double>& A22, const double* x, double* y, double* xcopy, int n1, int n2,
                   hipStream_t s) {
  blk_spmv_bell_impl<double, double>(K, A12, A21, A22, x, x + n1, nullptr, nullptr, y, y + n1, n1, n2, 0, xcopy,
                                     s);
}

template <typename T>
void smooth_first_l(const DCSR<T>& B, const T* bu, const T* bl, const T* jinv, const T* sdinv, T omega, T alpha,
                    T* znl, T* delta, T* rhs_out, int n_l, hipStream_t s) {
  if (n_l <= 0) return;
  CAMG_SG_DISPATCH(rows_sg(B.nnz, n_l), {
    k_smooth_l_first<T, SG><<<grid_for(n_l, kBlock / SG), kBlock, 0, s>>>(B, bu, jinv, omega, bl, sdinv, alpha,
                                                                          znl, delta, rhs_out, n_l);
  });
  CAMG_LAUNCHED();
}

template <typename T>
void smooth_first_u(const DCSR<T>& G, const T* bu, const T* jinv, const T* ainv, const T* delta, T omega, T alpha,
                    T* znu, int n_u, hipStream_t s) {
  if (n_u <= 0) return;
  if (n_u > kWideRows)
    k_smooth_u_first_corr<T, 1><<<grid_for(n_u, kBlock), kBlock, 0, s>>>(G, bu, jinv, omega, delta, ainv, alpha, znu,
                                                                         n_u);
  else
    k_smooth_u_first_corr<T, 4><<<grid_for(n_u, kBlock / 4), kBlock, 0, s>>>(G, bu, jinv, omega, delta, ainv, alpha,
                                                                             znu, n_u);
  CAMG_LAUNCHED();
}

template <typename T>
void smooth_u_bell(const DBELL<T>& K, const DCSR<T>& G, const T* zu, const T* zl, const T* bu, const T* jinv,
                   T omega, T* znu, T* r_out, T* w_out, int n_u, hipStream_t s) {
  if (n_u <= 0) return;
  if (K.lptr && K.stream && K.bs == 3) {
    k_smooth_u_bell_npl<T, 3><<<(K.n_slices + 3) / 4, kNplBlock, 0, s>>>(K, G, zu, zl, bu, jinv, omega, znu, r_out,
                                                                         w_out);
    CAMG_LAUNCHED();
    return;
  }
  CAMG_BS_DISPATCH(K.bs, {
    k_smooth_u_bell<T, BS><<<K.n_slices, 64 * K.bs, 0, s>>>(K, G, zu, zl, bu, jinv, omega, znu, r_out, w_out);
  });
  CAMG_LAUNCHED();
}

template <typename T>
void tsmooth_u_bell(const DBELL<T>& KT, const DCSR<T>& BT, const T* zu, const T* zl, const T* bu, T* su, int n_u,
                    hipStream_t s) {
  if (n_u <= 0) return;
  if (KT.lptr && KT.stream && KT.bs == 3) {
    k_tsmooth_u_bell_npl<T, 3><<<(KT.n_slices + 3) / 4, kNplBlock, 0, s>>>(KT, BT, zu, zl, bu, su);
    CAMG_LAUNCHED();
    return;
  }
  CAMG_BS_DISPATCH(KT.bs, { k_tsmooth_u_bell<T, BS><<<KT.n_slices, 64 * KT.bs, 0, s>>>(KT, BT, zu, zl, bu, su); });
  CAMG_LAUNCHED();
}

template <typename T>
void jacobi_extra_bell(const DBELL<T>& M, const T* w, const T* r, const T* jinv, T omega, T* w_out, const T* zu,
                       T* znu, bool last, int n_u, hipStream_t s) {
  if (n_u <= 0) return;
  CAMG_BS_DISPATCH(M.bs, {
    k_jacobi_extra_bell<T, BS><<<M.n_slices, 64 * M.bs, 0, s>>>(M, w, r, jinv, omega, w_out, zu, znu, last ? 1 : 0);
  });
  CAMG_LAUNCHED();
}

template <typename T>
void smooth_u_bell_nodal(const DBELL<T>& K, const DCSR<T>& G, const T* zu, const T* zl, const T* bu, const T* M,
                         T omega, T* znu, T* t_out, T* w_out, int n_u, hipStream_t s) {
  if (n_u <= 0) return;
  if ((int64_t)K.n_nodes * K.bs != n_u) throw std::runtime_error("smooth_u_bell_nodal: layout does not match n_u");
  switch (K.bs) {
    case 2: k_smooth_u_bell_nodal<T, 2><<<K.n_slices, 128, 0, s>>>(K, G, zu, zl, bu, M, omega, znu, t_out, w_out); break;
    case 3: k_smooth_u_bell_nodal<T, 3><<<K.n_slices, 192, 0, s>>>(K, G, zu, zl, bu, M, omega, znu, t_out, w_out); break;
    case 6: k_smooth_u_bell_nodal<T, 6><<<K.n_slices, 384, 0, s>>>(K, G, zu, zl, bu, M, omega, znu, t_out, w_out); break;
    default: throw std::runtime_error("smooth_u_bell_nodal: node block size must be 2, 3 or 6");
  }
  CAMG_LAUNCHED();
}

#define CAMG_NODE_BS_DISPATCH(bs, ...)                                               \
  switch (bs) {                                                                      \
    case 1: { constexpr int BS = 1; __VA_ARGS__; } break;                            \
    case 2: { constexpr int BS = 2; __VA_ARGS__; } break;                            \
    case 3: { constexpr int BS = 3; __VA_ARGS__; } break;                            \
    case 4: { constexpr int BS = 4; __VA_ARGS__; } break;                            \
    case 5: { constexpr int BS = 5; __VA_ARGS__; } break;                            \
    case 6: { constexpr int BS = 6; __VA_ARGS__; } break;                            \
    default: throw std::runtime_error("nodal kernels: node block size must be 1..6"); \
  }

template <typename T>
void node_correct(const DCSR<T>& G, const int32_t* nodes, int n_list, const T* delta, const T* M, T scale, T* znu,
                  int bs, hipStream_t s) {
  if (n_list <= 0) return;
  CAMG_NODE_BS_DISPATCH(bs, {
    k_node_correct<T, BS><<<grid_for(n_list, kBlock / 64), kBlock, 0, s>>>(G, nodes, n_list, delta, M, scale, znu);
  });
  CAMG_LAUNCHED();
}

template <typename T>
void tcorrect_nodal(const DCSR<T>& BT, const T* su, const T* delta, const T* M, T omega, T a_bt, T c_w, const T* zu,
                    T* znu, T* t_out, T* w_out, int n_u, int bs, hipStream_t s) {
  if (n_u <= 0) return;
  if (bs < 1 || n_u % bs) throw std::runtime_error("tcorrect_nodal: node block size must divide n_u");
  const int nn = n_u / bs;
  CAMG_NODE_BS_DISPATCH(bs, {
    k_tcorrect_nodal<T, BS><<<grid_for(nn, kBlock), kBlock, 0, s>>>(BT, su, delta, M, omega, a_bt, c_w, zu, znu,
                                                                     t_out, w_out, nn);
  });
  CAMG_LAUNCHED();
}
#undef CAMG_NODE_BS_DISPATCH

template <typename T>
bool agg_transfer(const AggTransferView<T>& t, bool restrict_dir, const T* xu, const T* xl, T* yu, T* yl,
                  hipStream_t s) {
  const int nfine = t.n_u + t.n_l;
  if (restrict_dir) {
    constexpr int SG = 64;  // one wave per aggregate (enough loads in flight per aggregate)
    const int na = t.n_agg_u + t.n_agg_l;
    if (na <= 0) return true;
    const unsigned g = grid_for(na, kBlock / SG);
    if (t.ns_u == 6 && t.ns_l == 3)
      k_restrict_agg<T, 6, 3, SG><<<g, kBlock, 0, s>>>(t.ptr_u, t.rows_u, t.pu, t.ptr_l, t.rows_l, t.pl, xu, xl, yu, yl,
                                                       t.n_agg_u, t.n_agg_l);
    else if (t.ns_u == 3 && t.ns_l == 2)
      k_restrict_agg<T, 3, 2, SG><<<g, kBlock, 0, s>>>(t.ptr_u, t.rows_u, t.pu, t.ptr_l, t.rows_l, t.pl, xu, xl, yu, yl,
                                                       t.n_agg_u, t.n_agg_l);
    else
      return false;
  } else {
    if (nfine <= 0) return true;
    const unsigned g = grid_for(nfine, kBlock);
    if (t.ns_u == 6 && t.ns_l == 3)
      k_prolong_agg<T, 6, 3><<<g, kBlock, 0, s>>>(t.base_u, t.pu, t.base_l, t.pl, xu, xl, yu, yl, t.n_u, t.n_l);
    else if (t.ns_u == 3 && t.ns_l == 2)
      k_prolong_agg<T, 3, 2><<<g, kBlock, 0, s>>>(t.base_u, t.pu, t.base_l, t.pl, xu, xl, yu, yl, t.n_u, t.n_l);
    else
      return false;
  }
  CAMG_LAUNCHED();
  return true;
}

int cgs_blocks(int64_t n) { return (int)std::max<int64_t>(1, (n + kCgsBlock - 1) / kCgsBlock); }

#define CAMG_KMAX_DISPATCH(kk, ...)  \
  if (kk <= 8) {                     \
    constexpr int KMAX = 8;          \
    __VA_ARGS__;                     \
  } else if (kk <= 16) {             \
    constexpr int KMAX = 16;         \
    __VA_ARGS__;                     \
  } else if (kk <= 32) {             \
    constexpr int KMAX = 32;         \
    __VA_ARGS__;                     \
  } else {                           \
    constexpr int KMAX = 64;         \
    __VA_ARGS__;                     \
  }

void cgs_pass1(const double* V, int64_t ld, int kk, const double* w, int64_t n, double* partial, double* h1,
               hipStream_t s) {
  if (kk < 1 || kk > 64) throw HipError{hipErrorInvalidValue, "cgs_pass1: kk out of range"};
  const int nb = cgs_blocks(n);
  CAMG_KMAX_DISPATCH(kk, {
    k_cgs<KMAX, 1><<<nb, kCgsBlock, 0, s>>>(V, ld, kk, const_cast<double*>(w), n, nullptr, partial);
  });
  CAMG_LAUNCHED();
  k_mdot_reduce<<<kk, kBlock, 0, s>>>(partial, nb, h1);
  CAMG_LAUNCHED();
}

void cgs_pass2(const double* V, int64_t ld, int kk, double* w, int64_t n, const double* h1, double* partial,
               double* h2, hipStream_t s) {
  if (kk < 1 || kk > 64) throw HipError{hipErrorInvalidValue, "cgs_pass2: kk out of range"};
  const int nb = cgs_blocks(n);
  CAMG_KMAX_DISPATCH(kk, { k_cgs<KMAX, 2><<<nb, kCgsBlock, 0, s>>>(V, ld, kk, w, n, h1, partial); });
  CAMG_LAUNCHED();
  k_mdot_reduce<<<kk, kBlock, 0, s>>>(partial, nb, h2);
  CAMG_LAUNCHED();
}

void cgs2_gram(const double* V, int64_t ld, int kk, double* w, int64_t n, double* partial, double* h1, double* h2,
               double* c, double* G, double* gn, const double* scale, double* H, int ldh, double* cs, double* sn,
               double* g, double* out, double* out_host, hipStream_t s) {
  if (kk < 1 || kk > 64) throw HipError{hipErrorInvalidValue, "cgs2_gram: kk out of range"};
  const int nb = cgs_blocks(n);
  const int j = kk - 1;
  // pass 1: h1 = V^T w
  CAMG_KMAX_DISPATCH(kk, { k_cgs<KMAX, 1><<<nb, kCgsBlock, 0, s>>>(V, ld, kk, w, n, nullptr, partial); });
  CAMG_LAUNCHED();
  k_mdot_reduce<<<kk, kBlock, 0, s>>>(partial, nb, h1);
  CAMG_LAUNCHED();
  // h2 from the Gram matrix (column j from the previous step's dots gn)
  k_gram_step<<<1, 256, 0, s>>>(G, j, gn, scale, h1, h2, c);
  CAMG_LAUNCHED();
  // pass 2: w -= V c, gn = V^T w (next Gram column) and ||w||^2 in gn[kk]
  CAMG_KMAX_DISPATCH(kk, { k_cgs<KMAX, 5><<<nb, kCgsBlock, 0, s>>>(V, ld, kk, w, n, c, partial); });
  CAMG_LAUNCHED();
  k_mdot_reduce<<<kk + 1, kBlock, 0, s>>>(partial, nb, gn);
  CAMG_LAUNCHED();
  // Hessenberg column h1 + h2, its Givens rotation, the residual estimate
  // (the squared norm is already reduced: one partial)
  k_cgs_finish<<<1, kBlock, 0, s>>>(gn + kk, 1, kk, h1, h2, H, ldh, cs, sn, g, out, out_host);
  CAMG_LAUNCHED();
}

void cgs_pass3(const double* V, int64_t ld, int kk, double* w, int64_t n, const double* h1, const double* h2,
               double* partial, double* H, int ldh, double* cs, double* sn, double* g, double* out, double* out_host,
               hipStream_t s) {
  if (kk < 1 || kk > 64) throw HipError{hipErrorInvalidValue, "cgs_pass3: kk out of range"};
  const int nb = cgs_blocks(n);
  CAMG_KMAX_DISPATCH(kk, { k_cgs<KMAX, 3><<<nb, kCgsBlock, 0, s>>>(V, ld, kk, w, n, h2, partial); });
  CAMG_LAUNCHED();
  k_cgs_finish<<<1, kBlock, 0, s>>>(partial, nb, kk, h1, h2, H, ldh, cs, sn, g, out, out_host);
  CAMG_LAUNCHED();
}

template <typename T>
void arnoldi_prep(const double* w, const double* scale, double* vj, T* b_out, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_arnoldi_prep<T><<<grid_for(n, kBlock), kBlock, 0, s>>>(w, scale, vj, b_out, n);
  CAMG_LAUNCHED();
}

int mdot_blocks(int64_t n) {
  int64_t nb = (n + 511) / 512;
  return (int)std::max<int64_t>(1, std::min<int64_t>(2048, nb));
}

void mdot(const double* V, int64_t ld, int kk, const double* w, int64_t n, double* partial, double* h,
          hipStream_t s) {
  if (kk <= 0) return;
  const int nb = mdot_blocks(n);
  const int64_t chunk = (n + nb - 1) / nb;
  k_mdot_partial<<<nb, kBlock, 0, s>>>(V, ld, kk, w, n, chunk, partial, nb);
  CAMG_LAUNCHED();
  k_mdot_reduce<<<kk, kBlock, 0, s>>>(partial, nb, h);
  CAMG_LAUNCHED();
}

void gemv_acc(const double* M, int64_t ld, int kk, const double* c, double sign, double* y, int64_t n,
              hipStream_t s) {
  if (kk <= 0 || n <= 0) return;
  k_gemv_acc<<<grid_for(n, kBlock), kBlock, 0, s>>>(M, ld, kk, c, sign, y, n);
  CAMG_LAUNCHED();
}

void arnoldi_update(double* H, int ldh, double* cs, double* sn, double* g, const double* h1, const double* h2,
                    const double* hn2, int j, double* out, double* out_host, hipStream_t s) {
  k_arnoldi_update<<<1, 64, 0, s>>>(H, ldh, cs, sn, g, h1, h2, hn2, j, out, out_host);
  CAMG_LAUNCHED();
}

void restart_init(const double* r, const double* beta2, double* V0, double* g, int gl, double* out, int64_t n,
                  hipStream_t s) {
  const int64_t m = std::max<int64_t>(n, gl);
  k_restart_init<<<grid_for(m, kBlock), kBlock, 0, s>>>(r, beta2, V0, g, gl, out, n);
  CAMG_LAUNCHED();
}

void hess_solve(const double* H, int ldh, const double* g, double* y, int k, hipStream_t s) {
  if (k <= 0) return;
  k_hess_solve<<<1, 64, 0, s>>>(H, ldh, g, y, k);
  CAMG_LAUNCHED();
}

void grad_K(const DCSR<double>& K, const double* lam, const double* x, double* dK, hipStream_t s) {
  if (K.nrows <= 0) return;
  const int sg = pick_subgroup(K.nnz, K.nrows);
  CAMG_SG_DISPATCH(sg, { k_grad_K<SG><<<grid_for(K.nrows, kBlock / SG), kBlock, 0, s>>>(K, lam, x, dK); });
  CAMG_LAUNCHED();
}

template <typename T>
void scatter_perm(const double* src, const int32_t* perm, T* dst, int64_t nnz, hipStream_t s) {
  if (nnz <= 0) return;
  k_scatter_perm<T><<<grid_for(nnz, kBlock), kBlock, 0, s>>>(src, perm, dst, nnz);
  CAMG_LAUNCHED();
}

void scatter_pos64(const double* src, const int64_t* pos, double* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  k_scatter_pos64<<<grid_for(n, kBlock), kBlock, 0, s>>>(src, pos, dst, n);
  CAMG_LAUNCHED();
}

void check_symmetric(const double* v, const int32_t* perm, int64_t n, int32_t* flag, hipStream_t s) {
  if (n <= 0) return;
  k_check_symmetric<<<grid_for(n, kBlock), kBlock, 0, s>>>(v, perm, n, flag);
  CAMG_LAUNCHED();
}

#define CAMG_INSTANTIATE(T)                                                                                        \
  template void blk_spmv<T>(const DCSR<T>&, const DCSR<T>&, const DCSR<T>&, const DCSR<T>&, const T*, const T*,   \
                            const T*, const T*, T*, T*, int, int, int, int, hipStream_t);                         \
  template void smooth_u<T>(const DCSR<T>&, const DCSR<T>&, const T*, const T*, const T*, const T*, T, T*, T*, T*, \
                            int, bool, int, hipStream_t);                                                          \
  template void jacobi_extra<T>(const DCSR<T>&, const T*, const T*, const T*, T, T*, const T*, T*, bool, int, int, \
                                hipStream_t);                                                                      \
  template void smooth_l<T>(const DCSR<T>&, const DCSR<T>&, const T*, const T*, const T*, const T*, T, T*, T*, T*, \
                            int, bool, hipStream_t);                                                               \
  template T* schur_steps<T>(const DCSR<T>&, const T*, T*, T*, const T*, const T*, T, T*, int, int, int,          \
                             hipStream_t);                                                                         \
  template T* schur_block_steps<T>(const DCSR<T>&, const T*, T*, T*, const T*, bool, const T*, T, T*, int, int, int, \
                                   hipStream_t);                                                                   \
  template void node_apply<T>(const T*, const T*, T, const T*, T*, T*, int, int, bool, hipStream_t, const int32_t*, \
                              int);                                                                                \
  template void smooth_u_bell_nodal<T>(const DBELL<T>&, const DCSR<T>&, const T*, const T*, const T*, const T*, T,  \
                                       T*, T*, T*, int, hipStream_t);                                              \
  template bool agg_transfer<T>(const AggTransferView<T>&, bool, const T*, const T*, T*, T*, hipStream_t);          \
  template void node_correct<T>(const DCSR<T>&, const int32_t*, int, const T*, const T*, T, T*, int, hipStream_t);  \
  template void tcorrect_nodal<T>(const DCSR<T>&, const T*, const T*, const T*, T, T, T, const T*, T*, T*, T*, int, \
                                  int, hipStream_t);                                                               \
  template void correct_u<T>(const DCSR<T>&, const int32_t*, int, const T*, const T*, T, T*, hipStream_t);         \
  template void tsmooth_u<T>(const DCSR<T>&, const DCSR<T>&, const T*, const T*, const T*, T*, int, bool, int,      \
                             hipStream_t);                                                                         \
  template void tsmooth_l<T>(const DCSR<T>&, const DCSR<T>&, const T*, const T*, const T*, const T*, const T*,      \
                             const T*, T, T*, T*, T*, int, bool, hipStream_t);                                     \
  template void tcorrect_u<T>(const DCSR<T>&, const T*, const T*, const T*, T, T, const T*, T*, T*, T*, int, bool,  \
                              hipStream_t);                                                                        \
  template void dense_gemv<T>(const T*, const T*, T*, int, hipStream_t);                                           \
  template void uzawa_update<T>(const T*, const T*, T, T*, int, hipStream_t);                                      \
  template void copy_vec<T>(const T*, T*, int64_t, hipStream_t);                                                   \
  template void zero_vec<T>(T*, int64_t, hipStream_t);                                                             \
  template void scatter_perm<T>(const double*, const int32_t*, T*, int64_t, hipStream_t);                          \
  template void smooth_first_l<T>(const DCSR<T>&, const T*, const T*, const T*, const T*, T, T, T*, T*, T*, int,   \
                                  hipStream_t);                                                                    \
  template void smooth_first_u<T>(const DCSR<T>&, const T*, const T*, const T*, const T*, T, T, T*, int,          \
                                  hipStream_t);                                                                    \
  template void blk_spmv_bell<T>(const DBELL<T>&, const DCSR<T>&, const DCSR<T>&, const DCSR<T>&, const T*,        \
                                 const T*, const T*, const T*, T*, T*, int, int, int, hipStream_t);               \
  template void smooth_u_bell<T>(const DBELL<T>&, const DCSR<T>&, const T*, const T*, const T*, const T*, T, T*,   \
                                 T*, T*, int, hipStream_t);                                                        \
  template void tsmooth_u_bell<T>(const DBELL<T>&, const DCSR<T>&, const T*, const T*, const T*, T*, int,          \
                                  hipStream_t);                                                                    \
  template void jacobi_extra_bell<T>(const DBELL<T>&, const T*, const T*, const T*, T, T*, const T*, T*, bool, int, \
                                     hipStream_t);                                                                 \
  template void arnoldi_prep<T>(const double*, const double*, double*, T*, int64_t, hipStream_t);

CAMG_INSTANTIATE(float)
CAMG_INSTANTIATE(double)

}  // namespace camg
