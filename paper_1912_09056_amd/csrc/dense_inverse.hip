// Explicit inverse of a dense FP64 matrix on one GPU (gfx950): the direct
// solve of the merged coarsest level (the weak-scaling study's solver
// settings, Sec. 6.2, merge the coarse blocks and factorise them by LU).
//
// Right-looking blocked LU with partial pivoting (largest magnitude, first
// row on ties) on 64-column panels, then the inverse from L U X = P by a
// blocked forward and a blocked backward substitution.  Every rank-64
// update C -= A B of the three phases runs on the FP64 matrix cores
// (v_mfma_f64_16x16x4f64, 64 x 64 output tile per workgroup); the panel
// factorisation (one workgroup) and the 64 x 64 triangular solves run on the
// vector units.  Work matrices are column-major with the order padded to a
// multiple of 64 by an identity block, which pivoting never touches (its
// rows are zero in the leading columns) and which adds no fill.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "common.hpp"
#include "dense_inverse.hpp"

namespace camg {

namespace {

constexpr int kNb = 64;              // panel width = depth of every update
constexpr int kPanelThreads = 1024;  // one workgroup factors a panel
constexpr int kTile = 256;           // threads of the update and solve kernels

typedef double d4 __attribute__((ext_vector_type(4)));

// W (N x N, column-major) = the row-major n x n matrix a, transposed into
// column order, padded with the identity.
__global__ void k_pad_transpose(const double* __restrict__ a, int n, double* __restrict__ W, int N) {
  const int64_t e = (int64_t)blockIdx.x * kTile + threadIdx.x;
  if (e >= (int64_t)N * N) return;
  const int c = (int)(e / N), r = (int)(e % N);
  W[e] = (r < n && c < n) ? a[(int64_t)r * n + c] : (r == c ? 1.0 : 0.0);
}

__global__ void k_identity(double* __restrict__ Y, int N) {
  const int64_t e = (int64_t)blockIdx.x * kTile + threadIdx.x;
  if (e >= (int64_t)N * N) return;
  Y[e] = (e / N == e % N) ? 1.0 : 0.0;
}

// Factors rows [k, N) of columns [k, k + 64) in place.  Per column: the pivot
// row (largest |a|, first on ties) is swapped into place within the panel,
// the column below the diagonal is divided by the pivot, and the rank-1
// update reaches the panel's remaining columns.  piv[c] = pivot row of
// column c; *status = 1 when a pivot is not above tiny (the row is then
// kept and the column left unscaled).
__global__ void __launch_bounds__(kPanelThreads) k_lu_panel(double* __restrict__ A, int N, int k,
                                                            int32_t* __restrict__ piv, double tiny,
                                                            int* __restrict__ status) {
  __shared__ double sval[kPanelThreads / 64];
  __shared__ int sidx[kPanelThreads / 64];
  __shared__ int spiv;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  for (int j = 0; j < kNb; ++j) {
    const int c = k + j;
    double* col = A + (int64_t)c * N;
    double best = -1.0;
    int bi = N;
    for (int i = c + t; i < N; i += kPanelThreads) {
      const double v = fabs(col[i]);
      if (v > best) {
        best = v;
        bi = i;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const double ov = __shfl_down(best, off);
      const int oi = __shfl_down(bi, off);
      if (ov > best || (ov == best && oi < bi)) {
        best = ov;
        bi = oi;
      }
    }
    if (lane == 0) {
      sval[wave] = best;
      sidx[wave] = bi;
    }
    __syncthreads();
    if (t == 0) {
      double bv = sval[0];
      int b = sidx[0];
      for (int w = 1; w < kPanelThreads / 64; ++w)
        if (sval[w] > bv || (sval[w] == bv && sidx[w] < b)) {
          bv = sval[w];
          b = sidx[w];
        }
      if (!(bv > tiny)) {
        status[0] = 1;
        b = c;
      }
      piv[c] = b;
      spiv = b;
    }
    __syncthreads();
    const int p = spiv;
    if (p != c && t < kNb) {
      double* cc = A + (int64_t)(k + t) * N;
      const double x = cc[c];
      cc[c] = cc[p];
      cc[p] = x;
    }
    __syncthreads();
    const double d = col[c];
    if (d != 0.0 && fabs(d) > tiny)
      for (int i = c + 1 + t; i < N; i += kPanelThreads) col[i] = col[i] / d;
    __syncthreads();
    for (int jj = c + 1; jj < k + kNb; ++jj) {
      double* cj = A + (int64_t)jj * N;
      const double u = cj[c];
      if (u != 0.0)
        for (int i = c + 1 + t; i < N; i += kPanelThreads) cj[i] -= col[i] * u;
    }
    __syncthreads();
  }
}

// Applies the row interchanges of rows [r0, r1) (piv, in order) to every
// column c of the N x N column-major M outside [skip0, skip1).
__global__ void k_row_swaps(double* __restrict__ M, int N, int r0, int r1, const int32_t* __restrict__ piv,
                            int skip0, int skip1) {
  const int c = blockIdx.x * kTile + threadIdx.x;
  if (c >= N || (c >= skip0 && c < skip1)) return;
  double* cc = M + (int64_t)c * N;
  for (int r = r0; r < r1; ++r) {
    const int p = piv[r];
    if (p != r) {
      const double x = cc[r];
      cc[r] = cc[p];
      cc[p] = x;
    }
  }
}

// X = T^-1 X for the 64 x 64 diagonal block T = A[k:k+64, k:k+64] (unit
// lower triangle of the LU factors when LOWER, else the upper triangle with
// its diagonal) and the right-hand sides X = M[k:k+64, c0:c0+m] of the
// column-major M; one thread per column.
template <bool LOWER>
__global__ void __launch_bounds__(kTile) k_trsm64(const double* __restrict__ A, int lda, int k, double* __restrict__ M,
                                                  int ldm, int c0, int m) {
  __shared__ double T[kNb][kNb + 1];  // T[i][q] = A[k + i][k + q]
  for (int e = threadIdx.x; e < kNb * kNb; e += kTile) {
    const int q = e / kNb, i = e % kNb;
    T[i][q] = A[(int64_t)(k + q) * lda + k + i];
  }
  __syncthreads();
  const int c = blockIdx.x * kTile + threadIdx.x;
  if (c >= m) return;
  double* b = M + (int64_t)(c0 + c) * ldm + k;
  double x[kNb];
#pragma unroll
  for (int i = 0; i < kNb; ++i) x[i] = b[i];
  if (LOWER) {
#pragma unroll
    for (int i = 1; i < kNb; ++i) {
      double s = x[i];
#pragma unroll
      for (int q = 0; q < i; ++q) s -= T[i][q] * x[q];
      x[i] = s;
    }
  } else {
#pragma unroll
    for (int i = kNb - 1; i >= 0; --i) {
      double s = x[i];
#pragma unroll
      for (int q = i + 1; q < kNb; ++q) s -= T[i][q] * x[q];
      x[i] = s / T[i][i];
    }
  }
#pragma unroll
  for (int i = 0; i < kNb; ++i) b[i] = x[i];
}

// C -= A B with A (M x 64), B (64 x Nc), C (M x Nc), all column-major, M and
// Nc multiples of 64; one 64 x 64 tile of C per workgroup.  The tiles of A
// and B are staged in LDS; each wave accumulates a 32 x 32 quarter as 2 x 2
// blocks of v_mfma_f64_16x16x4f64 over the 64-deep product.  Operand lanes:
// lane l carries A[l % 16][q0 + l / 16] and B[q0 + l / 16][l % 16]; result
// element r of lane l is D[l / 16 + 4 r][l % 16] (checked on the device).
__global__ void __launch_bounds__(kTile) k_gemm64_sub(const double* __restrict__ A, int lda,
                                                      const double* __restrict__ B, int ldb, double* __restrict__ C,
                                                      int ldc) {
  __shared__ double As[kNb][kNb + 1];  // As[q][i] = A[i0 + i][q]
  __shared__ double Bs[kNb][kNb + 1];  // Bs[j][q] = B[q][j0 + j]
  const int i0 = blockIdx.x * kNb, j0 = blockIdx.y * kNb;
  const int t = threadIdx.x;
  for (int e = t; e < kNb * kNb; e += kTile) {
    const int outer = e >> 6, inner = e & 63;
    As[outer][inner] = A[(int64_t)outer * lda + i0 + inner];
    Bs[outer][inner] = B[(int64_t)(j0 + outer) * ldb + inner];
  }
  __syncthreads();
  const int w = t >> 6, l = t & 63;
  const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
  const int lr = l & 15, lq = l >> 4;
  d4 acc00 = {0.0, 0.0, 0.0, 0.0}, acc01 = acc00, acc10 = acc00, acc11 = acc00;
#pragma unroll
  for (int q0 = 0; q0 < kNb; q0 += 4) {
    const int q = q0 + lq;
    const double a0 = As[q][wi + lr], a1 = As[q][wi + 16 + lr];
    const double b0 = Bs[wj + lr][q], b1 = Bs[wj + 16 + lr][q];
    acc00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc00, 0, 0, 0);
    acc01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc01, 0, 0, 0);
    acc10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc10, 0, 0, 0);
    acc11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc11, 0, 0, 0);
  }
  const d4* acc[2][2] = {{&acc00, &acc01}, {&acc10, &acc11}};
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int col = j0 + wj + 16 * bj + lr;
      double* cc = C + (int64_t)col * ldc + i0 + wi + 16 * bi + lq;
#pragma unroll
      for (int r = 0; r < 4; ++r) cc[4 * r] -= (*acc[bi][bj])[r];
    }
}

// inv (row-major n x n) = Y's leading block read transposed, invT
// (row-major) = Y's leading block as stored; Y is column-major N x N.
template <typename T>
__global__ void k_extract(const double* __restrict__ Y, int N, int n, T* __restrict__ inv, T* __restrict__ invT) {
  const int64_t e = (int64_t)blockIdx.x * kTile + threadIdx.x;
  if (e >= (int64_t)n * n) return;
  const int c = (int)(e / n), r = (int)(e % n);
  const double v = Y[(int64_t)c * N + r];  // (A^-1)[r][c]
  if (inv) inv[(int64_t)r * n + c] = (T)v;
  if (invT) invT[e] = (T)v;
}

// out[0] = max |a_e| over e < n, NaN when some entry is not finite; one
// workgroup.
__global__ void __launch_bounds__(1024) k_max_abs(const double* __restrict__ a, int64_t n, double* __restrict__ out) {
  __shared__ double sm[1024 / 64];
  double m = 0.0;
  bool bad = false;
  for (int64_t e = threadIdx.x; e < n; e += 1024) {
    const double v = fabs(a[e]);
    bad |= !(v <= 1.7976931348623157e308);
    m = v > m ? v : m;
  }
  if (bad) m = __builtin_nan("");
  for (int off = 32; off > 0; off >>= 1) {
    const double o = __shfl_down(m, off);
    m = (o != o || o > m) ? o : m;
  }
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = sm[0];
    for (int w = 1; w < 1024 / 64; ++w) r = (sm[w] != sm[w] || sm[w] > r) ? sm[w] : r;
    out[0] = r;
  }
}

inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

template <typename T>
bool dense_inverse(const double* a, int64_t n, double tiny, T* inv, T* invT, hipStream_t s) {
  if (n <= 0) return true;
  if (n > 46000) throw OomError{(size_t)(n * n * 16)};
  const int N = (int)((n + kNb - 1) / kNb * kNb);
  const int64_t NN = (int64_t)N * N;
  DBuf<double> W((size_t)NN), Y((size_t)NN);
  DBuf<int32_t> piv((size_t)N);
  DBuf<int> status(1);
  CAMG_HIP(hipMemsetAsync(status.p, 0, sizeof(int), s));
  k_pad_transpose<<<blocks_for(NN, kTile), kTile, 0, s>>>(a, (int)n, W.p, N);
  CAMG_LAUNCHED();
  // LU: W = P^T L U, factors in place
  for (int k = 0; k < N; k += kNb) {
    k_lu_panel<<<1, kPanelThreads, 0, s>>>(W.p, N, k, piv.p, tiny, status.p);
    CAMG_LAUNCHED();
    k_row_swaps<<<blocks_for(N, kTile), kTile, 0, s>>>(W.p, N, k, k + kNb, piv.p, k, k + kNb);
    CAMG_LAUNCHED();
    const int rest = N - k - kNb;
    if (rest > 0) {
      k_trsm64<true><<<blocks_for(rest, kTile), kTile, 0, s>>>(W.p, N, k, W.p, N, k + kNb, rest);
      CAMG_LAUNCHED();
      k_gemm64_sub<<<dim3(rest / kNb, rest / kNb), kTile, 0, s>>>(W.p + (int64_t)k * N + k + kNb, N,
                                                                   W.p + (int64_t)(k + kNb) * N + k, N,
                                                                   W.p + (int64_t)(k + kNb) * N + k + kNb, N);
      CAMG_LAUNCHED();
    }
  }
  // Y = P, then Y = L^-1 Y (forward, right-looking) and Y = U^-1 Y (backward)
  k_identity<<<blocks_for(NN, kTile), kTile, 0, s>>>(Y.p, N);
  CAMG_LAUNCHED();
  k_row_swaps<<<blocks_for(N, kTile), kTile, 0, s>>>(Y.p, N, 0, N, piv.p, 0, 0);
  CAMG_LAUNCHED();
  for (int k = 0; k < N; k += kNb) {
    k_trsm64<true><<<blocks_for(N, kTile), kTile, 0, s>>>(W.p, N, k, Y.p, N, 0, N);
    CAMG_LAUNCHED();
    const int rest = N - k - kNb;
    if (rest > 0) {
      k_gemm64_sub<<<dim3(rest / kNb, N / kNb), kTile, 0, s>>>(W.p + (int64_t)k * N + k + kNb, N, Y.p + k, N,
                                                               Y.p + k + kNb, N);
      CAMG_LAUNCHED();
    }
  }
  for (int k = N - kNb; k >= 0; k -= kNb) {
    k_trsm64<false><<<blocks_for(N, kTile), kTile, 0, s>>>(W.p, N, k, Y.p, N, 0, N);
    CAMG_LAUNCHED();
    if (k > 0) {
      k_gemm64_sub<<<dim3(k / kNb, N / kNb), kTile, 0, s>>>(W.p + (int64_t)k * N, N, Y.p + k, N, Y.p, N);
      CAMG_LAUNCHED();
    }
  }
  k_extract<T><<<blocks_for(n * n, kTile), kTile, 0, s>>>(Y.p, N, (int)n, inv, invT);
  CAMG_LAUNCHED();
  int st = 0;
  CAMG_HIP(hipMemcpyAsync(&st, status.p, sizeof(int), hipMemcpyDeviceToHost, s));
  CAMG_HIP(hipStreamSynchronize(s));
  return st == 0;
}

void max_abs(const double* a, int64_t n, double* out, hipStream_t s) {
  k_max_abs<<<1, 1024, 0, s>>>(a, n, out);
  CAMG_LAUNCHED();
}

template bool dense_inverse<double>(const double*, int64_t, double, double*, double*, hipStream_t);
template bool dense_inverse<float>(const double*, int64_t, double, float*, float*, hipStream_t);

}  // namespace camg
