// Launch wrappers for the libcamg device kernels (gfx950, wave64).
//
// All kernels are deterministic: no atomics, fixed reduction trees, one
// writer per output element.  Sparse kernels are row-parallel CSR with a
// subgroup of `sg` lanes per row (1..16) whose column/value streams are
// read contiguously by the subgroup.
#pragma once

#include "common.hpp"

namespace camg {

// sg: lanes per row (1, 8 or 16), chosen from the mean row length.
int pick_subgroup(int64_t nnz, int64_t nrows);

// Two-by-two block row SpMV over rows [0, n1) -> (A11 x1 + A12 x2) and rows
// [n1, n1 + n2) -> (A21 x1 + A22 x2).  Empty blocks (nnz = 0) are skipped.
//   mode 0: y = A x     mode 1: y = b - A x     mode 2: y += A x
template <typename T>
void blk_spmv(const DCSR<T>& A11, const DCSR<T>& A12, const DCSR<T>& A21, const DCSR<T>& A22, const T* x1,
              const T* x2, const T* b1, const T* b2, T* y1, T* y2, int n1, int n2, int mode, int sg,
              hipStream_t s);

// CheapSIMPLE forward sweep, displacement rows: r = b_u - K z_u - G z_l,
// w = omega * jinv * r, zn_u = z_u + w.  first: z = 0 (no SpMV).
// If r_out / w_out are non-null they receive r and w (extra Jacobi sweeps).
template <typename T>
void smooth_u(const DCSR<T>& K, const DCSR<T>& G, const T* zu, const T* zl, const T* bu, const T* jinv, T omega,
              T* znu, T* r_out, T* w_out, int n_u, bool first, int sg, hipStream_t s);

// First forward sweep from z = 0 (one Jacobi sweep) in two kernels:
// smooth_first_l: q = -(b_l - B (omega*jinv.*b_u)), delta = q .* sdinv,
// zn_l = alpha*delta (q stored in rhs_out when non-null); then, after any
// Schur sweeps, smooth_first_u: zn_u = omega*jinv.*b_u - alpha*ainv.*(G delta).
template <typename T>
void smooth_first_l(const DCSR<T>& B, const T* bu, const T* bl, const T* jinv, const T* sdinv, T omega, T alpha,
                    T* znl, T* delta, T* rhs_out, int n_l, hipStream_t s);
template <typename T>
void smooth_first_u(const DCSR<T>& G, const T* bu, const T* jinv, const T* ainv, const T* delta, T omega, T alpha,
                    T* znu, int n_u, hipStream_t s);

// Extra damped-Jacobi sweep on M w = r: w_out = w + omega*jinv*(r - M w);
// when last, also zn_u = z_u + w_out (z_u null: zn_u = w_out).
template <typename T>
void jacobi_extra(const DCSR<T>& M, const T* w, const T* r, const T* jinv, T omega, T* w_out, const T* zu, T* znu,
                  bool last, int n_u, int sg, hipStream_t s);

// CheapSIMPLE forward sweep, multiplier rows: rt = b_l - B zn_u - C z_l,
// delta = -rt * sdinv, zn_l = z_l + alpha * delta.  first: z_l = 0.
// rhs_out (optional) receives q = -rt, the right-hand side of S delta = q.
template <typename T>
void smooth_l(const DCSR<T>& B, const DCSR<T>& C, const T* znu, const T* zl, const T* bl, const T* sdinv, T alpha,
              T* znl, T* delta, T* rhs_out, int n_l, bool first, hipStream_t s);

// `steps` undamped Jacobi sweeps on S delta = q continuing from d_a (the
// first sweep's delta = q .* sdinv), ping-ponging between d_a and d_b; the
// last one also writes zn_l = z_l + alpha * delta (z_l null: zero).
// Returns the buffer holding the final delta.
template <typename T>
T* schur_steps(const DCSR<T>& S, const T* q, T* d_a, T* d_b, const T* sdinv, const T* zl, T alpha, T* znl,
               int steps, int n_l, int sg, hipStream_t s);
// Nodal block Jacobi steps on the Schur system (block option): steps >= 1,
// the first from zero; blk holds the inverse bs x bs diagonal blocks of S
// (row-major), applied transposed with trans (S passed as S^T then).  The
// last step writes zn_l = z_l + alpha * delta; returns the buffer holding
// delta.
template <typename T>
T* schur_block_steps(const DCSR<T>& S, const T* q, T* d_a, T* d_b, const T* blk, bool trans, const T* zl, T alpha,
                     T* znl, int steps, int n_l, int bs, hipStream_t s);

// Nodal lumping option: y_out = y_in + scale * M x and w_out = scale * M x
// per node of bs consecutive rows (M: row-major bs x bs blocks, applied
// transposed with trans); y_in null reads as zero, either output may be
// null, y_in may alias y_out.
template <typename T>
void node_apply(const T* M, const T* x, T scale, const T* y_in, T* y_out, T* w_out, int n, int bs, bool trans,
                hipStream_t s, const int32_t* list = nullptr, int n_list = 0);

// Nodal lumping option on the level-0 blocked-ELL layout: t = b_u - K z_u -
// G z_l, w = omega M t per node, zn_u = z_u + w (t_out, w_out optional).
template <typename T>
void smooth_u_bell_nodal(const DBELL<T>& K, const DCSR<T>& G, const T* zu, const T* zl, const T* bu, const T* M,
                         T omega, T* znu, T* t_out, T* w_out, int n_u, hipStream_t s);

// Aggregation transfers with the tentative pattern (no column indices):
// fine row i couples to coarse columns base[i] .. base[i] + ns - 1 (base -1:
// none) with dense per-row values pv[i * ns + k]; ptr/rows list each
// aggregate's fine rows (ascending) for the restriction.
template <typename T>
struct AggTransferView {
  int n_u = 0, n_l = 0, ns_u = 0, ns_l = 0, n_agg_u = 0, n_agg_l = 0;
  const int32_t *base_u = nullptr, *base_l = nullptr;
  const int32_t *ptr_u = nullptr, *rows_u = nullptr, *ptr_l = nullptr, *rows_l = nullptr;
  const T *pu = nullptr, *pl = nullptr;
};

// Restriction (restrict_dir: y = P^T x, coarse y) or prolongation (y += P x,
// fine y) for both blocks in one launch; false when the null-space sizes
// have no instantiation (the caller then uses the CSR transfers).
template <typename T>
bool agg_transfer(const AggTransferView<T>& t, bool restrict_dir, const T* xu, const T* xl, T* yu, T* yl,
                  hipStream_t s);

// Nodal lumping option: zn_u += scale * M (G delta) on the listed nodes.
template <typename T>
void node_correct(const DCSR<T>& G, const int32_t* nodes, int n_list, const T* delta, const T* M, T scale, T* znu,
                  int bs, hipStream_t s);

// Nodal lumping option, adjoint: t = s_u - a_bt B^T delta, w = omega M^T t,
// zn_u = z_u + c_w w per node (z_u null: zero; t_out, w_out optional).
template <typename T>
void tcorrect_nodal(const DCSR<T>& BT, const T* su, const T* delta, const T* M, T omega, T a_bt, T c_w, const T* zu,
                    T* znu, T* t_out, T* w_out, int n_u, int bs, hipStream_t s);

// zn_u[i] -= alpha * ainv[i] * (G delta)[i] for the listed rows of G.
template <typename T>
void correct_u(const DCSR<T>& G, const int32_t* rows, int n_rows, const T* delta, const T* ainv, T alpha, T* znu,
               hipStream_t s);

// Adjoint sweep, step 1: s_u = b_u - K^T z_u - B^T z_l (first: s_u = b_u).
template <typename T>
void tsmooth_u(const DCSR<T>& KT, const DCSR<T>& BT, const T* zu, const T* zl, const T* bu, T* su, int n_u,
               bool first, int sg, hipStream_t s);

// Adjoint sweep, step 2: s_l = b_l - G^T z_u - C^T z_l,
// delta = -(s_l - G^T (ainv .* s_u)) * sdinv, zn_l = z_l + alpha * delta
// (ainv null: no G^T ainv s_u term, the adjoint Uzawa sweep);
// rhs_out (optional) receives q = -(s_l - G^T (ainv .* s_u)).
template <typename T>
void tsmooth_l(const DCSR<T>& GT, const DCSR<T>& CT, const T* zu, const T* zl, const T* bl, const T* su,
               const T* ainv, const T* sdinv, T alpha, T* znl, T* delta, T* rhs_out, int n_l, bool first,
               hipStream_t s);

// Adjoint sweep, step 3: t = s_u - alpha * B^T delta, w = omega*jinv*t,
// zn_u = z_u + w (first: z_u = 0).  t_out / w_out optional.
template <typename T>
void tcorrect_u(const DCSR<T>& BT, const T* su, const T* delta, const T* jinv, T omega, T alpha, const T* zu,
                T* znu, T* t_out, T* w_out, int n_u, bool first, hipStream_t s);

// ---- sliced blocked-ELL (BELL) variants ----------------------------------
// The displacement rows use K (or K^T) in BELL layout with one thread per
// (node, component) row: a workgroup of 64*bs threads covers one slice, wave
// a computes component a of its 64 nodes.  The sparse couplings G, B, C
// stay CSR (one thread per row; they are short and mostly empty).
template <typename T>
void blk_spmv_bell(const DBELL<T>& K, const DCSR<T>& A12, const DCSR<T>& A21, const DCSR<T>& A22, const T* x1,
                   const T* x2, const T* b1, const T* b2, T* y1, T* y2, int n1, int n2, int mode, hipStream_t s);
template <typename T>
void smooth_u_bell(const DBELL<T>& K, const DCSR<T>& G, const T* zu, const T* zl, const T* bu, const T* jinv,
                   T omega, T* znu, T* r_out, T* w_out, int n_u, hipStream_t s);
template <typename T>
void tsmooth_u_bell(const DBELL<T>& KT, const DCSR<T>& BT, const T* zu, const T* zl, const T* bu, T* su, int n_u,
                    hipStream_t s);
template <typename T>
void jacobi_extra_bell(const DBELL<T>& M, const T* w, const T* r, const T* jinv, T omega, T* w_out, const T* zu,
                       T* znu, bool last, int n_u, hipStream_t s);

// FP64 outer operator y = A x (BELL K) reading x in FP32 (the mixed V-cycle
// output) or FP64, and storing x widened to FP64 in xcopy in the same pass.
void op_apply_from_f32(const DBELL<double>& K, const DCSR<double>& A12, const DCSR<double>& A21,
                       const DCSR<double>& A22, const float* x, double* y, double* xcopy, int n1, int n2,
                       hipStream_t s);
void op_apply_copy(const DBELL<double>& K, const DCSR<double>& A12, const DCSR<double>& A21,
                   const DCSR<double>& A22, const double* x, double* y, double* xcopy, int n1, int n2,
                   hipStream_t s);

// Uzawa update of the displacements: zn_u = z_u + alpha w (z_u null: zero).
template <typename T>
void uzawa_update(const T* zu, const T* w, T alpha, T* znu, int n_u, hipStream_t s);

// y = M x for a dense row-major n x n matrix (coarsest level).
template <typename T>
void dense_gemv(const T* M, const T* x, T* y, int n, hipStream_t s);

// Elementwise helpers.
void cast_d2f(const double* x, float* y, int64_t n, hipStream_t s);
void cast_f2d(const float* x, double* y, int64_t n, hipStream_t s);
template <typename T>
void copy_vec(const T* x, T* y, int64_t n, hipStream_t s);
template <typename T>
void zero_vec(T* y, int64_t n, hipStream_t s);

// ---- FP64 Krylov kernels --------------------------------------------------
// Number of partial-sum blocks used by mdot for a vector length n.
int mdot_blocks(int64_t n);
// h[k] = sum_i V[k*ld + i] * w[i] for k < kk (two-stage, fixed order).
// partial must hold kk * mdot_blocks(n) doubles.
void mdot(const double* V, int64_t ld, int kk, const double* w, int64_t n, double* partial, double* h,
          hipStream_t s);
// y[i] += sign * sum_k M[k*ld + i] * c[k]  (c on device)
void gemv_acc(const double* M, int64_t ld, int kk, const double* c, double sign, double* y, int64_t n,
              hipStream_t s);
// Arnoldi column j: H[:, j] = h1 + h2 (kk = j + 1 entries), H[j+1, j] =
// sqrt(*hn2); apply the previous Givens rotations, build rotation j, update
// g.  out[0] = |g[j+1]|, out[1] = H[j+1,j] before rotation, out[2] = 1/out[1]
// (0 when it vanishes).
void arnoldi_update(double* H, int ldh, double* cs, double* sn, double* g, const double* h1, const double* h2,
                    const double* hn2, int j, double* out, double* out_host, hipStream_t s);
// V0 = r * (1 / sqrt(*beta2)); g = [sqrt(*beta2), 0, ...]; out[0] = sqrt(*beta2)
void restart_init(const double* r, const double* beta2, double* V0, double* g, int gl, double* out, int64_t n,
                  hipStream_t s);
// Back substitution H(0:k,0:k) y = g(0:k).
void hess_solve(const double* H, int ldh, const double* g, double* y, int k, hipStream_t s);

// ---- fused CGS2 passes -------------------------------------------------------
// Three passes over the Krylov basis V (n x kk, column-major, ld) per
// Arnoldi step, each followed by a fixed-order reduction of its per-workgroup
// partial sums:
//   pass 1: h1 = V^T w
//   pass 2: w <- w - V h1, h2 = V^T w
//   pass 3: w <- w - V h2, ||w||, then column j = kk - 1 of the Hessenberg
//           matrix, its Givens rotation and g (as arnoldi_update; out[0..2]).
// partial: kk * cgs_blocks(n) doubles.  kk <= 64.
int cgs_blocks(int64_t n);
void cgs_pass1(const double* V, int64_t ld, int kk, const double* w, int64_t n, double* partial, double* h1,
               hipStream_t s);
void cgs_pass2(const double* V, int64_t ld, int kk, double* w, int64_t n, const double* h1, double* partial,
               double* h2, hipStream_t s);
// One CGS2 orthogonalisation of w against the kk columns of V with two
// passes over V instead of three: h1 = V^T w; h2 = h1 - G h1 with the Gram
// matrix G = V^T V (column kk-1 from the previous step's dots gn, scaled by
// *scale = 1/||w_prev||; G is 64 x 64 column-major); w -= V (h1 + h2), whose
// dots with V (the next Gram column) and squared norm land in gn[0..kk];
// then the Hessenberg column, Givens rotation and result block as in
// cgs_pass3.  In exact arithmetic h2 is what CGS2's second pass measures.
void cgs2_gram(const double* V, int64_t ld, int kk, double* w, int64_t n, double* partial, double* h1, double* h2,
               double* c, double* G, double* gn, const double* scale, double* H, int ldh, double* cs, double* sn,
               double* g, double* out, double* out_host, hipStream_t s);
void cgs_pass3(const double* V, int64_t ld, int kk, double* w, int64_t n, const double* h1, const double* h2,
               double* partial, double* H, int ldh, double* cs, double* sn, double* g, double* out, double* out_host,
               hipStream_t s);
// v_j of the Arnoldi basis and the V-cycle input: with scale (device
// scalar, 1/||w||) given, vj = w * scale is written first; then
// b_out = (T) vj.  Without scale, vj is only read.
template <typename T>
void arnoldi_prep(const double* w, const double* scale, double* vj, T* b_out, int64_t n, hipStream_t s);

// dK[e] = -lam[row(e)] * x[col(e)] over the entries of K.
void grad_K(const DCSR<double>& K, const double* lam, const double* x, double* dK, hipStream_t s);
// dst[perm[e]] = src[e] (value refresh of an explicit transpose).
template <typename T>
void scatter_perm(const double* src, const int32_t* perm, T* dst, int64_t nnz, hipStream_t s);
// dst[pos[e]] = src[e] with 64-bit positions (BELL value refresh).
void scatter_pos64(const double* src, const int64_t* pos, double* dst, int64_t n, hipStream_t s);
// flag = 1 when some v[e] != v[perm[e]] (the caller zeroes flag first)
void check_symmetric(const double* v, const int32_t* perm, int64_t n, int32_t* flag, hipStream_t s);

}  // namespace camg
