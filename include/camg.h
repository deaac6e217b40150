/*
 * camg.h -- C-ABI of libcamg: fully coupled block-AMG preconditioned FGMRES
 * for mortar-contact saddle-point systems on one AMD Instinct MI355X (gfx950).
 *
 * The system is the compact block form of the linearised mortar-contact
 * problem (Wiesner, Mayr, Popp, Gee, Wall, "Algebraic multigrid methods for
 * saddle point systems arising from mortar contact formulations",
 * Sec. 2.3, the 2x2 block system and its short notation):
 *
 *     [ K  G ] [u]   [f]       G = C1^T  (n_u x n_l, upper-right coupling)
 *     [ B  C ] [l] = [g]       B = C2    (n_l x n_u, constraint rows)
 *                              C = -Z    (n_l x n_l)
 *
 * Vectors crossing this interface are contiguous [u; l] of length
 * n = n_u + n_l.
 *
 * Conventions for every entry point:
 *  - Return value: CAMG_OK (0) on success, CAMG_NOT_CONVERGED (1) when a
 *    solve stopped at its iteration limit (the output then holds the last
 *    iterate), or a negative CAMG_ERR_* code.  amg_last_error() returns a
 *    message for the most recent failure on the calling thread.
 *  - "host" pointers point to CPU memory, "device" pointers to memory on the
 *    GPU that is current when amg_setup is called (e.g. torch CUDA tensors
 *    on ROCm).  The library never frees caller memory.
 *  - hip_stream is a hipStream_t (NULL = the default stream).  Work is
 *    enqueued on it; entry points that return numbers computed on the GPU
 *    synchronise that stream before returning.
 *  - A handle may be used from one thread at a time; calls on one handle
 *    that overlap on different streams race.
 */
#ifndef CAMG_H
#define CAMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define CAMG_OK 0
#define CAMG_NOT_CONVERGED 1
#define CAMG_ERR_INVALID_ARG (-1)      /* NULL / out-of-range argument         */
#define CAMG_ERR_SHAPE (-2)            /* block sizes or CSR structure invalid */
#define CAMG_ERR_NONFINITE (-3)        /* NaN/Inf in input or residual         */
#define CAMG_ERR_ZERO_DIAG (-4)        /* zero Jacobi / Atilde / Schur diagonal*/
#define CAMG_ERR_RANK_DEFICIENT_AGG (-5) /* null space rank-deficient on an aggregate */
#define CAMG_ERR_SINGULAR_COARSE (-6)  /* coarsest merged matrix singular      */
#define CAMG_ERR_HIP (-7)              /* HIP runtime error                    */
#define CAMG_ERR_OOM (-8)              /* device or host allocation failed     */
#define CAMG_ERR_UNMAPPED_MULTIPLIER (-9) /* multiplier coupled to no slave dof */
#define CAMG_ERR_TOO_LARGE (-10)       /* V-cycle work vectors exceed the no-allocation scratch */

typedef struct amg_handle amg_handle;

/* Compressed sparse row matrix (host pointers unless the problem says
 * device_ptrs = 1).  rowptr has nrows+1 entries
 * starting at 0; column indices are sorted and unique within each row;
 * nnz = rowptr[nrows] must be below 2^31.  An all-empty block (nnz = 0) may
 * pass NULL col/val. */
typedef struct {
  int64_t nrows, ncols, nnz;
  const int64_t* rowptr;
  const int32_t* col;
  const double* val;
} amg_csr;

/* Problem statement (Sec. 2.3 blocks; Sec. 4.2/4.3 interface data).  Its
 * arrays are host pointers, or device pointers with device_ptrs = 1 (then
 * amg_setup copies them to the host once, since the hierarchy is built
 * there; sizes always come from this structure).  Layout rules:
 *  - displacement dofs are node-major: dof = node * dim + component;
 *  - slave_dofs / master_dofs list the displacement dofs of the slave /
 *    master interface nodes (any order); a node is an interface node when
 *    one of its dofs is listed;
 *  - lm_node maps each multiplier dof to its pseudo-node (NULL: j / dim);
 *    the component of multiplier j is j % dim;
 *  - nullspace is n_u x n_ns, column-major (rigid-body modes for
 *    elasticity); NULL means the dim translations.
 * All data are copied; the caller may free them after amg_setup returns. */
typedef struct {
  int32_t dim;                 /* 2 or 3: dofs per displacement node      */
  amg_csr K, G, B, C;          /* n_u x n_u, n_u x n_l, n_l x n_u, n_l x n_l */
  int32_t n_slave, n_master;
  const int32_t* slave_dofs;
  const int32_t* master_dofs;
  const int32_t* lm_node;      /* optional, length n_l                    */
  int32_t n_ns;
  const double* nullspace;     /* optional, n_u * n_ns                    */
  int32_t device_ptrs;         /* 1: every array above is a device pointer on the
                                  current GPU (amg_setup only; amg_setup_host
                                  returns CAMG_ERR_INVALID_ARG)             */
} amg_problem;

/* Preconditioner options (defaults from amg_default_options). */
#define CAMG_ATILDE_ROWSUM_ABS 0 /* SIMPLEC lumping diag(sum_j |K_ij|)     */
#define CAMG_ATILDE_DIAG 1       /* diag(K)                                 */
#define CAMG_ATILDE_NODAL 2      /* nodal blocks K_ii + sum_j ||K_ij||_F I   */
#define CAMG_JACOBI_ATILDE 0     /* Jacobi prediction relaxes with Atilde   */
#define CAMG_JACOBI_DIAG 1       /* Jacobi prediction relaxes with diag(K)  */
#define CAMG_PREC_FP64 0         /* hierarchy, smoother, transfers in FP64  */
#define CAMG_PREC_MIXED 1        /* ... in FP32 inside the FP64 FGMRES      */
#define CAMG_PREC_MIXED_BF16 2   /* as MIXED, with the fine level's K stored in bfloat16 for the V-cycle
                                    when it has the sliced blocked-ELL layout (FP32 arithmetic: each
                                    value FP64 -> FP32 -> bfloat16, nearest even, widened on load); the
                                    outer operator keeps K in FP64 */
#define CAMG_SPMV_AUTO 0         /* K as sliced blocked-ELL on large levels */
#define CAMG_SPMV_CSR 1          /* K as CSR on every level                 */
#define CAMG_SPMV_BELL 2         /* K as sliced blocked-ELL on every level  */
#define CAMG_SPMV_FULL 4         /* flag (AUTO or BELL | FULL): a blocked-ELL K that equals its transpose
                                    exactly is kept in full, not in symmetric storage */
#define CAMG_PROLONG_TENTATIVE 0 /* displacement transfers: tentative (PA)  */
#define CAMG_PROLONG_SMOOTHED 1  /* ... smoothed aggregation (SA)           */
#define CAMG_SCHUR_DIAG 0        /* Schur diagonal: diag(B Atilde^-1 G - C) */
#define CAMG_SCHUR_L1 1          /* ... signed l1 row sums of that matrix   */
#define CAMG_SCHUR_BLOCK 2       /* ... its nodal diagonal blocks (block Jacobi) */
#define CAMG_COARSE_LU 0         /* coarsest level: merged dense LU inverse */
#define CAMG_COARSE_SIMPLE 1     /* ... CheapSIMPLE sweeps from zero        */
#define CAMG_SMOOTHER_SIMPLE 0   /* block smoother: CheapSIMPLE (Alg. 3 of Sec. 5.1.3) */
#define CAMG_SMOOTHER_UZAWA 1    /* inexact Uzawa (Sec. 5.1.1, Alg. 2)      */
#define CAMG_SMOOTHER_BRAESS_SARAZIN 2 /* cheap Braess-Sarazin (Sec. 5.1.2) */
typedef struct {
  int32_t max_levels;      /* >= 1; 1 = direct solve of the whole system  */
  int32_t max_coarse_rows; /* stop coarsening at or below this many rows   */
  int32_t nu_pre, nu_post; /* CheapSIMPLE sweeps before / after correction */
  int32_t jacobi_sweeps;   /* damped Jacobi sweeps in the prediction (>=1) */
  int32_t atilde;          /* CAMG_ATILDE_* (NODAL needs jacobi_diag = CAMG_JACOBI_ATILDE) */
  int32_t jacobi_diag;     /* CAMG_JACOBI_*                                */
  int32_t precision;       /* CAMG_PREC_*                                  */
  int32_t spmv_format;     /* CAMG_SPMV_* (storage of K on device); blocked-ELL levels whose K equals
                              its transpose bit for bit use symmetric storage unless CAMG_SPMV_FULL is set */
  int32_t graphs;          /* 1: capture the V-cycle once into a HIP graph and replay it */
  double jacobi_omega;     /* Jacobi damping                               */
  double simple_alpha;     /* block damping alpha (Alg. 3; see smoother), > 0 */
  /* Robustness settings for strong stiffness contrast (defaults keep the
   * plain method):
   * prolongator: CAMG_PROLONG_SMOOTHED smooths the displacement transfers,
   *   P = P_tent - sa_omega Atilde^-1 K P_tent (Sec. 3.1.2, prolongator
   *   smoothing; the weak-scaling settings use 4/3), with the lumped
   *   diagonal Atilde = diag(sum_j |K_ij|); multiplier transfers stay
   *   tentative.
   * schur / schur_sweeps: the correction step solves S delta = -r with
   *   S = B Atilde^-1 G - C by schur_sweeps undamped Jacobi sweeps from zero
   *   (1 = division by the diagonal), the diagonal chosen by CAMG_SCHUR_*.
   *   CAMG_SCHUR_BLOCK relaxes with the inverses of S's diagonal blocks over
   *   multiplier nodes (the bs_l multipliers of one node, consecutive; the
   *   problem's lm_node must map multiplier j to node j / dim): with Cartesian
   *   multipliers the normal and tangential constraint rows of a node mix its
   *   components wherever the interface normal is not a coordinate axis, and
   *   the diagonal alone can vanish there (the rotated two-body experiment of
   *   Sec. 6.1).  A singular node block is CAMG_ERR_ZERO_DIAG.
   * CAMG_ATILDE_NODAL replaces the point lumping by one block per node (bs_u
   *   dofs): A_i = K_ii + (sum over other nodes j of ||K_ij||_F) I, which
   *   bounds x^T K x from above for symmetric K as the row sums do, and
   *   transforms as R A_i R^T when the node frames rotate.  Its inverse
   *   blocks relax the prediction (block Jacobi), back-substitute and form
   *   S = B A^-1 G - C (and smooth the prolongator with CAMG_PROLONG_SMOOTHED);
   *   with CAMG_SCHUR_BLOCK every smoother is then covariant under a rigid
   *   rotation of the problem (the iteration counts do not depend on the
   *   angles).  The nodal sweep runs from generic kernels (block applies and
   *   separate products) rather than the fused point-diagonal ones. */
  int32_t prolongator;     /* CAMG_PROLONG_*                               */
  int32_t schur;           /* CAMG_SCHUR_*                                 */
  int32_t schur_sweeps;    /* 1..64                                        */
  double sa_omega;         /* prolongator smoothing factor, > 0            */
  /* Coarsest-level solver (the two variants of the weak-scaling study,
   * Sec. 6.2): CAMG_COARSE_LU merges the blocks and applies the explicit
   * inverse; CAMG_COARSE_SIMPLE runs coarse_sweeps CheapSIMPLE sweeps from
   * zero there (adjoint sweeps in the transposed cycle), with no merge and no
   * factorisation, so a singular coarsest matrix is no error. */
  int32_t coarse_solver;   /* CAMG_COARSE_*                                */
  int32_t coarse_sweeps;   /* 1..64                                        */
  /* Block smoother of every smoothing level (and of the CheapSIMPLE coarse
   * solver).  simple_alpha is its block damping alpha in all three cases
   * (the paper's CheapSIMPLE(0.8), CheapUzawa(0.7), CheapBraessSarazin(1.9)):
   * Uzawa damps both updates by alpha and has no back-substitution;
   * Braess-Sarazin predicts with one step of the lumped diagonal scaled by
   * alpha (jacobi_omega and jacobi_sweeps are not used) and solves with
   * S_a = B Atilde^-1 G / alpha - C. */
  int32_t smoother;        /* CAMG_SMOOTHER_*                              */
} amg_options;

/* FGMRES options. */
typedef struct {
  int32_t m;           /* restart length (Krylov vectors per cycle), 1..512 */
  int32_t max_iters;   /* total iteration limit                            */
  int32_t fixed_iters; /* > 0: run exactly this many iterations, ignore rtol */
  int32_t lookahead;   /* 1..7: the host reads each step's residual estimate this many
                          steps behind the launches, so the device never waits for the
                          host; steps launched past convergence are discarded */
  double rtol;         /* stop when ||b - A x|| <= rtol ||b - A x0||        */
  int32_t ortho;       /* Arnoldi orthogonalisation (m <= 63): 0 CGS2 with three passes over the
                          basis (dots, update + dots, update + norm); 1 (default) CGS2 with two
                          passes, the second projection's coefficients taken from the Gram matrix
                          of the basis (h2 = h1 - V^T V h1, V^T V built from the update pass's own
                          dots).  Equal in exact arithmetic; m > 63 always uses separate dot and
                          update kernels */
} amg_gmres_options;

typedef struct {
  int32_t iters, restarts, status;
  double rel_res_est;  /* |g_{j+1}| / ||r0|| from the Hessenberg recursion   */
  double rel_res_true; /* ||b - A x|| / ||r0||, recomputed at the end        */
  double seconds;      /* device time of the solve (hipEvents)               */
} amg_gmres_result;

typedef struct {
  int64_t n_u, n_l;
  int64_t nnz_K, nnz_G, nnz_B, nnz_C;
  int32_t bs_u, bs_l;     /* dofs per displacement node / multiplier node */
  int64_t n_nodes_u, n_nodes_l;
  int64_t n_agg_u, n_agg_l; /* aggregates built on this level (0 on the coarsest) */
  double op_complexity;   /* sum over levels of nnz / level-0 nnz (all blocks) */
  int32_t k_layout;       /* device storage of K: 0 CSR, 1 sliced blocked-ELL, 2 CSR plus a node-blocked
                             copy used by the row dots, 3 sliced blocked-ELL in symmetric storage (K = K^T
                             exactly: the blocks on and right of the block diagonal are stored, each block
                             left of it is read transposed from its mirror; it serves K and K^T)
                             (-1: host-only handle) */
  int32_t k_bs;           /* block size of the blocked layout                */
  int64_t k_blocks;       /* nonzero bs x bs blocks of K (blocked layouts)   */
  int64_t k_slots;        /* stored blocks including slice padding           */
  int32_t transfer_layout; /* P and R on device: 0 CSR, 1 tentative aggregate pattern without column
                              indices (per-row base column, dense row values, per-aggregate row lists);
                              -1 on the coarsest level or a host-only handle */
  int32_t k_index_bytes;  /* bytes per stored block-column index of the blocked layouts: 2 when the
                             columns are kept as 16-bit deltas from the row's node, else 4 (0: CSR
                             or host-only) */
  int64_t k_lower_blocks; /* symmetric storage: nonzero blocks left of the block diagonal, read through
                             their mirrors (each costs a 2-byte delta and a 2-byte mirror position) */
  int64_t k_nnz_stored;   /* entries of K held in the blocked layout's nonzero blocks (all of K's
                             nonzeros, or those on and right of the block diagonal) */
  int32_t k_sym_stale;    /* level 0: 1 after amg_update_fine_values gave K values that are not
                             symmetric; the FP64 kernels then use CSR copies of K and K^T */
} amg_level_info;

void amg_default_options(amg_options* opts);
void amg_default_gmres_options(amg_gmres_options* opts);

/* Builds the hierarchy (Sec. 4: displacement aggregation with slave/master
 * couplings dropped, multiplier aggregation by Alg. 1, tentative segregated
 * transfers, Galerkin blocks; Sec. 5.1.3 smoother data; dense LU of the
 * merged coarsest matrix) and uploads it to the current device.
 * On success *out owns all device memory of the hierarchy. */
int amg_setup(const amg_problem* prob, const amg_options* opts, void* hip_stream, amg_handle** out);

/* The same hierarchy construction on the host only, with no device upload
 * and no HIP call: the handle answers amg_num_levels, amg_level_info_get,
 * amg_get_aggregates and amg_get_level_matrix; device entry points return
 * CAMG_ERR_INVALID_ARG for it.  Release with amg_destroy. */
int amg_setup_host(const amg_problem* prob, const amg_options* opts, amg_handle** out);

int amg_num_levels(const amg_handle* h);
int amg_level_info_get(const amg_handle* h, int level, amg_level_info* out);

/* Aggregates of `level` (0 <= level < levels-1), host arrays:
 * disp_agg[n_nodes_u] (node -> aggregate, -1 for clamped nodes),
 * lm_agg[n_nodes_l] (multiplier pseudo-node -> aggregate of Alg. 1).
 * Either pointer may be NULL. */
int amg_get_aggregates(const amg_handle* h, int level, int32_t* disp_agg, int32_t* lm_agg);

/* Copies block `which` (0=K, 1=G, 2=B, 3=C, 4=P_u, 5=P_l, 6=S, the Schur
 * matrix B Atilde^-1 G - C kept when schur_sweeps > 1, else 0 x 0; 7=the
 * inverse nodal blocks of S as a block-diagonal matrix with CAMG_SCHUR_BLOCK,
 * 8=the inverse nodal lumping blocks with CAMG_ATILDE_NODAL, else 0 x 0) of
 * `level` to host arrays in FP64 (rowptr: nrows+1, col/val: nnz).  Call with
 * NULL arrays to query *nrows, *ncols, *nnz first. */
int amg_get_level_matrix(const amg_handle* h, int level, int which, int64_t* nrows, int64_t* ncols,
                         int64_t* nnz, int64_t* rowptr, int32_t* col, double* val);

/* Replaces the values of the level-0 blocks (device pointers, FP64, same
 * patterns and order as at setup; NULL keeps a block).  The outer FGMRES
 * operator and the FP64 level-0 smoother operator use the new values; the
 * coarse levels, the smoother diagonals, the Schur matrix and an FP32
 * level-0 copy keep the setup-time values (a fixed preconditioner for the
 * new operator).  When K is kept in symmetric blocked-ELL storage, new K
 * values are checked on the device (the call then waits for hip_stream): if
 * they are not symmetric, the FP64 kernels use CSR copies of K and K^T until
 * a later update is symmetric again (amg_level_info.k_sym_stale). */
int amg_update_fine_values(amg_handle* h, const double* K_val, const double* G_val, const double* B_val,
                           const double* C_val, void* hip_stream);

/* y = A x (transpose = 0) or y = A^T x on the level-0 operator; device
 * FP64 vectors of length n.  Asynchronous. */
int amg_apply_operator(amg_handle* h, int transpose, const double* x, double* y, void* hip_stream);

/* One V-cycle (Sec. 3.1.1, Fig. 2a, started from zero) as preconditioner:
 * z = M^-1 r (transpose = 0) or z = M^-T r, the exact transpose of the
 * forward cycle (adjoint sweeps, pre/post counts swapped, A_c^-T).  Device
 * FP64 vectors of length n; r and z must not overlap.  Asynchronous. */
int amg_vcycle_apply(amg_handle* h, int transpose, const double* r, double* z, void* hip_stream);

/* The V-cycle of amg_vcycle_apply for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels in the same order and the same result,
 * but it allocates nothing, captures no graph and times no kernel.  Its work
 * vectors (every level's right-hand side, iterates, residual, multiplier
 * increments and prediction buffers, in the precision of the hierarchy)
 * live in a fixed array of CAMG_NOALLOC_SCRATCH_BYTES per GPU, held from the
 * library's first amg_setup on that GPU until the process ends; the call
 * clears it with a fill kernel first (no memset node).  Problems whose work
 * vectors do not fit return CAMG_ERR_TOO_LARGE before anything is launched
 * (about 1.1M unknowns in FP64, 2.2M in mixed precision).  Every call on one
 * GPU shares that array: calls that overlap on one GPU (other streams, other
 * handles, other threads) race.  r, z: device FP64, length n, not
 * overlapping.  Asynchronous. */
#define CAMG_NOALLOC_SCRATCH_BYTES (64u << 20)
int amg_vcycle_apply_noalloc(amg_handle* h, int transpose, const double* r, double* z, void* hip_stream);

/* Right-preconditioned flexible GMRES(m) with CGS2 and Givens rotations,
 * one V-cycle per iteration (Sec. 3), on A (transpose = 0) or A^T.
 * b: device FP64 length n; x: device FP64 length n, initial guess on entry,
 * solution on exit.  Synchronises hip_stream.  res may be NULL. */
int fgmres_solve(amg_handle* h, int transpose, const double* b, double* x, const amg_gmres_options* gopts,
                 amg_gmres_result* res, void* hip_stream);

/* dK[k] = -lam_u[i] * x_u[j] for the k-th stored entry (i, j) of K in setup
 * order: the gradient of a scalar loss with respect to K's nonzeros, given
 * the forward solution x and the adjoint solution lam (device FP64, length
 * n).  dK: device FP64, nnz(K).  Asynchronous. */
int amg_grad_K(amg_handle* h, const double* lam, const double* x, double* dK, void* hip_stream);

/* The same outer product on every block of A = [[K, G], [B, C]]: for the
 * k-th stored entry (i, j) of a block, in setup order, d[k] = -lam_r[i] *
 * x_c[j], where lam_r is the row part of lam (lam_u for K and G, lam_l for B
 * and C) and x_c the column part of x (x_u for K and B, x_l for G and C).
 * That is dL/dA_ij = -lam_i x_j restricted to A's sparsity pattern, for x
 * solving A x = b and lam solving A^T lam = dL/dx (the differentiation of
 * the block system of Sec. 2.3 with respect to its stored entries).
 * lam, x: device FP64, length n.  dK, dG, dB, dC: device FP64 arrays of the
 * blocks' nnz; NULL skips a block.  Asynchronous. */
int amg_grad_A(amg_handle* h, const double* lam, const double* x, double* dK, double* dG, double* dB, double* dC,
               void* hip_stream);

/* Explicit inverse of a dense n x n FP64 matrix on the device: the
 * factorisation behind the coarsest-level direct solve (the coarse blocks
 * merged and factorised by LU, weak-scaling solver settings of Sec. 6.2),
 * which amg_setup runs on the merged coarsest matrix.  Blocked LU with
 * partial pivoting (largest magnitude, first row on ties) on 64-column
 * panels, then L U X = P by blocked substitution; every rank-64 update runs
 * on the FP64 matrix cores.  A, Ainv: device, row-major n x n, not
 * overlapping; 1 <= n <= 46000.  A pivot not above 1e-13 max |A_ij| returns
 * CAMG_ERR_SINGULAR_COARSE (Ainv undefined), a non-finite entry
 * CAMG_ERR_NONFINITE.  Allocates a workspace of two (n rounded up to 64)^2
 * FP64 matrices; synchronises hip_stream. */
int amg_dense_inverse(const double* A, double* Ainv, int64_t n, void* hip_stream);

/* Per-kernel timing with hipEvents around every launch of the selected
 * kernel classes (bit mask of CAMG_KCLASS_*), recorded on the stream the
 * kernel runs on.  amg_profile_read synchronises and returns the number of
 * timed launches and their summed duration in milliseconds. */
#define CAMG_KCLASS_SMOOTH_U 1   /* level-0 residual + Jacobi prediction (CSR) */
#define CAMG_KCLASS_OPERATOR 2   /* FP64 outer operator apply              */
#define CAMG_KCLASS_ORTHO 4      /* CGS2 GEMV passes                        */
#define CAMG_KCLASS_RESIDUAL 8   /* level-0 residual before restriction    */
int amg_profile_enable(amg_handle* h, int mask);
int amg_profile_read(amg_handle* h, int kclass, int64_t* launches, double* total_ms);

void amg_destroy(amg_handle* h);
const char* amg_strerror(int code);
const char* amg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CAMG_H */
