/*
 * nullspace.h -- C ABI of the MI355X null-space library.
 *
 * The library computes an orthonormal basis V (n x N) of the null space of a
 * large sparse A (m x n, CSR) with the randomized small-block Lanczos method
 * of Kressner & Shao, "On a randomized small-block Lanczos method for
 * large-scale null space computations": block Lanczos with block size d >= 1
 * on B = A^T A + eps D (Eq. "defB", Sec. 1.2), D a random diagonal with iid
 * U[0,1) entries and a Gaussian start block Omega (Alg. 1), thick restarts with
 * Ritz vectors (Sec. 4.1), partial reorthogonalisation monitored by the
 * W-recurrence (Sec. 4.2), adaptive nullity detection N = #{theta < 3 eps}
 * (Remark "cormain") and the convergence-speed stop (Alg. 2, Sec. 4.3).
 * B is applied matrix-free as y = A x, z = A^T y + eps D x (Sec. 1.2), with A^T
 * stored as its own CSR so the second product needs no atomics.
 *
 * Beyond the paper: an FP64 refinement of the Ritz basis (Rayleigh-Ritz with
 * the perturbation removed, as in the Remark after Alg. 1, then a projection
 * onto null(A) by range-restricted CGLS), a backward pass (gradient of a loss on
 * the null projector P = V V^T w.r.t. the stored values of A), and a mixed
 * precision mode.
 *
 * Conventions for every call:
 *  - Array arguments are DEVICE pointers (HIP, gfx950) owned by the caller,
 *    unless a comment says "host".  The library never frees caller memory.
 *  - Dense matrices are column-major with an explicit leading dimension.
 *  - All GPU work is ordered on the stream passed to nullspace_init.  Calls
 *    that return host data synchronise that stream before returning.
 *  - Every call returns an nsp_status; no C++ exception crosses the ABI.  On
 *    failure nullspace_last_error() returns a message for the calling thread.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef NULLSPACE_H
#define NULLSPACE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nsp_ctx nsp_ctx;

typedef enum {
  NSP_OK = 0,
  NSP_ERR_ARG = 1,       /* invalid argument (shape, pointer, parameter)            */
  NSP_ERR_HIP = 2,       /* a HIP / rocBLAS / rocSOLVER call failed                 */
  NSP_ERR_NOMEM = 3,     /* device allocation failed                                */
  NSP_ERR_STATE = 4,     /* call out of order (e.g. extract_basis before the solve) */
  NSP_ERR_NOCONV = 5,    /* matvec budget exhausted before the stopping rule fired;
                            the basis from the last cycle is still extractable      */
  NSP_ERR_BREAKDOWN = 6, /* a Lanczos block lost rank (invariant Krylov subspace)   */
  NSP_ERR_NONFINITE = 7  /* NaN/Inf met in the input or during the iteration        */
} nsp_status;

typedef enum {
  NSP_PREC_FP64 = 0,  /* everything in FP64                                          */
  NSP_PREC_MIXED = 1  /* FP32 SpMV, FP32 basis and reorthogonalisation; FP64 for the
                         T / Ritz eigenproblem, the Lanczos scalars, the refinement,
                         the residual check and the backward pass                    */
} nsp_precision;

typedef enum {
  NSP_OP_NORMAL = 0, /* B = A^T A + eps D (Eq. "defB"), any A                         */
  NSP_OP_SYM = 1     /* B = A + eps D for a symmetric positive semi-definite A (the
                        graph Laplacian experiments of Sec. 5.1): one product with A
                        per step, condition number not squared.  Requires m = n and
                        A stored with a symmetric pattern and equal mirrored values
                        (checked at init, NSP_ERR_ARG otherwise).  Semi-definiteness
                        is the caller's promise; the null space is then null(A).  */
} nsp_op;

typedef enum {
  NSP_PRECOND_NONE = 0,   /* Lanczos on B as given by op                              */
  NSP_PRECOND_JACOBI = 1, /* outer preconditioning (Sec. 4.4, "Outer preconditioning")
                             with the diagonal P_R = diag(p): Lanczos on
                             B_R = P_R^{-1} A^T A P_R^{-T} + eps D (NSP_OP_NORMAL,
                             p_j = ||A e_j||_2) or P_R^{-1} A P_R^{-T} + eps D
                             (NSP_OP_SYM, p_j = sqrt(A_jj)); p_j = 1 where that is
                             0.  The Lanczos basis approximates null(A P_R^{-T}) =
                             P_R^T null(A); V = P_R^{-T} V_R, orthonormalised, is
                             what extract_basis returns.  Undoes column scaling
                             exactly (A S has the same B_R as A for diagonal S > 0). */
  NSP_PRECOND_IC = 2      /* outer preconditioning with an incomplete Cholesky factor,
                             the preconditioner of the paper's Laplacian experiments
                             (Sec. 5.1): P_R = L, L L^T ~ M + ic_diagcomp diag(M)
                             with M = A (NSP_OP_SYM) or M = A^T A (NSP_OP_NORMAL,
                             formed on the host at init), factored on the host at
                             init in the library's order of the unknowns.  Every
                             application of B_R = L^{-1} A^T A L^{-T} + eps D (or
                             L^{-1} A L^{-T} + eps D) solves with L^T and L on the
                             device, level by level; V = L^{-T} V_R, orthonormalised.
                             NSP_ERR_ARG at init on a non-positive pivot (raise
                             ic_diagcomp) or a factor above 64 nnz(M) entries. */
} nsp_precond;

/* Solver parameters (host struct).  nsp_default_params() fills defaults. */
typedef struct {
  double eps;            /* perturbation strength eps > 0 (Eq. "defB"); the paper's
                            analysis needs eps < sigma_min(A)^2 / 3 (Thm. "thmmain") */
  int32_t d;             /* block size, 1..8                                         */
  int32_t max_dim;       /* dim K: maximum Krylov dimension, multiple of d, >= 3d    */
  int64_t max_matvec;    /* budget of single-vector B applications                   */
  double ro_tol;         /* reorthogonalisation threshold u_RO; 0 -> sqrt(u)          */
  int32_t prec;          /* nsp_precision                                            */
  int32_t refine;        /* 1: run the FP64 refinement after the Lanczos iteration   */
  double tol_rel_resid;  /* refinement target ||A V||_F <= this * ||A||_F; a column is
                            done once ||A v|| <= this * ||A||_F / sqrt(N)              */
  double tol_abs_resid;  /* absolute per-column target ||A v|| <= this                */
  double tol_angle;      /* target sine of the largest principal angle to null(A): a
                            column is done once ||A v|| <= this * s / (2 sqrt(N)),
                            s = sigma_min(A) estimated from the smallest Ritz value
                            above 3 eps: s^2 = theta_next - eps max(D) for
                            NSP_OP_NORMAL, s = theta_next - eps max(D) for NSP_OP_SYM.
                            The smallest threshold of the enabled (non-zero)
                            criteria applies.                                       */
  int64_t max_refine_iter; /* CGLS iteration cap of the refinement                   */
  int32_t max_cycles;    /* stop after this many restart cycles (0 = no limit)       */
  int32_t profile;       /* 1: time the SpMV pair and the reorthogonalisation pair
                            with HIP events on the library's stream at every 4th
                            Lanczos step (nsp_stats.t_spmv_*, ro_*)                  */
  int32_t reorder;       /* 1 (default): store A with rows and columns in a locality
                            order (breadth-first over the row/column graph, see
                            nullspace_locality_order) so the SpMV gathers stay in
                            cache; B is then P B P^T for a permutation P, the same
                            operator up to renumbering.  Every argument and result
                            of the API stays in the caller's order.  0: keep it.   */
  int32_t op;            /* nsp_op: operator form, NSP_OP_NORMAL by default           */
  int32_t precond;       /* nsp_precond: NSP_PRECOND_NONE by default. With
                            NSP_PRECOND_JACOBI, eps, the 3 eps nullity threshold,
                            ||B||, the Ritz values and apply_op refer to B_R, the
                            refinement works on A P_R^{-T}, and rel_resid_fro is
                            ||A V||_F / ||A||_F of the returned basis.               */
  uint64_t seed;         /* seed of the built-in Philox4x32-10 draws of D and Omega,
                            used only when the caller passes D or Omega as NULL       */
  double ic_droptol;     /* NSP_PRECOND_IC: > 0 drops the factor entries l_ij (i > j)
                            with |l_ij| < ic_droptol ||Mc(j:n, j)||_1, Mc = M +
                            ic_diagcomp diag(M) (threshold incomplete Cholesky);
                            0 keeps exactly the pattern of M (IC(0)).  Default 1e-3. */
  double ic_diagcomp;    /* NSP_PRECOND_IC: diagonal compensation alpha >= 0 (M +
                            alpha diag(M) is factored).  Default 0.1.               */
} nsp_params;

/* Statistics of the last lanczos_run (host struct). */
typedef struct {
  int32_t nullity;         /* N: number of Ritz values below 3 eps at the end         */
  int32_t converged;       /* 1 if the convergence-speed rule stopped the iteration   */
  int32_t restarts;        /* number of thick restarts                                */
  int32_t cycles;          /* number of Rayleigh-Ritz extractions                     */
  int64_t matvecs;         /* single-vector applications of B                          */
  int64_t reorths;         /* partial reorthogonalisation events                       */
  int64_t refine_iters;    /* CGLS iterations of the refinement                        */
  double norm_b;           /* ||B|| estimate used in u_d                               */
  double theta_last;       /* largest Ritz value below 3 eps                           */
  double theta_next;       /* smallest Ritz value at or above 3 eps                    */
  double rel_resid_fro;    /* ||A V||_F / ||A||_F after refinement (FP64)               */
  double orth_err_fro;     /* ||V^T V - I||_F                                           */
  double t_total_s;        /* wall time of lanczos_run                                  */
  double t_lanczos_s;      /* time in the Lanczos steps (device events)                 */
  double t_restart_s;      /* time in Rayleigh-Ritz + restarts                          */
  double t_refine_s;       /* time in the refinement                                    */
  double t_spmv_a_us;      /* profile: mean duration of one y = A x launch (us)         */
  double t_spmv_at_us;     /* profile: mean duration of one fused A^T launch (us)       */
  int64_t spmv_samples;    /* profile: number of timed launch pairs                     */
  double ro_tn_ms;         /* profile: summed duration of the sampled projection
                              launches H = Z^T [Q_l, Q_l+1] (partials per row chunk)
                              at steps that reorthogonalised, ms                      */
  double ro_tn_bytes;      /* ... their algorithmic bytes, (k n + 2 d n) elements each */
  double ro_nn_ms;         /* profile: same for the updates [Q_l, Q_l+1] -= Z H, ms   */
  double ro_nn_bytes;      /* ... (k n + 4 d n) elements each                          */
  double ro_idle_ms;       /* profile: summed duration of the sampled projection plus
                              update launches at steps whose flag was clear (they
                              return at once), ms                                    */
  int64_t ro_samples;      /* profile: number of sampled steps                         */
  int64_t ro_active;       /* profile: how many of them reorthogonalised               */
  int64_t refine_defl;     /* Ritz vectors deflating the refinement's CGLS (0: none)  */
} nsp_stats;

/* Fill *p with defaults: eps = 1e-3 (Sec. 5.3), d = 1, max_dim = 64,
   max_matvec = 10^7, ro_tol = 0, prec = FP64, refine = 1, tol_rel_resid = 1e-10,
   tol_abs_resid = 0, tol_angle = 1e-9, max_refine_iter = 10^6, max_cycles = 0,
   profile = 0, reorder = 1, op = NSP_OP_NORMAL, precond = NSP_PRECOND_NONE,
   seed = 20240704, ic_droptol = 1e-3, ic_diagcomp = 0.1 (the drop tolerance and
   compensation of the incomplete Cholesky in Sec. 5.1). */
void nsp_default_params(nsp_params* p);

/* Create a solver context for A (m x n, nnz stored entries, CSR).
 *  rowptr  [m+1] int64, device; rowptr[0] = 0, non-decreasing, rowptr[m] = nnz.
 *  colind  [nnz] int32, device; 0 <= colind < n.
 *  vals    [nnz] float64, device; copied into the library's own (reordered)
 *          copies of A and A^T during the call.
 *  D       [n] float64, device or NULL: the perturbation diagonal (entries in
 *          [0,1]); NULL -> drawn with Philox4x32-10 (Salmon et al., SC'11):
 *          (x0, x1, x2, x3) = Philox4x32-10(counter (i, 0, 0, 0), key
 *          (seed mod 2^32, seed >> 32)), D_i = u53(x0, x1) with
 *          u53(a, b) = ((a >> 5) 2^26 + (b >> 6)) 2^-53 in [0, 1).  Copied.
 *  Omega   [n x d] float64 column-major (ld = n), device or NULL: the Gaussian
 *          start block; NULL -> Box-Muller on the same generator with counter
 *          (i, j + 1, 0, 0) for column j: Omega(i, j) =
 *          sqrt(-2 ln(1 - u53(x0, x1))) cos(2 pi u53(x2, x3)).  Copied.
 *          Both are drawn in the caller's order of the unknowns.
 *  p       host parameters (copied).
 *  stream  hipStream_t to order all work on (NULL = default stream).
 * Builds the transposed CSR (A^T) once.  nnz must be < 2^31.
 * Errors: NSP_ERR_ARG (shape, NULL pointer, bad parameter, colind out of range),
 *         NSP_ERR_NOMEM, NSP_ERR_HIP.  On error *out is NULL. */
nsp_status nullspace_init(nsp_ctx** out, int64_t m, int64_t n, int64_t nnz,
                          const int64_t* rowptr, const int32_t* colind, const double* vals,
                          const double* D, const double* Omega, const nsp_params* p,
                          void* stream);

/* Y = B X for ncols >= 1 columns: A^T (A X) + eps D X (Sec. 1.2), or
 * A X + eps D X with NSP_OP_SYM; with NSP_PRECOND_JACOBI the preconditioned
 * operator B_R the solver iterates with.
 *  X [n x ncols], ld ldx >= n; Y [n x ncols], ld ldy >= n; device, FP64.
 *  Uses the FP64 values regardless of the precision mode.  X and Y must not
 *  overlap.  Allowed in any state after init. */
nsp_status apply_op(nsp_ctx* ctx, const double* X, int64_t ldx, double* Y, int64_t ldy,
                    int32_t ncols);

/* apply_op without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and errors as apply_op, computed by the
 * same kernels; its scratch (X in the library's order, A X and B X: 3 n + m
 * doubles per column) lives in a 64 MiB device array of the library, one per
 * device, held until the process ends and shared by every call on that
 * device.  Columns go in chunks of 8, 4, 2 or 1 as they fit; a matrix whose
 * single column needs more than 64 MiB (3 n + m > 8 Mi) is rejected with
 * NSP_ERR_ARG.  Calls that overlap in time on one device (other contexts or
 * streams) race on the array and must be serialised by the caller.  The
 * stream synchronisation at the end is the same as apply_op's. */
nsp_status apply_op_noalloc(nsp_ctx* ctx, const double* X, int64_t ldx, double* Y, int64_t ldy,
                            int32_t ncols);

/* Run Algorithm 2 (Sec. 4.3) and, if p->refine, the FP64 refinement.
 *  st  host, may be NULL.
 * Returns NSP_OK, or NSP_ERR_NOCONV when the budget ran out (the basis of the
 * last cycle is kept and extractable), NSP_ERR_BREAKDOWN, NSP_ERR_NONFINITE,
 * NSP_ERR_HIP.  May be called again to re-solve (the state is reset). */
nsp_status lanczos_run(nsp_ctx* ctx, nsp_stats* st);

/* Nullity N found by the last lanczos_run (host out). */
nsp_status nullspace_nullity(nsp_ctx* ctx, int32_t* nullity);

/* Copy V (n x N, FP64, orthonormal columns) into V [ldv >= n], device: the
 * output of Alg. 2 ("Return V = Z_ell V_Z(:, 1:N_ell)", an orthonormal basis
 * approximating null(A)), after the FP64 refinement when params.refine is set
 * and mapped back by P_R^{-T} with outer preconditioning (Sec. 4.4), in the
 * caller's order of the unknowns.
 * Errors: NSP_ERR_STATE before a successful (or NOCONV) lanczos_run. */
nsp_status extract_basis(nsp_ctx* ctx, double* V, int64_t ldv);

/* Ritz values of the last Rayleigh-Ritz extraction, ascending (host out).
 *  theta  host buffer of capacity cap; *count receives the number written
 *  (min(cap, dim K)).  Before refinement, i.e. eigenvalues of T_ell. */
nsp_status nullspace_ritz_values(nsp_ctx* ctx, double* theta, int32_t cap, int32_t* count);

/* Residual norms of the Ritz pairs of the last Rayleigh-Ritz extraction, in
 * the order of nullspace_ritz_values (host out).  The Lanczos decomposition
 * B Z = Z T + Q_{ell+1} [0, Gamma_ell] (Eq. "laniter", with the arrowhead T
 * of Eq. "defT" after a restart) gives the Ritz pair (theta_i, Z V_Z(:, i))
 * the residual Q_{ell+1} Gamma_ell V_Z(last d rows, i); the value returned is
 * its norm ||Gamma_ell V_Z(last d rows, i)||, the usual convergence measure
 * (Sec. 4.1: the coupling block F of the kept pairs is made of these rows).
 *  res  host buffer of capacity cap; *count receives min(cap, dim K).
 * Errors: NSP_ERR_ARG for NULL pointers. */
nsp_status nullspace_ritz_residuals(nsp_ctx* ctx, double* res, int32_t cap, int32_t* count);

/* Wall time of each restart cycle of the last lanczos_run, in order (host
 * out): one cycle of Alg. 2's outer loop = the block Lanczos steps from
 * ell_0 + 1 to dim K / d with their partial reorthogonalisation, the
 * Rayleigh-Ritz step on T (Eq. "defT") and the thick restart (Sec. 4.1), or
 * the extraction of V after the last one.  Each interval runs from one
 * synchronisation of the library's stream to the next (host clock).
 *  seconds  host buffer of capacity cap; *count receives min(cap, cycles).
 * Errors: NSP_ERR_ARG for NULL pointers. */
nsp_status nullspace_cycle_times(nsp_ctx* ctx, double* seconds, int32_t cap, int32_t* count);

/* Eigen-decomposition of the restart matrix of Alg. 2 for block size 1
 * (Eq. "defT"), the Rayleigh-Ritz step the solver runs once per restart:
 *     T = [diag(theta)  f      0 ...      ]
 *         [f^T          alpha0 beta0      ]
 *         [0            beta0  alpha1 ... ]   (tridiagonal below the arrow tip)
 * of order K >= 2 with 0 <= kk <= K-2 kept Ritz values.
 *  theta  [kk] ascending, f [kk], alpha [K-kk], beta [K-kk-1]: device, FP64.
 *  evals  [K] out, ascending; evecs [K x K] out, column-major (ld K), device.
 * Exposed so the structured solver can be tested on its own; it runs on the
 * context's stream and synchronises.  Errors: NSP_ERR_ARG, NSP_ERR_HIP. */
nsp_status nullspace_ritz_eig(nsp_ctx* ctx, int32_t K, int32_t kk, const double* theta,
                              const double* f, const double* alpha, const double* beta,
                              double* evals, double* evecs);

/* The same for block size d (Eq. "defT"):
 *     T = [diag(theta)  F^T     0        ...]
 *         [F            Xi_1    Gamma_1^T   ]
 *         [0            Gamma_1 Xi_2     ...]   (block tridiagonal below)
 * with K/d - kk/d diagonal blocks Xi_j (symmetric d x d) and the couplings
 * Gamma_j = T(block j+1, block j) (d x d) between consecutive ones.
 *  d      1, 2, 4 or 8, dividing K and kk; kk = 0 or kk <= K - 2d; K <= 4096.
 *  theta  [kk] ascending; F [d x kk] column-major (ld d);
 *  xi     [(K-kk)/d blocks of d x d], each column-major, first block first;
 *  gam    [(K-kk)/d - 1 blocks of d x d] (may be NULL when there is one block);
 *  evals  [K] out, ascending; evecs [K x K] out, column-major; all device FP64.
 * The solver tears each coupling by its SVD into d rank-one updates (block
 * divide and conquer) and treats the kept part as d chained arrowheads.
 * Runs on the context's stream and synchronises.  Errors: NSP_ERR_ARG,
 * NSP_ERR_HIP. */
nsp_status nullspace_ritz_eig_blocks(nsp_ctx* ctx, int32_t K, int32_t d, int32_t kk, const double* theta,
                                     const double* f, const double* xi, const double* gam, double* evals,
                                     double* evecs);

/* New values of A for the same sparsity pattern (optimisation loops that
 * change A between solves).  vals [nnz] float64, device, in the caller's CSR
 * order of nullspace_init; copied during the call.  Reuses the locality order,
 * the stored transpose and the value permutations built at init (no host
 * work), then redoes what init does with values: the NSP_OP_SYM value check,
 * the FP32 copies, the norms and the Jacobi P_R.  D, Omega and the parameters
 * stay.  The previous basis is dropped: extract_basis and backward need a new
 * lanczos_run.  Errors: NSP_ERR_ARG (NULL, or asymmetric values with
 * NSP_OP_SYM), NSP_ERR_NONFINITE (a NaN or Inf value); apply_op and
 * lanczos_run then return NSP_ERR_STATE until a call with valid values. */
nsp_status nullspace_update_values(nsp_ctx* ctx, const double* vals);

/* Backward pass for a loss L(P) of the null projector P = V V^T (the
 * problem statement's null space, Sec. 1), with V from extract_basis.  The
 * loss must depend on V only through P (V is unique up to a rotation of its
 * columns); N is held fixed, so the derivative is that of the projector onto
 * the N smallest right singular vectors of A.
 *  dLdV       [n x N], ld >= n, device: dL/dV, the gradient of the loss with
 *             respect to the returned basis.  For such a loss dL/dV = 2 G_s V
 *             with G_s the symmetric part of dL/dP; the library uses
 *             G_s V = dL/dV / 2.
 *  grad_vals  [nnz], device, out: dL/d vals in A's CSR order,
 *             grad_p = -2 <(A W)_i, V_j> for the stored entry p = (i, j), where
 *             W = (A^T A)^+ (I - V V^T) G_s V is computed by CG on A^T A
 *             restricted to range(A^T), for the range of the right-hand side
 *             only (its directions with singular values above 3e-7 of the
 *             largest), deflated by the Ritz vectors the refinement used.
 *  tol        relative CG residual target per column (e.g. 1e-10).  With
 *             deflation the attainable level is about 1e-12: smaller values
 *             are raised to 1e-12.
 *  max_iter   CG iteration cap; the call returns NSP_ERR_NOCONV if reached.
 *             A run whose largest relative residual has not dropped by 1%
 *             within 4096 iterations has reached its attainable level (the
 *             null-space component of the residual is removed only to the
 *             accuracy of V) and ends there with NSP_OK.
 *  iters      host out (nullable): CG iterations used.
 * With NSP_PRECOND_JACOBI (normal form) the CG runs on the preconditioned
 * normal equations: A W = (A P_R^{-T}) X with (A P_R^{-T})^T (A P_R^{-T}) X =
 * P_R^{-1} (I - V V^T) G_s V, which gives the same A W.  NSP_ERR_ARG for the
 * preconditioned symmetric form. */
nsp_status backward(nsp_ctx* ctx, const double* dLdV, int64_t ld, double* grad_vals, double tol,
                    int64_t max_iter, int64_t* iters);

/* Release everything the context owns.  NULL is accepted. */
void nullspace_destroy(nsp_ctx* ctx);

/* The locality order nullspace_init uses when params.reorder = 1 (host only,
 * no GPU needed).  Breadth-first search over the bipartite graph of A's rows
 * and columns, started from the lowest-numbered unvisited column; columns are
 * numbered in the order the search reaches them and rows in the order they are
 * first met, rows without entries last.  Every connected piece of the graph
 * therefore occupies contiguous ranges of rows and columns.
 *   rowptr   : host, m + 1 int64 (CSR, rowptr[0] = 0, non-decreasing)
 *   colind   : host, rowptr[m] int32 in [0, n)
 *   row_order: host, m int32 out; row_order[r] is the caller's row at position r
 *   col_order: host, n int32 out; col_order[j] is the caller's column at position j
 * Errors: NSP_ERR_ARG for NULL pointers, sizes outside [1, 2^31) or an invalid
 * CSR. */
nsp_status nullspace_locality_order(int64_t m, int64_t n, const int64_t* rowptr,
                                    const int32_t* colind, int32_t* row_order,
                                    int32_t* col_order);

/* Message describing the last error on the calling thread ("" if none). */
const char* nullspace_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* NULLSPACE_H */
