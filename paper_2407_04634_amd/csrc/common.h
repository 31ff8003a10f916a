// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "nullspace.h"

namespace nsp {

// ---------------------------------------------------------------------------
// error handling: internal code throws nsp::Error, the C ABI converts it
// ---------------------------------------------------------------------------
struct Error : std::runtime_error {
  nsp_status code;
  Error(nsp_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define NSP_HIP(call)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (call);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw ::nsp::Error(e_ == hipErrorOutOfMemory ? NSP_ERR_NOMEM : NSP_ERR_HIP,         \
                         std::string(#call) + ": " + hipGetErrorString(e_));              \
  } while (0)

#define NSP_BLAS(call)                                                                    \
  do {                                                                                    \
    rocblas_status s_ = (call);                                                           \
    if (s_ != rocblas_status_success)                                                     \
      throw ::nsp::Error(NSP_ERR_HIP, std::string(#call) + ": rocblas status " +          \
                                          std::to_string((int)s_));                       \
  } while (0)

#define NSP_REQUIRE(cond, msg)                                                            \
  do {                                                                                    \
    if (!(cond)) throw ::nsp::Error(NSP_ERR_ARG, msg);                                    \
  } while (0)

// ---------------------------------------------------------------------------
// device buffer owned by the context
// ---------------------------------------------------------------------------
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  ~DBuf() { release(); }
  void alloc(size_t b) {
    if (b <= bytes && p) return;
    release();
    if (b == 0) return;
    NSP_HIP(hipMalloc(&p, b));
    bytes = b;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <typename T> T* as() const { return static_cast<T*>(p); }
};

constexpr int kMaxD = 8;            // largest supported block size
constexpr int kRedBlocks = 512;     // grid cap of kernels that write per-block partials
constexpr int kWideBlocks = 1024;   // grid cap of the many-column SpMM (its partials: x k)
constexpr int kDeflMax = 384;       // deflation vectors of the refinement (at most)
constexpr int kXcds = 8;            // accelerator complex dies; workgroups go round-robin over them
constexpr int kStreamBlocks = 2048; // grid cap of the streaming SpMV
constexpr int64_t kStreamMinNnz = 1 << 21;  // smaller matrices use the lanes-per-row kernels
constexpr int kThreads = 256;       // threads per block of streaming kernels

// ---------------------------------------------------------------------------
// the context
// ---------------------------------------------------------------------------
struct Csr {
  int64_t rows = 0, cols = 0, nnz = 0;
  const int32_t* rowptr = nullptr;  // int32 offsets (device)
  const int32_t* colind = nullptr;
  const double* val = nullptr;
  const float* val32 = nullptr;
  int lpr = 1;                      // lanes per row chosen from the mean row length
  // row blocks of the streaming kernels (each at most stream_tile(d) nonzeros,
  // or one longer row), built at init for the solver's block size d
  const int32_t* rblk = nullptr;
  int nrb = 0;
  int rblk_d = 0;
};

// nonzeros per row block of the streaming SpMV for a block of d columns
constexpr int stream_tile(int d) { return 2048 / d; }

// one triangular factor stored for a level-scheduled solve: CSR (int32), the
// rows grouped by level (perm), level boundaries on the host
struct TriSolve {
  DBuf rowptr, colind, val, perm;
  std::vector<int32_t> levptr;
  int64_t nnz = 0;
};
// incomplete Cholesky P_R = L: L by rows (forward solves) and L^T by rows (backward)
struct IcFactor {
  TriSolve fwd, bwd;
  int64_t m_nnz = 0;       // entries of the factored matrix M
  double norm_bound = 0.0; // estimate of ||B_R - eps D|| (power iteration, with a margin)
};

// pinned host buffer for the small read-backs (hipHostMalloc, grown on demand)
template <typename T>
struct PinBuf {
  T* p = nullptr;
  size_t count = 0;
  PinBuf() = default;
  PinBuf(const PinBuf&) = delete;
  PinBuf& operator=(const PinBuf&) = delete;
  ~PinBuf() { release(); }
  T* ensure(size_t n) {
    if (n <= count && p) return p;
    release();
    NSP_HIP(hipHostMalloc((void**)&p, sizeof(T) * n, hipHostMallocDefault));
    count = n;
    return p;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    count = 0;
  }
};

}  // namespace nsp

struct nsp_ctx {
  int64_t m = 0, n = 0, nnz = 0;
  int device = 0;                     // the device that was current at nullspace_init
  nsp_params prm{};
  hipStream_t stream = nullptr;       // the library's own non-blocking stream (all work)
  hipStream_t user_stream = nullptr;  // the caller's stream; ordered by events at each call
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  rocblas_handle blas = nullptr;
  nsp::PinBuf<double> pind;           // pinned read-back buffers
  nsp::PinBuf<int> pini;
  double* pin_d = nullptr;            // = pind.p, at least max_dim + 16 doubles
  int* pin_i = nullptr;               // = pini.p, at least 64 ints

  // A (own copy, int32 row offsets, see prepare_matrix) and its stored transpose
  nsp::Csr A, AT;
  nsp::DBuf rowptr32, rowptrT, colindT, valsT, permT, vals32, valsT32;
  // the library's own copy of A in the locality order (or the caller's order)
  nsp::DBuf colindA, valsA;
  nsp::DBuf permA;          // position in the stored A -> position in the caller's arrays
  nsp::DBuf rblkA, rblkT;   // row blocks of A and A^T for the streaming SpMV
  nsp::DBuf colperm;        // stored column (unknown) i -> caller's column colperm[i]
  bool reordered = false;
  double normA_fro = 0.0;
  double normA1_inf = 0.0;  // ||A||_1 * ||A||_inf
  double normA_inf = 0.0;   // ||A||_inf (bounds ||A||_2 when A is symmetric)
  bool sym = false;         // B = A + eps D (NSP_OP_SYM)
  // outer preconditioning with P_R = diag(pdiag) (NSP_PRECOND_JACOBI): the stored
  // values are those of A P_R^{-T} (or P_R^{-1} A P_R^{-T}); normA_fro is then the
  // norm of that matrix and normA_fro_orig the caller's ||A||_F
  bool precond = false;
  nsp::DBuf pdiag;          // p in the library's order of the unknowns
  // NSP_PRECOND_IC: the stored values stay those of A; every application of
  // B_R solves with L^T and L (precond_ic.hip)
  bool precond_ic = false;
  nsp::IcFactor ic;
  nsp::DBuf ic_tmp;         // n x d working-precision block of the Lanczos step
  nsp::DBuf ic_wide, ic_dots;  // n x k FP64 block and dot partials of the wide products
  double normA_fro_orig = 0.0;
  double maxD = 1.0;        // max of the perturbation diagonal

  // perturbation diagonal and start block
  nsp::DBuf Dv, omega;

  // Lanczos state (working precision: 8 or 4 bytes per element)
  int esize = 8;
  int64_t ldz = 0;          // leading dimension of the basis (>= n, padded)
  nsp::DBuf Z, Z2;          // basis, n x (K + d), column-major; Z2 for the restart
  nsp::DBuf ring;           // 3 row-interleaved copies of consecutive blocks (d > 1)
  nsp::DBuf Y;              // m x d, row-interleaved, working precision
  nsp::DBuf P;              // n x d, row-interleaved, working precision
  nsp::DBuf theta_kept;     // K Ritz values kept at the last restart
  nsp::DBuf fmat;           // d x K coupling block F
  nsp::DBuf tmat, evals, ework; // T (K x K), eigenvalues, rocSOLVER E workspace
  nsp::DBuf flags;          // device ints: [0] reorth flag, [1] breakdown, [2] nonfinite,
                            // [3] reorth event counter
  nsp::DBuf part_xi, part_g, part_g2, part_c;  // per-block partials of the step reductions

  // result
  nsp::DBuf V;              // n x N column-major FP64 (final basis)
  nsp::DBuf Vs;             // preconditioned runs: orthonormal basis of null(A P_R^{-T})
  nsp::DBuf Wd;             // n x defl_r column-major FP64: the Ritz vectors just above
  int32_t defl_r = 0;       // the null cluster, deflation space of the refinement
  // the deflation space after its Rayleigh-Ritz rotation with A^T A (W^T A^T A W =
  // Lambda), row-major blocks: W, Ws = W Lambda^-1, MWs = A^T A W Lambda^-1 (n x df_r),
  // AW, AWs = A W Lambda^-1 (m x df_r); shared by the refinement and backward
  nsp::DBuf dfW, dfWs, dfMWs, dfAW, dfAWs;
  int32_t df_r = 0;
  int32_t nullity = 0;
  int state = 0;            // 0 = initialised, 1 = basis available
  bool values_ok = true;    // false after a rejected nullspace_update_values
  std::vector<double> ritz; // last Ritz values (host)
  std::vector<double> ritz_res; // their Lanczos residual norms (host)
  std::vector<double> cycle_s; // wall time of each restart cycle of the last solve (host)
  nsp_stats stats{};
};

namespace nsp {

// launchers implemented in kernels_*.hip -----------------------------------
void prepare_matrix(nsp_ctx* c, const int64_t* rowptr64, const int32_t* colind, const double* vals);
// Locality order of A (host arrays): breadth-first search over the bipartite
// row/column graph; row_order[r] / col_order[j] give the caller's row / column
// placed at position r / j.  Connected pieces come out contiguous.
void locality_order(int64_t m, int64_t n, const int64_t* rowptr, const int32_t* colind,
                    int32_t* row_order, int32_t* col_order);
// dst(i, j) = src(idx[i], j) (gather) or dst(idx[i], j) = src(i, j) (scatter),
// column-major FP64; idx == nullptr is the identity
void gather_rows(nsp_ctx* c, int64_t n, int ncols, const int32_t* idx, const double* src,
                 int64_t lds, double* dst, int64_t ldd);
void scatter_rows(nsp_ctx* c, int64_t n, int ncols, const int32_t* idx, const double* src,
                  int64_t lds, double* dst, int64_t ldd);
// dst[permA[p]] = src[p] over the nonzeros (results per stored nonzero back to
// the caller's order)
void scatter_vals(nsp_ctx* c, const double* src, double* dst);
void init_random(nsp_ctx* c, const double* D, const double* Omega);
double matrix_norms(nsp_ctx* c);
// NSP_PRECOND_JACOBI: p from the stored matrix, stored values -> those of the
// preconditioned matrix (FP32 copies included); call after matrix_norms
void precondition(nsp_ctx* c);
// NSP_PRECOND_IC (precond_ic.hip): factor M = A or A^T A, store L for the solves
void ic_setup(nsp_ctx* c);
// in-place solves L y = b / L^T y = b on a row-major n x k block
template <typename VT> void ic_solve_l(nsp_ctx* c, int k, VT* y);
template <typename VT> void ic_solve_lt(nsp_ctx* c, int k, VT* y);
// y += eps D x on row-major n x k FP64 blocks
void add_eps_dx(nsp_ctx* c, int k, const double* x, double* y);
// P += eps D X - Xp Gamma_prev^T with Xi = X^T P partials (the Lanczos step's
// epilogue when B is not applied by the fused products); returns the count
template <typename VT>
int step_epilogue(nsp_ctx* c, int d, const VT* x, const VT* xp, const double* gprev, VT* p,
                  double* part_xi);
void check_symmetric_values(nsp_ctx* c);
void copy_f32(nsp_ctx* c);
// nullspace_update_values: new values, same pattern (caller's order)
void refresh_values(nsp_ctx* c, const double* vals);

// apply_op helper: Y = B X (FP64, column-major, ld)
void apply_b_colmajor(nsp_ctx* c, const double* X, int64_t ldx, double* Y, int64_t ldy, int ncols);
// the same with caller-provided scratch: chunks of at most wmax (<= kMaxD)
// columns, xc / xr / zr of n * wmax doubles and yr of m * wmax doubles
void apply_b_chunks(nsp_ctx* c, const double* X, int64_t ldx, double* Y, int64_t ldy, int ncols,
                    int wmax, double* xc, double* xr, double* yr, double* zr);
// allocation-free apply_op (noalloc.hip): the scratch lives in a file-scope
// device array; noalloc_setup resolves its address on the current device
void noalloc_setup();
void apply_b_noalloc(nsp_ctx* c, const double* X, int64_t ldx, double* Y, int64_t ldy, int ncols);

// Lanczos solve (solver.hip)
void solve(nsp_ctx* c);
void run_backward(nsp_ctx* c, const double* dLdV, int64_t ld, double* grad, double tol,
                  int64_t max_iter, int64_t* iters);

}  // namespace nsp
