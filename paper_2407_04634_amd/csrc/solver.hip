// Host driver of Algorithm 2 (Sec. 4.3) with device-resident state, the FP64
// refinement, and the backward pass.
//
// Readings of the paper used here (same as the design notes):
//  R1  restart keeps k_keep = d * floor((N_ell + K) / (2d)) vectors, clamped to
//      [d, K - 2d];
//  R2  the recurrence subtracts Q_{ell-1} Gamma_{ell-1}^T;
//  R3/R4 the W-recurrence cases (see k_wrec);
//  R5  partial reorthogonalisation = one classical Gram-Schmidt pass, accepted
//      by the Kahan-Parlett criterion (each unit column keeps >= 1/sqrt(2) of
//      its norm; checked on the device, a violation stops the run); the
//      cycle's first step and the restart use two passes;
//  R6  QR = Cholesky QR (twice for d > 1), positive diagonal;
//  R7  ||B|| = ||A||_1 ||A||_inf + eps max(D) in the first cycle, then the
//      largest Ritz value;
//  R8  u = 2^-52 (FP64) or 2^-23 (FP32 working precision), u_RO = sqrt(u);
//  R9  Frobenius norms of the blocks in the W-recurrence;
//  R10 convergence-speed stop;
//  R11 F = R Gamma_ell V_Z(last d rows, 1:k_keep);
//  R12 with N_ell = 0, stop once the smallest Ritz value has converged above
//      3 eps (nothing_below_rule).
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <limits>
#include <memory>

#include "common.h"
#include "kernels.h"

namespace nsp {

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int restart_size(int n_ell, int K, int d) {
  int kk = d * ((n_ell + K) / (2 * d));
  return std::min(std::max(kk, d), K - 2 * d);
}

// Reading R10: speed s = matvecs per d newly converged Ritz values, sampled
// over intervals (starting at the first increase of N_ell) that close once
// N_ell has grown by at least d; stop when more than 2 max(samples) matvecs
// passed since the last increase.
bool speed_rule(const std::vector<std::pair<int64_t, int>>& hist, int d) {
  std::vector<std::pair<int64_t, int>> ev;
  int best = 0;
  for (auto& h : hist)
    if (h.second > best) { ev.push_back(h); best = h.second; }
  if (ev.empty()) return false;
  double s = 0.0;
  bool have = false;
  auto start = ev[0];
  for (size_t i = 1; i < ev.size(); ++i)
    if (ev[i].second - start.second >= d) {
      s = std::max(s, (double)(ev[i].first - start.first) * d / (ev[i].second - start.second));
      start = ev[i];
      have = true;
    }
  if (!have) return false;
  return (double)(hist.back().first - ev.back().first) > 2.0 * s;
}

// Reading R12: with no Ritz value below 3 eps the speed rule never gets a
// sample.  Sec. 4.3 names the simpler stopping idea of ending once an
// unwanted Ritz value above 3 eps has converged; used for that case only:
// stop when N_ell = 0 and the smallest Ritz value theta_1 has a residual
// r_1 <= eps with theta_1 - r_1 >= 3 eps (some eigenvalue of B lies in
// [theta_1 - r_1, theta_1 + r_1], above the nullity threshold).
bool nothing_below_rule(const std::vector<double>& theta, const std::vector<double>& res, double eps) {
  if (theta.empty() || res.size() != theta.size() || theta[0] < 3.0 * eps) return false;
  return res[0] <= eps && theta[0] - res[0] >= 3.0 * eps;
}

template <typename T> T* alloc_as(DBuf& b, size_t count) {
  b.alloc(sizeof(T) * std::max<size_t>(count, 1));
  return b.as<T>();
}

// The operator the refinement and the backward pass iterate with, on row-major
// blocks of k columns: A_R = A (no preconditioner, or the diagonal one, which
// is folded into the stored values), A L^{-T} (incomplete Cholesky, normal
// form) or L^{-1} A L^{-T} (incomplete Cholesky, symmetric form).
// op_a: y = A_R x; with ``part`` it also leaves the column sums of y.^2 (or
// of y .* x with ``dot``) as partials and returns their count.
int op_a(nsp_ctx* c, int k, const double* x, double* y, double* part = nullptr, bool dot = false) {
  if (!c->precond_ic) return spmm_wide(c, c->A, k, x, y, part, dot);
  const int64_t n = c->n, m = c->m;
  double* t = alloc_as<double>(c->ic_wide, (size_t)n * k);
  NSP_HIP(hipMemcpyAsync(t, x, sizeof(double) * n * k, hipMemcpyDeviceToDevice, c->stream));
  ic_solve_lt<double>(c, k, t);
  spmm_wide(c, c->A, k, t, y);
  if (c->sym) ic_solve_l<double>(c, k, y);
  if (!part) return 0;
  coldots(c, m, k, y, dot ? x : y, part, alloc_as<double>(c->ic_dots, (size_t)coldots_parts(m) * k));
  return 1;
}

// op_at: x = A_R^T y (normal form); with ``part`` the column sums of x.^2
int op_at(nsp_ctx* c, int k, const double* y, double* x, double* part = nullptr) {
  if (!c->precond_ic) return spmm_wide(c, c->AT, k, y, x, part);
  const int64_t n = c->n;
  spmm_wide(c, c->AT, k, y, x);
  ic_solve_l<double>(c, k, x);
  if (!part) return 0;
  coldots(c, n, k, x, x, part, alloc_as<double>(c->ic_dots, (size_t)coldots_parts(n) * k));
  return 1;
}

// ||B_R - eps D|| for reading R7's first cycle with the incomplete Cholesky
// preconditioner, where no cheap norm bound exists: 30 power steps on
// A_R^T A_R (or A_R) from D, times 1.5 (the estimate approaches the largest
// eigenvalue from below).  Later cycles use the largest Ritz value.
double ic_norm_bound(nsp_ctx* c) {
  if (c->ic.norm_bound > 0.0) return c->ic.norm_bound;
  const int64_t n = c->n, m = c->m;
  DBuf bx, by, bz, bd, bp;
  double* x = alloc_as<double>(bx, n);
  double* y = alloc_as<double>(by, std::max(n, m));
  double* z = alloc_as<double>(bz, n);
  double* dots = alloc_as<double>(bd, 1);
  double* part = alloc_as<double>(bp, coldots_parts(std::max(n, m)));
  NSP_HIP(hipMemcpyAsync(x, c->Dv.as<double>(), sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  double lam = 0.0, nrm = 0.0;
  // the library's stream is non-blocking: read back through it
  auto read = [&](double& out) {
    NSP_HIP(hipMemcpyAsync(c->pin_d, dots, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    NSP_HIP(hipStreamSynchronize(c->stream));
    out = c->pin_d[0];
  };
  coldots(c, n, 1, x, x, dots, part);
  read(nrm);
  for (int it = 0; it < 30 && nrm > 0.0; ++it) {
    const double s = 1.0 / std::sqrt(nrm);
    NSP_BLAS(rocblas_dscal(c->blas, (rocblas_int)n, &s, x, 1));
    if (c->sym) {
      op_a(c, 1, x, z);
    } else {
      op_a(c, 1, x, y);
      op_at(c, 1, y, z);
    }
    coldots(c, n, 1, x, z, dots, part);  // Rayleigh quotient of the unit x
    read(lam);
    std::swap(x, z);
    coldots(c, n, 1, x, x, dots, part);
    read(nrm);
  }
  if (!(lam > 0.0) || !std::isfinite(lam)) throw Error(NSP_ERR_NONFINITE, "norm estimate of B_R failed");
  c->ic.norm_bound = 1.5 * lam;
  return c->ic.norm_bound;
}

// dense small GEMM helpers on column-major FP64 (rocBLAS)
void dgemm(nsp_ctx* c, rocblas_operation ta, rocblas_operation tb, int64_t m, int64_t n, int64_t k,
           double alpha, const double* a, int64_t lda, const double* b, int64_t ldb, double beta,
           double* out, int64_t ldc) {
  NSP_BLAS(rocblas_dgemm(c->blas, ta, tb, (rocblas_int)m, (rocblas_int)n, (rocblas_int)k, &alpha, a,
                         (rocblas_int)lda, b, (rocblas_int)ldb, &beta, out, (rocblas_int)ldc));
}
void sgemm(nsp_ctx* c, rocblas_operation ta, rocblas_operation tb, int64_t m, int64_t n, int64_t k,
           float alpha, const float* a, int64_t lda, const float* b, int64_t ldb, float beta,
           float* out, int64_t ldc) {
  NSP_BLAS(rocblas_sgemm(c->blas, ta, tb, (rocblas_int)m, (rocblas_int)n, (rocblas_int)k, &alpha, a,
                         (rocblas_int)lda, b, (rocblas_int)ldb, &beta, out, (rocblas_int)ldc));
}

// symmetric eigen-decomposition on the device (FP64): A (k x k) is replaced by
// its eigenvectors, w receives the eigenvalues ascending.
// out (m1 x m2, column-major) = A B^T for column-major A (m1 x rows, ld lda)
// and B (m2 x rows, ld ldb): a long inner dimension with a small output, as in
// the Gram and projection products of the refinement and backward.  One GEMM
// would run on a few workgroups, so the rows are cut into chunks computed by
// one strided-batched GEMM and the partial products are summed in chunk order.
void dgemm_nt_long(nsp_ctx* c, int64_t m1, int64_t m2, int64_t rows, const double* a, int64_t lda,
                   const double* b, int64_t ldb, double* out, DBuf& work) {
  const int64_t nch = std::min<int64_t>(64, std::max<int64_t>(1, rows / 2048));
  if (nch == 1) {
    dgemm(c, rocblas_operation_none, rocblas_operation_transpose, m1, m2, rows, 1.0, a, lda, b, ldb,
          0.0, out, m1);
    return;
  }
  const int64_t cs = rows / nch, rem = rows - cs * nch, np = nch + (rem > 0 ? 1 : 0);
  double* part = alloc_as<double>(work, (size_t)(np * m1 * m2));
  const double one = 1.0, zero = 0.0;
  NSP_BLAS(rocblas_dgemm_strided_batched(c->blas, rocblas_operation_none, rocblas_operation_transpose,
                                         (rocblas_int)m1, (rocblas_int)m2, (rocblas_int)cs, &one, a,
                                         (rocblas_int)lda, cs * lda, b, (rocblas_int)ldb, cs * ldb,
                                         &zero, part, (rocblas_int)m1, m1 * m2, (rocblas_int)nch));
  if (rem)
    dgemm(c, rocblas_operation_none, rocblas_operation_transpose, m1, m2, rem, 1.0, a + cs * nch * lda,
          lda, b + cs * nch * ldb, ldb, 0.0, part + nch * m1 * m2, m1);
  reduce_parts(c, (int)np, (int)(m1 * m2), part, out);
}

void syevd(nsp_ctx* c, int k, double* a, double* w, DBuf& ework, DBuf& info) {
  double* e = alloc_as<double>(ework, k);
  rocblas_int* inf = alloc_as<rocblas_int>(info, 1);
  NSP_BLAS(rocsolver_dsyevd(c->blas, rocblas_evect_original, rocblas_fill_lower, k, a, k, w, e, inf));
  NSP_HIP(hipMemcpyAsync(c->pin_i + 8, inf, sizeof(rocblas_int), hipMemcpyDeviceToHost, c->stream));
  NSP_HIP(hipStreamSynchronize(c->stream));
  const int h = c->pin_i[8];
  if (h != 0) throw Error(NSP_ERR_HIP, "rocsolver_dsyevd did not converge (info " + std::to_string(h) + ")");
}

// ---------------------------------------------------------------------------
template <typename VT>
struct Lanczos {
  nsp_ctx* c;
  int64_t n, m, ldz;
  int d, K, L;
  VT *Z, *Z2, *ring[3], *Y, *P;
  double *xi, *gam, *rinvc, *nrm_xi, *nrm_gam, *nrm_ginv, *nrm_theta, *nrm_f;
  double *part_xi, *part_g, *part_g2, *part_c;
  double *W, *theta_kept, *fmat, *T, *evals, *H, *hpart;
  int ldw;
  int* flags;
  std::unique_ptr<EigWork, void (*)(EigWork*)> eigw{eig_work_new(), eig_work_delete};
  DBuf b_xi, b_gam, b_rinvc, b_nxi, b_ngam, b_nginv, b_ntheta, b_nf, b_W, b_hpart,
      b_H, b_info, b_vzf, b_tmpv;

  // HIP-event timing at sampled steps (profile mode): the SpMV pair and the
  // reorthogonalisation pair (projection H = Z^T C with its reduction, then the
  // update C -= Z H), with the per-step flag telling which pairs really ran
  struct Prof {
    static constexpr int kSlots = 160;
    static constexpr int kEv = 7;
    bool on = false;
    int used = 0;
    int ell[kSlots];
    int kcols[kSlots];
    int64_t samples = 0, ro_active = 0;
    double sum_a = 0.0, sum_at = 0.0, tn_ms = 0.0, nn_ms = 0.0, tn_bytes = 0.0, nn_bytes = 0.0;
    double idle_ms = 0.0;
    hipEvent_t ev[kEv * kSlots];
    void init(bool enable) {
      on = enable;
      if (on)
        for (auto& e : ev) NSP_HIP(hipEventCreate(&e));
    }
    hipEvent_t e(int slot, int i) { return ev[kEv * slot + i]; }
    // hist: per-step reorthogonalisation flags of this cycle (host copy)
    void collect(const int* hist, int64_t n, int d, int esize) {
      for (int i = 0; i < used; ++i) {
        // events: 0 | A x | 1 | A^T y | 2 ... 3 | Z^T C | 4 | reduce | 5 | C -= Z H | 6
        float a = 0.f, b = 0.f, t = 0.f, u = 0.f;
        NSP_HIP(hipEventElapsedTime(&a, e(i, 0), e(i, 1)));
        NSP_HIP(hipEventElapsedTime(&b, e(i, 1), e(i, 2)));
        NSP_HIP(hipEventElapsedTime(&t, e(i, 3), e(i, 4)));
        NSP_HIP(hipEventElapsedTime(&u, e(i, 5), e(i, 6)));
        sum_a += a;
        sum_at += b;
        ++samples;
        if (hist[ell[i]]) {
          const double k = kcols[i];
          tn_ms += t;
          nn_ms += u;
          tn_bytes += esize * (k * n + 2.0 * d * n);
          nn_bytes += esize * (k * n + 4.0 * d * n);
          ++ro_active;
        } else {
          idle_ms += t + u;
        }
      }
      used = 0;
    }
    ~Prof() {
      if (on)
        for (auto& x : ev) (void)hipEventDestroy(x);
    }
  } prof;
  DBuf b_rohist;
  int* ro_hist = nullptr;

  explicit Lanczos(nsp_ctx* ctx) : c(ctx) {
    n = c->n; m = c->m; d = c->prm.d; K = c->prm.max_dim; L = K / d;
    ldz = (n + 63) / 64 * 64;
    Z = alloc_as<VT>(c->Z, (size_t)ldz * (K + d));
    Z2 = alloc_as<VT>(c->Z2, (size_t)ldz * (K + d));
    if (d > 1) {
      VT* r = alloc_as<VT>(c->ring, (size_t)3 * n * d);
      for (int i = 0; i < 3; ++i) ring[i] = r + (size_t)i * n * d;
    }
    Y = alloc_as<VT>(c->Y, (size_t)m * d);
    P = alloc_as<VT>(c->P, (size_t)n * d);
    const int nb = L + 3;
    xi = alloc_as<double>(b_xi, (size_t)nb * d * d);
    gam = alloc_as<double>(b_gam, (size_t)nb * d * d);
    rinvc = alloc_as<double>(b_rinvc, (size_t)2 * 4 * d * d);
    part_xi = c->part_xi.as<double>();
    part_g = c->part_g.as<double>();
    part_g2 = c->part_g2.as<double>();
    part_c = alloc_as<double>(c->part_c, (size_t)ts_part_c_len(n, 2 * d));
    nrm_xi = alloc_as<double>(b_nxi, nb);
    nrm_gam = alloc_as<double>(b_ngam, nb);
    nrm_ginv = alloc_as<double>(b_nginv, nb);
    nrm_theta = alloc_as<double>(b_ntheta, nb);
    nrm_f = alloc_as<double>(b_nf, nb);
    ldw = L + 3;
    W = alloc_as<double>(b_W, (size_t)ldw * ldw);
    theta_kept = alloc_as<double>(c->theta_kept, K);
    fmat = alloc_as<double>(c->fmat, (size_t)d * K);
    T = alloc_as<double>(c->tmat, (size_t)K * K);
    evals = alloc_as<double>(c->evals, K);
    H = alloc_as<double>(b_H, (size_t)(K + d) * 2 * d);
    int64_t maxchunks = 1;
    for (int nc : {d, 2 * d}) {
      const int64_t chunk = ts_chunk_rows(n, 1, nc, (int)sizeof(VT));
      maxchunks = std::max(maxchunks, (n + chunk - 1) / chunk);
    }
    hpart = alloc_as<double>(b_hpart, (size_t)maxchunks * (K + d) * 2 * d);
    // read-backs per cycle: K Ritz values, the last d rows of V_Z, Gamma_L
    c->pin_d = c->pind.ensure((size_t)K * (d + 1) + (size_t)d * d + 16);
    flags = alloc_as<int>(c->flags, 8);
    NSP_HIP(hipMemsetAsync(flags, 0, sizeof(int) * 8, c->stream));
    NSP_HIP(hipMemsetAsync(W, 0, sizeof(double) * ldw * ldw, c->stream));
    NSP_HIP(hipMemsetAsync(nrm_theta, 0, sizeof(double) * nb, c->stream));
    NSP_HIP(hipMemsetAsync(nrm_f, 0, sizeof(double) * nb, c->stream));
    prof.init(c->prm.profile != 0);
    if (prof.on) {
      ro_hist = alloc_as<int>(b_rohist, L + 3);
      NSP_HIP(hipMemsetAsync(ro_hist, 0, sizeof(int) * (L + 3), c->stream));
    }
  }

  // row-interleaved copy of Lanczos block ``blk`` (1-based); for d = 1 it is
  // the basis column itself
  VT* slot(int blk) const { return d == 1 ? Z + (int64_t)(blk - 1) * ldz : ring[blk % 3]; }
  VT* zcol(int blk) const { return d == 1 ? nullptr : Z + (int64_t)(blk - 1) * d * ldz; }

  // Q = orth(X) for the block in slot ``blk``: Cholesky QR (twice for d > 1)
  void orthonormalize_slot(int blk, double* gam_out) {
    VT* x = slot(blk);
    int np = sub_gram<VT>(c, d, n, x, nullptr, nullptr, 0, nullptr, nullptr, part_g);
    np = scale_block<VT>(c, d, n, x, part_g, np, x, zcol(blk), ldz, gam_out, nullptr, nullptr,
                         d > 1 ? part_g2 : nullptr);
    if (d > 1) scale_block2<VT>(c, d, n, part_g2, np, x, zcol(blk), ldz, gam_out, nullptr, nullptr);
  }

  // Xi_{blk_from} from the SpMV partials and the QR of P into slot ``blk_to``
  // (Gamma_{blk_from} stored), with or without the subtraction of X Xi
  void qr_step(int blk_from, int blk_to, bool subtract, int nparts_xi, const WArgs* wa = nullptr) {
    double* g = gam + (size_t)blk_from * d * d;
    int np = sub_gram<VT>(c, d, n, P, subtract ? slot(blk_from) : nullptr, part_xi, nparts_xi,
                          xi + (size_t)blk_from * d * d, nrm_xi + blk_from, part_g);
    np = scale_block<VT>(c, d, n, P, part_g, np, slot(blk_to), zcol(blk_to), ldz, g,
                         nrm_gam + blk_from, nrm_ginv + blk_from, d > 1 ? part_g2 : nullptr,
                         d > 1 ? nullptr : wa);
    if (d > 1)
      scale_block2<VT>(c, d, n, part_g2, np, slot(blk_to), zcol(blk_to), ldz, g, nrm_gam + blk_from,
                       nrm_ginv + blk_from, wa);
  }

  // P = B X - Xp Gamma_prev^T with the Xi partials (Alg. 2 inner loop):
  // A^T (A X) + eps D X, or A X + eps D X for the symmetric form (the stored
  // A^T is A itself then).  ``mid`` is recorded between the two products.
  int apply_b(VT* x, const VT* xp, const double* gprev, hipEvent_t mid = nullptr) {
    if (c->precond_ic) {
      // B_R X = L^{-1} (A^T A or A) L^{-T} X + eps D X: solve with L^T into a
      // copy, the products, solve with L in place, then the step's epilogue
      VT* t = alloc_as<VT>(c->ic_tmp, (size_t)n * d);
      NSP_HIP(hipMemcpyAsync(t, x, sizeof(VT) * n * d, hipMemcpyDeviceToDevice, c->stream));
      ic_solve_lt<VT>(c, d, t);
      if (!c->sym) {
        spmm_block<VT>(c, c->A, d, t, Y);
        spmm_block<VT>(c, c->AT, d, Y, P);
      } else {
        spmm_block<VT>(c, c->A, d, t, P);
      }
      if (mid) NSP_HIP(hipEventRecord(mid, c->stream));
      ic_solve_l<VT>(c, d, P);
      return step_epilogue<VT>(c, d, x, xp, gprev, P, part_xi);
    }
    const VT* yin = x;
    if (!c->sym) {
      spmm_block<VT>(c, c->A, d, x, Y);
      yin = Y;
    }
    if (mid) NSP_HIP(hipEventRecord(mid, c->stream));
    return spmmT_step<VT>(c, d, yin, x, xp, gprev, P, part_xi);
  }

  void cgs2_full(VT* a, int k, bool final_gram, double* rinv_out) {
    ts_project<VT>(c, nullptr, d, 1, n, Z, ldz, k, a, nullptr, H, hpart, false, nullptr, nullptr);
    ts_project<VT>(c, nullptr, d, 1, n, Z, ldz, k, a, nullptr, H, hpart, final_gram, part_c,
                   rinv_out);
  }

  void run() {
    nsp_params& p = c->prm;
    nsp_stats& st = c->stats;
    st = nsp_stats{};
    const double t0 = now_s();
    // Reading R8: u of the working (storage) precision sets u_RO = sqrt(u).  The
    // round-off of one step (Eq. "defmprd") is d sqrt(n) u ||B|| when all
    // arithmetic is in that precision; the FP32 mode accumulates in FP64 and
    // rounds each stored vector once, so its per-step error is d (sqrt(n) u64
    // + u32) ||B||.
    const double u64 = std::ldexp(1.0, -52), u32 = std::ldexp(1.0, -23);
    const double u = sizeof(VT) == 8 ? u64 : u32;
    const double u_ro = p.ro_tol > 0 ? p.ro_tol : std::sqrt(u);
    const double u_step = sizeof(VT) == 8 ? std::sqrt((double)n) * u64 : std::sqrt((double)n) * u64 + u32;
    // reading R7: a cheap upper bound of ||B|| until the first Ritz values exist
    const double norm_t = (c->precond_ic ? ic_norm_bound(c) : c->sym ? c->normA_inf : c->normA1_inf) +
                          p.eps * c->maxD;
    double norm_b = norm_t;
    double u_d = d * u_step * norm_b;

    // Q_1 = orth(Omega)
    cm_to_ri<double, VT>(c, n, d, c->omega.as<double>(), n, slot(1));
    orthonormalize_slot(1, gam);

    int l0 = 0;
    int64_t matvecs = 0;
    std::vector<std::pair<int64_t, int>> hist;
    std::vector<double> hev(K);
    int flags_h[8];
    double t_lan = 0.0, t_rr = 0.0;
    bool stop = false;
    int n_ell = 0;
    const char* ve = std::getenv("NSP_VERBOSE");
    const bool verbose = ve && (ve[0] == '1' || ve[0] == '2');
    const bool verbose_all = ve && ve[0] == '2';
    const char* de = std::getenv("NSP_DENSE_EIG");
    const bool dense_eig = de && de[0] == '1';
    // diagnostics: NSP_NO_SPEED_STOP=1 runs until the matvec or cycle budget
    const char* ns = std::getenv("NSP_NO_SPEED_STOP");
    const bool no_speed_stop = ns && ns[0] == '1';
    double last_print = now_s();
    c->cycle_s.clear();
    for (;;) {
      const double tc0 = now_s();
      const int kk = l0 * d;
      // ---- first step of the cycle: Q' = B Q_{l0+1}, Xi, QR((I - Z Z^T) Q')
      {
        const int blk = l0 + 1;
        const int npx = apply_b(slot(blk), nullptr, nullptr);
        cgs2_full(P, kk + d, false, nullptr);
        qr_step(blk, blk + 1, false, npx);
        w_reset(c, l0 + 1, 2, u_d, W, ldw);
        matvecs += d;
      }
      // ---- Lanczos steps ell = l0+2 .. L with partial reorthogonalisation
      for (int ell = l0 + 2; ell <= L; ++ell) {
        VT* x = slot(ell);
        VT* xp = slot(ell - 1);
        VT* xn = slot(ell + 1);
        const bool timed = prof.on && (ell % 4 == 0) && prof.used < Prof::kSlots;
        const int slot = prof.used;
        if (timed) NSP_HIP(hipEventRecord(prof.e(slot, 0), c->stream));
        const int npx = apply_b(x, xp, gam + (size_t)(ell - 1) * d * d,
                                timed ? prof.e(slot, 1) : nullptr);
        if (timed) NSP_HIP(hipEventRecord(prof.e(slot, 2), c->stream));
        const WArgs wa{ell, l0, ldw, u_d, u_ro, nrm_xi, nrm_gam, nrm_theta, nrm_f, W, flags, ro_hist};
        qr_step(ell, ell + 1, true, npx, &wa);
        // partial reorthogonalisation of [Q_ell, Q_ell+1] against Z_{ell-1} when the
        // W-recurrence raised the flag: one CGS pass (reading R5), then Cholesky QR
        const int kz = (ell - 1) * d;
        if (timed) NSP_HIP(hipEventRecord(prof.e(slot, 3), c->stream));
        ts_project<VT>(c, flags, d, 2, n, Z, ldz, kz, x, xn, H, hpart, true, part_c, rinvc,
                       timed ? prof.e(slot, 4) : nullptr, timed ? prof.e(slot, 5) : nullptr);
        if (timed) {
          NSP_HIP(hipEventRecord(prof.e(slot, 6), c->stream));
          prof.ell[slot] = ell;
          prof.kcols[slot] = kz;
          prof.used++;
        }
        ts_scale<VT>(c, flags, d, 2, n, x, xn, part_c, rinvc, d > 1 ? zcol(ell) : nullptr, ldz);
        matvecs += d;
      }
      NSP_HIP(hipStreamSynchronize(c->stream));
      const double tc1 = now_s();
      t_lan += tc1 - tc0;
      if (prof.on) {
        std::vector<int> hh(L + 3);
        NSP_HIP(hipMemcpy(hh.data(), ro_hist, sizeof(int) * (L + 3), hipMemcpyDeviceToHost));
        prof.collect(hh.data(), n, d, (int)sizeof(VT));
      }
      // ---- Rayleigh-Ritz on T (Eq. "defT"): the structured divide-and-conquer
      // solver up to K = 4096 (its secular kernels stage a problem in 64 KB of
      // LDS); dense FP64 rocSOLVER beyond, or with NSP_DENSE_EIG=1
      if (!dense_eig && K <= 4096) {
        eig_restart(c, *eigw, K, d, kk, norm_t, theta_kept, fmat, xi, gam, evals, T);
      } else {
        assemble_t(c, K, d, kk, theta_kept, fmat, xi, gam, T);
        syevd(c, K, T, evals, c->ework, b_info);
      }
      // Ritz values, the last d rows of V_Z and Gamma_L (for the residual norms)
      double* pin_s = c->pin_d + K;
      double* pin_g = pin_s + (size_t)K * d;
      NSP_HIP(hipMemcpyAsync(c->pin_d, evals, sizeof(double) * K, hipMemcpyDeviceToHost, c->stream));
      NSP_HIP(hipMemcpy2DAsync(pin_s, sizeof(double) * d, T + (K - d), sizeof(double) * K,
                               sizeof(double) * d, K, hipMemcpyDeviceToHost, c->stream));
      NSP_HIP(hipMemcpyAsync(pin_g, gam + (size_t)L * d * d, sizeof(double) * d * d,
                             hipMemcpyDeviceToHost, c->stream));
      NSP_HIP(hipMemcpyAsync(c->pin_i, flags, sizeof(int) * 8, hipMemcpyDeviceToHost, c->stream));
      NSP_HIP(hipStreamSynchronize(c->stream));
      std::copy(c->pin_d, c->pin_d + K, hev.begin());
      std::copy(c->pin_i, c->pin_i + 8, flags_h);
      ritz_residuals(pin_s, pin_g);
      if (flags_h[4] != 0)
        throw Error(NSP_ERR_HIP, "tridiagonal eigensolver did not converge (info " +
                                     std::to_string(flags_h[4]) + ")");
      if (flags_h[1] & 2)
        throw Error(NSP_ERR_BREAKDOWN,
                    "partial reorthogonalisation: one Gram-Schmidt pass removed more than "
                    "1 - 1/sqrt(2) of a vector's norm (the W bound failed)");
      if (flags_h[1]) throw Error(NSP_ERR_BREAKDOWN, "a Lanczos block lost rank (Krylov breakdown)");
      for (double v : hev)
        if (!std::isfinite(v)) throw Error(NSP_ERR_NONFINITE, "non-finite Ritz value");
      n_ell = (int)std::count_if(hev.begin(), hev.end(), [&](double v) { return v < 3.0 * p.eps; });
      hist.emplace_back(matvecs, n_ell);
      st.cycles++;
      if ((verbose && now_s() - last_print > 2.0) || verbose_all) {
        std::fprintf(stderr, "[nsp] cycle %d matvecs %lld N_ell %d theta0 %.3e theta_max %.3e reorth %d lanczos %.2fs rr %.2fs\n",
                     st.cycles, (long long)matvecs, n_ell, hev[0], hev[K - 1], flags_h[3], t_lan, t_rr);
        std::fflush(stderr);
        last_print = now_s();
      }
      stop = !no_speed_stop && (speed_rule(hist, d) || nothing_below(hev, p.eps));
      const bool budget = matvecs >= p.max_matvec || (p.max_cycles > 0 && st.cycles >= p.max_cycles);
      c->ritz = hev;
      if (stop || budget) {
        extract(n_ell);
        NSP_HIP(hipStreamSynchronize(c->stream));
        t_rr += now_s() - tc1;
        c->cycle_s.push_back(now_s() - tc0);
        break;
      }
      // ---- thick restart (Sec. 4.1)
      const int kn = restart_size(n_ell, K, d);
      if (n_ell > kn) throw Error(NSP_ERR_ARG, "max_dim too small for the detected nullity");
      restart(kn, hev);
      norm_b = hev[K - 1];  // reading R7
      u_d = d * u_step * norm_b;
      l0 = kn / d;
      st.restarts++;
      NSP_HIP(hipStreamSynchronize(c->stream));
      t_rr += now_s() - tc1;
      c->cycle_s.push_back(now_s() - tc0);
    }
    NSP_HIP(hipMemcpyAsync(c->pin_i, flags, sizeof(int) * 8, hipMemcpyDeviceToHost, c->stream));
    NSP_HIP(hipStreamSynchronize(c->stream));
    std::copy(c->pin_i, c->pin_i + 8, flags_h);
    st.nullity = n_ell;
    st.converged = stop ? 1 : 0;
    st.matvecs = matvecs;
    st.reorths = flags_h[3];
    st.norm_b = norm_b;
    st.theta_last = n_ell > 0 ? hev[n_ell - 1] : 0.0;
    st.theta_next = n_ell < K ? hev[n_ell] : 0.0;
    st.t_lanczos_s = t_lan;
    st.t_restart_s = t_rr;
    if (prof.samples) {
      st.t_spmv_a_us = prof.sum_a / prof.samples * 1e3;
      st.t_spmv_at_us = prof.sum_at / prof.samples * 1e3;
      st.spmv_samples = prof.samples;
      st.ro_tn_ms = prof.tn_ms;
      st.ro_tn_bytes = prof.tn_bytes;
      st.ro_nn_ms = prof.nn_ms;
      st.ro_nn_bytes = prof.nn_bytes;
      st.ro_idle_ms = prof.idle_ms;
      st.ro_samples = prof.samples;
      st.ro_active = prof.ro_active;
    }
    c->nullity = n_ell;
    c->state = 1;
    (void)t0;
  }

  bool nothing_below(const std::vector<double>& theta, double eps) const {
    return nothing_below_rule(theta, c->ritz_res, eps);
  }

  // Lanczos residual norms of the Ritz pairs (Eq. "laniter"): with
  // B Z = Z T + Q_{L+1} [0, Gamma_L], the pair (theta_i, Z V_Z(:, i)) has
  // residual Q_{L+1} Gamma_L V_Z(last d rows, i), of norm ||Gamma_L s_i||.
  // s: the last d rows of V_Z (d x K, column i at s + i d); g: Gamma_L
  // (upper triangular, column-major d x d).
  void ritz_residuals(const double* s, const double* g) {
    c->ritz_res.assign(K, 0.0);
    for (int i = 0; i < K; ++i) {
      double r2 = 0.0;
      for (int a = 0; a < d; ++a) {
        double t = 0.0;
        for (int b = a; b < d; ++b) t += g[a + b * d] * s[(size_t)i * d + b];
        r2 += t * t;
      }
      c->ritz_res[i] = std::sqrt(r2);
    }
  }

  // Z_new = Z V_Z(:, 1:kn); Q_{l0+1} = orth((I - Z_new Z_new^T) Q_{L+1}); F
  void restart(int kn, const std::vector<double>& hev) {
    // basis update Z2(:, 0:kn) = Z(:, 0:K) V_Z(:, 0:kn)
    if constexpr (sizeof(VT) == 8) {
      dgemm(c, rocblas_operation_none, rocblas_operation_none, n, kn, K, 1.0, (const double*)Z, ldz,
            T, K, 0.0, (double*)Z2, ldz);
    } else {
      float* vz = alloc_as<float>(b_vzf, (size_t)K * kn);
      convert<double, float>(c, (int64_t)K * kn, T, vz);
      sgemm(c, rocblas_operation_none, rocblas_operation_none, n, kn, K, 1.0f, (const float*)Z, ldz,
            vz, K, 0.0f, (float*)Z2, ldz);
    }
    // carry Q_{L+1} (columns K..K+d of Z) to columns kn..kn+d of Z2
    copy_panel<VT, VT>(c, n, d, Z + (int64_t)K * ldz, ldz, Z2 + (int64_t)kn * ldz, ldz);
    std::swap(Z, Z2);
    const int blk = kn / d + 1;
    if (d > 1) cm_to_ri<VT, VT>(c, n, d, Z + (int64_t)kn * ldz, ldz, slot(blk));
    // re-orthonormalise against the kept Ritz vectors: CGS2 with the Gram of the
    // result, then scale by R^{-1} (R ~ I)
    cgs2_full(slot(blk), kn, true, rinvc);
    ts_scale<VT>(c, nullptr, d, 1, n, slot(blk), nullptr, part_c, rinvc, d > 1 ? zcol(blk) : nullptr,
                 ldz);
    // F = R Gamma_L V_Z(K-d:K, 0:kn) (reading R11), Theta and the kept-block norms
    restart_coupling(c, K, d, kn, T, gam + (size_t)L * d * d, rinvc, evals, fmat, theta_kept,
                     nrm_theta, nrm_f);
    (void)hev;
  }

  // V = Z(:, 0:K) V_Z(:, 0:N) in FP64, column-major n x N
  // out (n x cols, FP64) = Z V_Z(:, col0 : col0 + cols)
  void ritz_vectors(int col0, int cols, double* out) {
    if constexpr (sizeof(VT) == 8) {
      dgemm(c, rocblas_operation_none, rocblas_operation_none, n, cols, K, 1.0, (const double*)Z, ldz,
            T + (size_t)col0 * K, K, 0.0, out, n);
    } else {
      float* vz = alloc_as<float>(b_vzf, (size_t)K * cols);
      convert<double, float>(c, (int64_t)K * cols, T + (size_t)col0 * K, vz);
      float* tmp = alloc_as<float>(b_tmpv, (size_t)n * cols);
      sgemm(c, rocblas_operation_none, rocblas_operation_none, n, cols, K, 1.0f, (const float*)Z, ldz,
            vz, K, 0.0f, tmp, n);
      convert<float, double>(c, (int64_t)n * cols, tmp, out);
    }
  }

  void extract(int nul) {
    double* v = alloc_as<double>(c->V, (size_t)n * std::max(nul, 1));
    c->defl_r = 0;
    c->df_r = 0;
    if (nul == 0) return;
    ritz_vectors(0, nul, v);
    // The next Ritz vectors (smallest nonzero part of the spectrum) deflate the
    // refinement's CGLS: they are the directions it converges slowest along.
    if (c->prm.refine && !c->sym) {
      const int64_t budget = (int64_t)1 << 29;  // bytes for each of its four n x r blocks
      const int r = (int)std::min<int64_t>({(int64_t)kDeflMax, (int64_t)K - nul - d,
                                           budget / (8 * std::max<int64_t>(n, m))});
      if (r >= 8) {
        ritz_vectors(nul, r, alloc_as<double>(c->Wd, (size_t)n * r));
        c->defl_r = r;
      }
    }
  }
};

// ---------------------------------------------------------------------------
// Deflation space shared by the refinement and the backward pass (normal
// form): the Ritz vectors the last Lanczos cycle left just above the null
// cluster (c->Wd), rotated by a Rayleigh-Ritz step with A^T A so that
// W^T A^T A W = Lambda; their Ritz values below 1e-12 of the largest are
// dropped.  Built once per solve.
// ---------------------------------------------------------------------------
void build_deflation(nsp_ctx* c) {
  if (c->df_r > 0 || c->defl_r <= 0) return;
  const int64_t n = c->n, m = c->m;
  const int r = c->defl_r;
  DBuf b_w0, b_aw0, b_S, b_l, b_ei, b_inf, b_U, b_UL, b_long;
  double* w0 = alloc_as<double>(b_w0, (size_t)n * r);
  colmajor_to_rows(c, n, r, c->Wd.as<double>(), n, w0);
  double* aw0 = alloc_as<double>(b_aw0, (size_t)m * r);
  op_a(c, r, w0, aw0);
  double* S = alloc_as<double>(b_S, (size_t)r * r);
  dgemm_nt_long(c, r, r, m, aw0, r, aw0, r, S, b_long);
  double* lam = alloc_as<double>(b_l, r);
  syevd(c, r, S, lam, b_ei, b_inf);
  std::vector<double> hl(r), hu((size_t)r * r);
  NSP_HIP(hipMemcpy(hl.data(), lam, sizeof(double) * r, hipMemcpyDeviceToHost));
  NSP_HIP(hipMemcpy(hu.data(), S, sizeof(double) * r * r, hipMemcpyDeviceToHost));
  const double lmax = hl[r - 1];
  std::vector<int> keep;
  for (int i = 0; i < r; ++i)
    if (std::isfinite(hl[i]) && hl[i] > 1e-12 * lmax) keep.push_back(i);
  const int rk = (int)keep.size();
  if (rk == 0) return;
  std::vector<double> uk((size_t)r * rk), ul((size_t)r * rk);
  for (int j = 0; j < rk; ++j)
    for (int i = 0; i < r; ++i) {
      uk[i + (size_t)j * r] = hu[i + (size_t)keep[j] * r];
      ul[i + (size_t)j * r] = hu[i + (size_t)keep[j] * r] / hl[keep[j]];
    }
  double* du = alloc_as<double>(b_U, (size_t)r * rk);
  double* dul = alloc_as<double>(b_UL, (size_t)r * rk);
  NSP_HIP(hipMemcpy(du, uk.data(), sizeof(double) * uk.size(), hipMemcpyHostToDevice));
  NSP_HIP(hipMemcpy(dul, ul.data(), sizeof(double) * ul.size(), hipMemcpyHostToDevice));
  // rotated blocks, column-major views (X_cm = row-major X transposed): X_cm = U^T X0_cm
  double* w = alloc_as<double>(c->dfW, (size_t)n * rk);
  double* ws = alloc_as<double>(c->dfWs, (size_t)n * rk);
  double* aw = alloc_as<double>(c->dfAW, (size_t)m * rk);
  double* aws = alloc_as<double>(c->dfAWs, (size_t)m * rk);
  double* mws = alloc_as<double>(c->dfMWs, (size_t)n * rk);
  dgemm(c, rocblas_operation_transpose, rocblas_operation_none, rk, n, r, 1.0, du, r, w0, r, 0.0, w, rk);
  dgemm(c, rocblas_operation_transpose, rocblas_operation_none, rk, n, r, 1.0, dul, r, w0, r, 0.0, ws, rk);
  dgemm(c, rocblas_operation_transpose, rocblas_operation_none, rk, m, r, 1.0, du, r, aw0, r, 0.0, aw, rk);
  dgemm(c, rocblas_operation_transpose, rocblas_operation_none, rk, m, r, 1.0, dul, r, aw0, r, 0.0, aws, rk);
  op_at(c, rk, aws, mws);
  NSP_HIP(hipStreamSynchronize(c->stream));
  c->df_r = rk;
}

// V <- V R^{-1}, R^T R = V^T V (Cholesky QR) for a row-major n x k block V
void cholqr_rows(nsp_ctx* c, double* vr, int64_t n, int k, DBuf& b_g, DBuf& b_info, DBuf& b_long) {
  double* g = alloc_as<double>(b_g, (size_t)k * k);
  rocblas_int* inf = alloc_as<rocblas_int>(b_info, 1);
  dgemm_nt_long(c, k, k, n, vr, k, vr, k, g, b_long);
  NSP_BLAS(rocsolver_dpotrf(c->blas, rocblas_fill_upper, k, g, k, inf));
  NSP_HIP(hipMemcpyAsync(c->pin_i + 8, inf, sizeof(rocblas_int), hipMemcpyDeviceToHost, c->stream));
  NSP_HIP(hipStreamSynchronize(c->stream));
  if (c->pin_i[8] != 0) throw Error(NSP_ERR_BREAKDOWN, "refined basis lost rank (Cholesky QR failed)");
  // V <- V R^{-1}: in the column-major view Vcm = V^T: Vcm <- R^{-T} Vcm
  const double one = 1.0;
  NSP_BLAS(rocblas_dtrsm(c->blas, rocblas_side_left, rocblas_fill_upper, rocblas_operation_transpose,
                         rocblas_diagonal_non_unit, k, (rocblas_int)n, &one, g, k, vr, k));
}

// Outer preconditioning (Sec. 4.4): vr holds an orthonormal basis V_R of
// null(A P_R^{-T}) (row-major n x k).  V_R is kept for the backward pass and vr
// becomes P_R^{-T} V_R, orthonormalised (Cholesky QR twice).
void unprecondition(nsp_ctx* c, double* vr, int k, DBuf& b_g, DBuf& b_info, DBuf& b_long) {
  const int64_t n = c->n;
  rows_to_colmajor(c, n, k, vr, alloc_as<double>(c->Vs, (size_t)n * k), n);
  if (c->precond_ic) ic_solve_lt<double>(c, k, vr);
  else scale_rows(c, n, k, c->pdiag.as<double>(), true, vr);
  cholqr_rows(c, vr, n, k, b_g, b_info, b_long);
  cholqr_rows(c, vr, n, k, b_g, b_info, b_long);
}

// ---------------------------------------------------------------------------
// FP64 refinement: Rayleigh-Ritz with A^T A, CGLS projection onto null(A),
// Cholesky QR twice, residual and orthogonality checks.
// ---------------------------------------------------------------------------
struct Refiner {
  nsp_ctx* c;
  int64_t n, m;
  int k;
  DBuf b_vr, b_u, b_x, b_s, b_r, b_p, b_q, b_small, b_small2, b_part, b_dots, b_act, b_info, b_e;
  DBuf b_long;  // partial products of dgemm_nt_long

  Refiner(nsp_ctx* ctx, int nul) : c(ctx), n(ctx->n), m(ctx->m), k(nul) {}

  // Deflation space of the CGLS (normal form): the Ritz vectors just above the
  // null cluster (build_deflation).  Deflated CG (x0 = W Lambda^-1 W^T b,
  // search directions kept A^T A-orthogonal to W) then converges at the rate
  // of the spectrum above the deflated part.
  int rd = 0;
  double *dW = nullptr, *dAW = nullptr, *dAWs = nullptr, *dMWs = nullptr;
  DBuf b_dmu;

  void setup_deflation() {
    build_deflation(c);
    rd = c->df_r;
    if (rd == 0) return;
    dW = c->dfW.as<double>();
    dAW = c->dfAW.as<double>();
    dAWs = c->dfAWs.as<double>();
    dMWs = c->dfMWs.as<double>();
  }

  // p -= W Lambda^-1 (A^T A W)^T r  (column-major views: mu = r_cm MWs_cm^T)
  void deflate_direction(const double* r, double* p) {
    double* mu = alloc_as<double>(b_dmu, (size_t)k * rd);
    dgemm_nt_long(c, k, rd, n, r, k, dMWs, rd, mu, b_long);
    dgemm(c, rocblas_operation_none, rocblas_operation_none, k, n, rd, -1.0, mu, k, dW, rd, 1.0, p, k);
  }

  // row-major n x k  <->  column-major k x n view with ld k
  void gram_rows(const double* a, int64_t rows, double* g) {
    // G = A^T A for row-major A (rows x k): column-major view Acm (k x rows)
    dgemm_nt_long(c, k, k, rows, a, k, a, k, g, b_long);
  }

  void cholqr(double* vr) { cholqr_rows(c, vr, n, k, b_small, b_info, b_long); }

  void run() {
    nsp_params& p = c->prm;
    nsp_stats& st = c->stats;
    const double t0 = now_s();
    c->pin_d = c->pind.ensure(std::max<size_t>((size_t)c->prm.max_dim + 16, (size_t)k * (k + 1) + 16));
    c->pin_i = c->pini.ensure(std::max<size_t>(64, (size_t)k + 16));
    double* vr = alloc_as<double>(b_vr, (size_t)n * k);
    // the symmetric form's CG needs fewer blocks: A V and the final residual
    // share the buffer of q
    double* q = alloc_as<double>(b_q, (size_t)m * k);
    double* u = c->sym ? q : alloc_as<double>(b_u, (size_t)m * k);
    colmajor_to_rows(c, n, k, c->V.as<double>(), n, vr);
    // Step 1: Rayleigh-Ritz with the unperturbed A^T A on span(V)
    op_a(c, k, vr, u);
    double* s = alloc_as<double>(b_small, (size_t)k * k);
    gram_rows(u, m, s);
    double* lam = alloc_as<double>(b_e, (size_t)2 * k);
    syevd(c, k, s, lam, b_small2, b_info);
    double* vnew = alloc_as<double>(b_x, (size_t)n * k);
    // Vr_new^T = Y^T Vr^T  (column-major views)
    dgemm(c, rocblas_operation_transpose, rocblas_operation_none, k, n, k, 1.0, s, k, vr, k, 0.0, vnew, k);
    NSP_HIP(hipMemcpyAsync(vr, vnew, sizeof(double) * n * k, hipMemcpyDeviceToDevice, c->stream));
    // Step 2: CGLS for x = A^+ A v per column, x_0 = 0; s = A v - A x = A (v - x)
    double* x = alloc_as<double>(b_x, (size_t)n * k);
    double* sv = c->sym ? q : alloc_as<double>(b_s, (size_t)m * k);
    double* r = alloc_as<double>(b_r, (size_t)n * k);
    double* pp = alloc_as<double>(b_p, (size_t)n * k);
    double* dots = alloc_as<double>(b_dots, (size_t)4 * k);  // gamma, qq, gnew, snorm2
    double* part = alloc_as<double>(b_part, (size_t)coldots_parts(std::max(n, m)) * k);
    int* act = alloc_as<int>(b_act, k);
    double *gamma = dots, *qq = dots + k, *gnew = dots + 2 * k, *sn2 = dots + 3 * k;
    NSP_HIP(hipMemsetAsync(x, 0, sizeof(double) * n * k, c->stream));
    op_a(c, k, vr, sv);
    if (!c->sym) {
      setup_deflation();
      if (rd > 0) {
        // x0 = W Lambda^-1 (A W)^T s0, s = s0 - A x0
        double* mu = alloc_as<double>(b_dmu, (size_t)k * rd);
        dgemm_nt_long(c, k, rd, m, sv, k, dAWs, rd, mu, b_long);
        dgemm(c, rocblas_operation_none, rocblas_operation_none, k, n, rd, 1.0, mu, k, dW, rd, 0.0, x, k);
        dgemm(c, rocblas_operation_none, rocblas_operation_none, k, m, rd, -1.0, mu, k, dAW, rd, 1.0, sv, k);
      }
      op_at(c, k, sv, r);
      NSP_HIP(hipMemcpyAsync(pp, r, sizeof(double) * n * k, hipMemcpyDeviceToDevice, c->stream));
      if (rd > 0) deflate_direction(r, pp);
      coldots(c, n, k, r, r, gamma, part);
    }
    coldots(c, m, k, sv, sv, sn2, part);
    // per-column target: the smallest threshold of the enabled criteria
    const double rk = std::sqrt((double)k);
    double tau = std::numeric_limits<double>::infinity();
    if (p.tol_rel_resid > 0) tau = std::min(tau, p.tol_rel_resid * c->normA_fro / rk);
    if (p.tol_abs_resid > 0) tau = std::min(tau, p.tol_abs_resid);
    if (p.tol_angle > 0) {
      // sigma_min(A) from the smallest Ritz value above 3 eps: B's eigenvalue
      // there is sigma^2 (normal form) or sigma (symmetric form) plus at most eps max D
      const double s2 = st.theta_next - p.eps * c->maxD;
      if (s2 > 0) tau = std::min(tau, p.tol_angle * (c->sym ? s2 : std::sqrt(s2)) / (2.0 * rk));
    }
    if (!std::isfinite(tau)) tau = 1e-10 * c->normA_fro / rk;
    // Attainable level: the recursively updated residual of CG / CGLS drifts
    // from the true one at about u ||A|| ||x|| (||x|| <= ||v|| = 1 here), so a
    // target below ~10 u ||A|| cannot be confirmed and would only run the
    // iteration into the stagnation stop.  ||A|| <= sqrt(||A||_1 ||A||_inf), or
    // ||A||_inf for the symmetric form.
    const double norm_a2 = c->sym ? c->normA_inf : std::sqrt(c->normA1_inf);
    const double floor_tau = 10.0 * std::ldexp(1.0, -52) * norm_a2;
    if (tau < floor_tau) {
      if (std::getenv("NSP_VERBOSE"))
        std::fprintf(stderr, "[nsp] refine target %.3e below the attainable %.3e: raised\n", tau,
                     floor_tau);
      tau = floor_tau;
    }
    std::vector<double> hs(k);
    std::vector<int> ha(k);
    // per column ||A v_j||^2 (the residual norms) -> active flags.  A run whose
    // largest residual has not dropped by 1% within 4096 iterations has
    // reached its attainable accuracy and stops (the residual check reports it).
    double best = std::numeric_limits<double>::infinity();
    int64_t last_gain = 0, it_now = 0;
    auto update_active = [&](const double* res2) -> bool {
      NSP_HIP(hipMemcpyAsync(c->pin_d, res2, sizeof(double) * k, hipMemcpyDeviceToHost, c->stream));
      NSP_HIP(hipStreamSynchronize(c->stream));
      std::copy(c->pin_d, c->pin_d + k, hs.begin());
      bool any = false;
      double mx = 0.0;
      for (int j = 0; j < k; ++j) {
        if (!std::isfinite(hs[j])) throw Error(NSP_ERR_NONFINITE, "non-finite value in refinement");
        ha[j] = std::sqrt(hs[j]) > tau ? 1 : 0;
        any |= ha[j] != 0;
        if (ha[j]) mx = std::max(mx, std::sqrt(hs[j]));
      }
      if (mx < 0.99 * best) {
        best = mx;
        last_gain = it_now;
      }
      if (any && it_now - last_gain > 4096) any = false;
      std::copy(ha.begin(), ha.end(), c->pin_i);
      NSP_HIP(hipMemcpyAsync(act, c->pin_i, sizeof(int) * k, hipMemcpyHostToDevice, c->stream));
      NSP_HIP(hipStreamSynchronize(c->stream));
      return any;
    };
    int64_t it = 0;
    const char* ve = std::getenv("NSP_VERBOSE");
    const bool verbose = ve && ve[0] == '1';
    double last_print = now_s();
    if (c->sym) {
      // Symmetric positive semi-definite A: CG on A x = A v from x = 0 stays in
      // range(A) and converges to x = A^+ A v like CGLS, in about sqrt(kappa(A))
      // instead of kappa(A) iterations; r = A (v - x) is the residual.
      NSP_HIP(hipMemcpyAsync(r, sv, sizeof(double) * n * k, hipMemcpyDeviceToDevice, c->stream));
      NSP_HIP(hipMemcpyAsync(pp, sv, sizeof(double) * n * k, hipMemcpyDeviceToDevice, c->stream));
      coldots(c, n, k, r, r, gamma, part);
    }
    bool any = update_active(c->sym ? gamma : sn2);
    while (any && it < p.max_refine_iter) {
      if (c->sym) {
        // q = A p with p . q fused; x += alpha p, r -= alpha q; p = r + beta p
        const int nq = op_a(c, k, pp, q, part, true);
        reduce_parts(c, nq, k, part, qq);
        cg_wr(c, n, k, gamma, qq, act, x, pp, r, q);
        coldots(c, n, k, r, r, gnew, part);
        cgls_p(c, n, k, gnew, gamma, act, r, pp);
        std::swap(gamma, gnew);
        ++it;
        if (it % 16 == 0) {
          it_now = it;
          any = update_active(gamma);
          if (verbose && now_s() - last_print > 2.0) {
            std::fprintf(stderr, "[nsp] refine (CG) it %lld\n", (long long)it);
            std::fflush(stderr);
            last_print = now_s();
          }
        }
        continue;
      }
      // q = A p with its column norms fused; r = A^T s likewise
      const int nq = op_a(c, k, pp, q, part);
      reduce_parts(c, nq, k, part, qq);
      cgls_xs(c, n, m, k, gamma, qq, act, x, pp, sv, q);
      const int nr = op_at(c, k, sv, r, part);
      reduce_parts(c, nr, k, part, gnew);
      cgls_p(c, n, k, gnew, gamma, act, r, pp);
      if (rd > 0) deflate_direction(r, pp);
      std::swap(gamma, gnew);  // the new gamma is the next iteration's old one
      ++it;
      if (it % 16 == 0) {
        if (rd > 0) {
          // rounding lets the residual regain components along W, which the
          // deflated directions no longer remove; the Galerkin step on span(W)
          // (x += W Lambda^-1 (A W)^T s, s -= A W Lambda^-1 (A W)^T s) takes
          // them out again and keeps x and s consistent
          double* mu = alloc_as<double>(b_dmu, (size_t)k * rd);
          dgemm_nt_long(c, k, rd, m, sv, k, dAWs, rd, mu, b_long);
          dgemm(c, rocblas_operation_none, rocblas_operation_none, k, n, rd, 1.0, mu, k, dW, rd, 1.0, x, k);
          dgemm(c, rocblas_operation_none, rocblas_operation_none, k, m, rd, -1.0, mu, k, dAW, rd, 1.0, sv, k);
        }
        coldots(c, m, k, sv, sv, sn2, part);
        it_now = it;
        any = update_active(sn2);
        if (verbose && now_s() - last_print > 2.0) {
          int na = 0;
          double mx = 0.0;
          for (int j = 0; j < k; ++j) { na += ha[j]; mx = std::max(mx, std::sqrt(hs[j])); }
          std::fprintf(stderr, "[nsp] refine it %lld active %d max|Av| %.3e target %.3e\n",
                       (long long)it, na, mx, tau);
          std::fflush(stderr);
          last_print = now_s();
        }
      }
    }
    st.refine_iters = it;
    st.refine_defl = rd;
    sub_inplace(c, n * k, vr, x);
    // Step 3: orthonormalise (Cholesky QR twice), residual and orthogonality
    cholqr(vr);
    cholqr(vr);
    const double* vres = vr;
    const bool jacobi = c->precond && !c->precond_ic;
    if (c->precond) {
      unprecondition(c, vr, k, b_small, b_info, b_long);
      // diagonal P_R: the stored values are those of A P^{-T} (P^{-1} A P^{-T}),
      // so A V = (A P^{-T}) (P^T V), times P for the symmetric form; the
      // incomplete Cholesky P_R leaves the stored A unchanged
      if (jacobi) {
        NSP_HIP(hipMemcpyAsync(x, vr, sizeof(double) * n * k, hipMemcpyDeviceToDevice, c->stream));
        scale_rows(c, n, k, c->pdiag.as<double>(), false, x);
        vres = x;
      }
    }
    spmm_wide(c, c->A, k, vres, u);
    if (jacobi && c->sym) scale_rows(c, m, k, c->pdiag.as<double>(), false, u);
    coldots(c, m, k, u, u, sn2, part);
    double* g = alloc_as<double>(b_small, (size_t)k * k);
    gram_rows(vr, n, g);
    std::vector<double> hg((size_t)k * k);
    NSP_HIP(hipMemcpyAsync(c->pin_d, sn2, sizeof(double) * k, hipMemcpyDeviceToHost, c->stream));
    NSP_HIP(hipMemcpyAsync(c->pin_d + k, g, sizeof(double) * k * k, hipMemcpyDeviceToHost, c->stream));
    NSP_HIP(hipStreamSynchronize(c->stream));
    std::copy(c->pin_d, c->pin_d + k, hs.begin());
    std::copy(c->pin_d + k, c->pin_d + k + (size_t)k * k, hg.begin());
    double res2 = 0.0, oe = 0.0;
    for (double v : hs) res2 += v;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < k; ++j) {
        const double e = hg[i + (size_t)j * k] - (i == j ? 1.0 : 0.0);
        oe += e * e;
      }
    st.rel_resid_fro = c->normA_fro_orig > 0 ? std::sqrt(res2) / c->normA_fro_orig : std::sqrt(res2);
    st.orth_err_fro = std::sqrt(oe);
    rows_to_colmajor(c, n, k, vr, c->V.as<double>(), n);
    NSP_HIP(hipStreamSynchronize(c->stream));
    st.t_refine_s = now_s() - t0;
  }
};

}  // namespace

void solve(nsp_ctx* c) {
  const double t0 = now_s();
  c->state = 0;
  c->nullity = 0;
  if (c->prm.prec == NSP_PREC_MIXED) {
    Lanczos<float> lz(c);
    lz.run();
  } else {
    Lanczos<double> lz(c);
    lz.run();
  }
  if (c->prm.refine && c->nullity > 0) {
    // the Lanczos basis is not needed any more: give its memory to the
    // refinement's blocks (n x N each); a new lanczos_run allocates it again
    c->Z.release();
    c->Z2.release();
    Refiner rf(c, c->nullity);
    rf.run();
  } else if (c->nullity > 0) {
    if (c->precond) {
      const int k = c->nullity;
      DBuf b_vr, b_g, b_info, b_long;
      double* vr = alloc_as<double>(b_vr, (size_t)c->n * k);
      colmajor_to_rows(c, c->n, k, c->V.as<double>(), c->n, vr);
      unprecondition(c, vr, k, b_g, b_info, b_long);
      rows_to_colmajor(c, c->n, k, vr, c->V.as<double>(), c->n);
      NSP_HIP(hipStreamSynchronize(c->stream));
    }
    // orthonormality / residual of the unrefined basis are still reported
    c->stats.rel_resid_fro = -1.0;
    c->stats.orth_err_fro = -1.0;
  }
  c->stats.t_total_s = now_s() - t0;
}

// ---------------------------------------------------------------------------
// backward: W = (A^T A)^+ (I - V V^T) G_s V by CG on range(A^T); grad = SDDMM
// ---------------------------------------------------------------------------
void run_backward(nsp_ctx* c, const double* dLdV, int64_t ld, double* grad, double tol,
                  int64_t max_iter, int64_t* iters) {
  const int64_t n = c->n, m = c->m;
  const int k = c->nullity;
  if (iters) *iters = 0;
  if (k == 0) {
    if (c->nnz) NSP_HIP(hipMemsetAsync(grad, 0, sizeof(double) * c->nnz, c->stream));
    NSP_HIP(hipStreamSynchronize(c->stream));
    return;
  }
  DBuf b_v, b_g, b_w, b_r, b_p, b_q, b_y, b_mm, b_dots, b_part, b_act;
  c->pin_d = c->pind.ensure(std::max<size_t>((size_t)c->prm.max_dim + 16, (size_t)k + 16));
  c->pin_i = c->pini.ensure(std::max<size_t>(64, (size_t)k + 16));
  double* vr = alloc_as<double>(b_v, (size_t)n * k);
  double* r = alloc_as<double>(b_r, (size_t)n * k);
  colmajor_to_rows(c, n, k, c->V.as<double>(), n, vr);
  {
    // dL/dV arrives in the caller's order of the unknowns
    DBuf b_gc;
    double* gc = alloc_as<double>(b_gc, (size_t)n * k);
    gather_rows(c, n, k, c->colperm.as<int32_t>(), dLdV, ld, gc, n);
    colmajor_to_rows(c, n, k, gc, n, r);
    NSP_HIP(hipStreamSynchronize(c->stream));
  }
  // R = G - V (V^T G)
  DBuf b_long;
  double* mm = alloc_as<double>(b_mm, (size_t)k * k);
  dgemm_nt_long(c, k, k, n, vr, k, r, k, mm, b_long);
  dgemm(c, rocblas_operation_transpose, rocblas_operation_none, k, n, k, -1.0, mm, k, vr, k, 1.0, r, k);
  // The solve only needs the range of R: R^T R = Y S^2 Y^T, keep the kr
  // directions with s^2 > 1e-13 s_max^2 (the eigenvalues of the Gram matrix
  // carry an absolute error of a few u s_max^2, so smaller ones are noise),
  // U = (I - V V^T) R Y_r S_r^{-1}, solve A^T A W_U = U and recombine
  // W = W_U S_r Y_r^T.  A loss of low rank (e.g. ||P X||_F^2 with X of a few
  // columns) needs only that many CG columns.
  DBuf b_eg, b_ew, b_ei, b_einfo, b_u, b_cr;
  double* eg = alloc_as<double>(b_eg, (size_t)k * k);
  double* ew = alloc_as<double>(b_ew, (size_t)k);
  dgemm_nt_long(c, k, k, n, r, k, r, k, eg, b_long);
  syevd(c, k, eg, ew, b_ei, b_einfo);
  std::vector<double> lam(k), yv((size_t)k * k);
  NSP_HIP(hipMemcpy(lam.data(), ew, sizeof(double) * k, hipMemcpyDeviceToHost));
  NSP_HIP(hipMemcpy(yv.data(), eg, sizeof(double) * k * k, hipMemcpyDeviceToHost));
  for (double v : lam)
    if (!std::isfinite(v)) throw Error(NSP_ERR_NONFINITE, "non-finite value in G_s V");
  const double lmax = std::max(lam[k - 1], 0.0);
  int kr = 0;
  while (kr < k && lam[k - 1 - kr] > 1e-13 * lmax && lam[k - 1 - kr] > 0.0) ++kr;
  if (kr == 0) {  // R = 0: the loss does not move the null space
    if (c->nnz) NSP_HIP(hipMemsetAsync(grad, 0, sizeof(double) * c->nnz, c->stream));
    NSP_HIP(hipStreamSynchronize(c->stream));
    return;
  }
  // Ys = Y_r S_r^{-1} (k x kr) and C = S_r Y_r^T (kr x k), column-major
  std::vector<double> ys((size_t)k * kr), cr((size_t)kr * k);
  for (int j = 0; j < kr; ++j) {
    const int col = k - 1 - j;
    const double sv = std::sqrt(lam[col]);
    for (int i = 0; i < k; ++i) {
      ys[i + (size_t)j * k] = yv[i + (size_t)col * k] / sv;
      cr[j + (size_t)i * kr] = sv * yv[i + (size_t)col * k];
    }
  }
  double* ysd = alloc_as<double>(b_eg, (size_t)k * kr);
  double* crd = alloc_as<double>(b_cr, (size_t)kr * k);
  NSP_HIP(hipMemcpy(ysd, ys.data(), sizeof(double) * ys.size(), hipMemcpyHostToDevice));
  NSP_HIP(hipMemcpy(crd, cr.data(), sizeof(double) * cr.size(), hipMemcpyHostToDevice));
  // U (row-major n x kr) = R Ys: column-major views Ucm (kr x n) = Ys^T Rcm
  double* u = alloc_as<double>(b_u, (size_t)n * kr);
  dgemm(c, rocblas_operation_transpose, rocblas_operation_none, kr, n, k, 1.0, ysd, k, r, k, 0.0, u, kr);
  NSP_HIP(hipMemcpyAsync(r, u, sizeof(double) * n * kr, hipMemcpyDeviceToDevice, c->stream));
  const int kc = kr;  // CG columns
  {
    // U -= V (V^T U): rounding in R leaves null-space components CG cannot reduce
    double* vu = alloc_as<double>(b_mm, (size_t)k * kc);
    dgemm_nt_long(c, k, kc, n, vr, k, r, kc, vu, b_long);
    dgemm(c, rocblas_operation_transpose, rocblas_operation_none, kc, n, k, -1.0, vu, k, vr, k, 1.0, r, kc);
  }
  // Outer preconditioning: A^T A W = U is P (A P^{-T})^T (A P^{-T}) P^T W = U, so
  // the CG solves for X = P^T W with right-hand side P^{-1} U and keeps its
  // residual orthogonal to null(A P^{-T}) = span(V_R); A W = (A P^{-T}) X.
  const double* vrange = vr;
  DBuf b_vs;
  if (c->precond) {
    double* vs = alloc_as<double>(b_vs, (size_t)n * k);
    colmajor_to_rows(c, n, k, c->Vs.as<double>(), n, vs);
    if (c->precond_ic) ic_solve_l<double>(c, kc, r);
    else scale_rows(c, n, kc, c->pdiag.as<double>(), true, r);
    vrange = vs;
  }
  double* w = alloc_as<double>(b_w, (size_t)n * kc);
  double* pp = alloc_as<double>(b_p, (size_t)n * kc);
  double* q = alloc_as<double>(b_q, (size_t)n * kc);
  double* y = alloc_as<double>(b_y, (size_t)m * std::max(kc, k));
  double* dots = alloc_as<double>(b_dots, (size_t)3 * kc);
  double* part = alloc_as<double>(b_part, (size_t)coldots_parts(std::max(n, m)) * kc);
  int* act = alloc_as<int>(b_act, kc);
  double *rr = dots, *pq = dots + kc, *rnew = dots + 2 * kc;
  // the tolerance is relative to the right-hand side's column norms
  coldots(c, n, kc, r, r, rr, part);
  std::vector<double> r0(kc), hr(kc);
  std::vector<int> ha(kc);
  NSP_HIP(hipMemcpyAsync(c->pin_d, rr, sizeof(double) * kc, hipMemcpyDeviceToHost, c->stream));
  NSP_HIP(hipStreamSynchronize(c->stream));
  std::copy(c->pin_d, c->pin_d + kc, r0.begin());
  // Deflated CG with the Ritz vectors above the null cluster (as in the
  // refinement): x0 = W Lambda^-1 W^T b, r0 = b - A^T A x0, directions kept
  // A^T A-orthogonal to W.
  build_deflation(c);
  const int rd = c->df_r;
  if (rd > 0) tol = std::max(tol, 1e-12);  // the deflated recurrence's attainable level
  DBuf b_mu;
  double* mu = rd > 0 ? alloc_as<double>(b_mu, (size_t)kc * rd) : nullptr;
  // For a right-hand side of 1, 2, 4 or 8 columns the two products of every
  // iteration are the tall-skinny pair of the reorthogonalisation (HBM
  // streaming kernels) on column-major copies of W and M W_s; a library GEMM
  // with a few columns reads the long operand far below the HBM rate.
  const bool ts_defl = rd > 0 && (kc == 1 || kc == 2 || kc == 4 || kc == 8);
  const int64_t ldd = (n + 63) / 64 * 64;
  DBuf b_wcm, b_mcm, b_hp;
  double *wcm = nullptr, *mcm = nullptr, *hp = nullptr;
  if (ts_defl) {
    wcm = alloc_as<double>(b_wcm, (size_t)(ldd * rd));
    mcm = alloc_as<double>(b_mcm, (size_t)(ldd * rd));
    rows_to_colmajor(c, n, rd, c->dfW.as<double>(), wcm, ldd);
    rows_to_colmajor(c, n, rd, c->dfMWs.as<double>(), mcm, ldd);
    hp = alloc_as<double>(b_hp, (size_t)ts_tn_parts_len(n, rd, kc));
  }
  auto deflate_direction = [&](const double* res, double* dir) {
    if (ts_defl) {
      ts_tn_only(c, kc, n, mcm, ldd, rd, res, mu, hp);
      ts_nn_only(c, kc, n, wcm, ldd, rd, mu, dir);
      return;
    }
    dgemm_nt_long(c, kc, rd, n, res, kc, c->dfMWs.as<double>(), rd, mu, b_long);
    dgemm(c, rocblas_operation_none, rocblas_operation_none, kc, n, rd, -1.0, mu, kc,
          c->dfW.as<double>(), rd, 1.0, dir, kc);
  };
  if (rd > 0) {
    dgemm_nt_long(c, kc, rd, n, r, kc, c->dfW.as<double>(), rd, mu, b_long);
    dgemm(c, rocblas_operation_none, rocblas_operation_none, kc, n, rd, 1.0, mu, kc,
          c->dfWs.as<double>(), rd, 0.0, w, kc);
    // r = b - A^T (A x0) with the SpMV pair (not through the stored A^T A W,
    // whose rounding would cap the attainable residual at u kappa(A^T A))
    op_a(c, kc, w, y);
    op_at(c, kc, y, q);
    sub_inplace(c, n * kc, r, q);
  } else {
    NSP_HIP(hipMemsetAsync(w, 0, sizeof(double) * n * kc, c->stream));
  }
  NSP_HIP(hipMemcpyAsync(pp, r, sizeof(double) * n * kc, hipMemcpyDeviceToDevice, c->stream));
  if (rd > 0) deflate_direction(r, pp);
  coldots(c, n, kc, r, r, rr, part);
  bool any = false;
  for (int j = 0; j < kc; ++j) {
    r0[j] = std::sqrt(r0[j]);
    ha[j] = r0[j] > 0.0 ? 1 : 0;
    any |= ha[j] != 0;
  }
  std::copy(ha.begin(), ha.end(), c->pin_i);
  NSP_HIP(hipMemcpyAsync(act, c->pin_i, sizeof(int) * kc, hipMemcpyHostToDevice, c->stream));
  NSP_HIP(hipStreamSynchronize(c->stream));
  double* mv = alloc_as<double>(b_mm, (size_t)k * kc);
  int64_t it = 0, last_gain = 0;
  double best_rel = std::numeric_limits<double>::infinity();
  bool stagnated = false;
  while (any && it < max_iter) {
    // q = A^T (A p); p^T q = ||A p||^2 comes fused with the first product
    const int ny = op_a(c, kc, pp, y, part);
    reduce_parts(c, ny, kc, part, pq);
    op_at(c, kc, y, q);
    cg_wr(c, n, kc, rr, pq, act, w, pp, r, q);
    coldots(c, n, kc, r, r, rnew, part);
    cgls_p(c, n, kc, rnew, rr, act, r, pp);
    if (rd > 0) deflate_direction(r, pp);
    std::swap(rr, rnew);  // the new r^T r is the next iteration's old one
    ++it;
    if (it % 16 == 0) {
      // re-project the residual onto range(A^T): V is a null basis only to
      // rounding accuracy, and A^T A cannot reduce a residual component in
      // null(A) (a no-op in exact arithmetic, where r stays in the range)
      dgemm_nt_long(c, k, kc, n, vrange, k, r, kc, mv, b_long);
      dgemm(c, rocblas_operation_transpose, rocblas_operation_none, kc, n, k, -1.0, mv, k, vrange, k, 1.0,
            r, kc);
      if (rd > 0) {
        // The recursive residual drifts back into span(W) by rounding, and
        // directions deflated against r alone stop removing that part: once
        // it dominates, the iteration diverges (seen on a 5000-column planted
        // matrix with kappa(A^T A) ~ 5e6 after ~1000 iterations).  The
        // Galerkin step on span(W), x += W Lambda^-1 W^T r and
        // r -= A^T A W Lambda^-1 W^T r, removes it and keeps x and r consistent.
        dgemm_nt_long(c, kc, rd, n, r, kc, c->dfW.as<double>(), rd, mu, b_long);
        dgemm(c, rocblas_operation_none, rocblas_operation_none, kc, n, rd, 1.0, mu, kc,
              c->dfWs.as<double>(), rd, 1.0, w, kc);
        dgemm(c, rocblas_operation_none, rocblas_operation_none, kc, n, rd, -1.0, mu, kc,
              c->dfMWs.as<double>(), rd, 1.0, r, kc);
      }
      coldots(c, n, kc, r, r, rr, part);
      NSP_HIP(hipMemcpyAsync(c->pin_d, rr, sizeof(double) * kc, hipMemcpyDeviceToHost, c->stream));
      NSP_HIP(hipStreamSynchronize(c->stream));
      std::copy(c->pin_d, c->pin_d + kc, hr.begin());
      any = false;
      double worst = 0.0;
      for (int j = 0; j < kc; ++j) {
        if (!std::isfinite(hr[j])) throw Error(NSP_ERR_NONFINITE, "non-finite value in backward CG");
        ha[j] = std::sqrt(hr[j]) > tol * r0[j] ? 1 : 0;
        any |= ha[j] != 0;
        if (ha[j]) worst = std::max(worst, std::sqrt(hr[j]) / r0[j]);
      }
      // attainable level: the residual's component along null(A) is removed
      // only to the accuracy of V, so a target below it cannot be reached; a
      // run whose largest relative residual has not dropped by 1% within 4096
      // iterations stops there (as the refinement does)
      if (worst < 0.99 * best_rel) {
        best_rel = worst;
        last_gain = it;
      }
      if (any && it - last_gain > 4096) {
        any = false;
        stagnated = true;
      }
      std::copy(ha.begin(), ha.end(), c->pin_i);
      NSP_HIP(hipMemcpyAsync(act, c->pin_i, sizeof(int) * kc, hipMemcpyHostToDevice, c->stream));
      NSP_HIP(hipStreamSynchronize(c->stream));
    }
  }
  // W = W_U C (row-major n x k): Wcm (k x n) = C^T W_Ucm; the buffer u is free now
  // (preconditioned: X = X_U C, and A W = (A P^{-T}) X below).  The right-hand
  // side so far was dL/dV; the projector's symmetric gradient enters as
  // G_s V = (dL/dV) / 2, hence the factor 1/2 here (W is linear in it).
  double* wf = alloc_as<double>(b_u, (size_t)n * k);
  dgemm(c, rocblas_operation_transpose, rocblas_operation_none, k, n, kc, 0.5, crd, kc, w, kc, 0.0, wf, k);
  // Y = A W, grad_p = -2 <Y_i, V_j>
  op_a(c, k, wf, y);
  {
    // gradient per stored nonzero, then back to the caller's order
    DBuf b_gs;
    double* gs = alloc_as<double>(b_gs, (size_t)std::max<int64_t>(c->nnz, 1));
    sddmm(c, k, y, vr, gs);
    scatter_vals(c, gs, grad);
    NSP_HIP(hipStreamSynchronize(c->stream));
  }
  if (iters) *iters = it;
  if (any) throw Error(NSP_ERR_NOCONV, "backward CG reached max_iter");
  (void)stagnated;
}

}  // namespace nsp
