// C ABI entry points (include/nullspace.h).  Validation, error codes, the
// thread-local error message and context ownership live here; the numerical
// work is in kernels_*.hip and solver.hip.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace {

thread_local std::string g_last_error;

template <typename F>
nsp_status guarded(F&& f) {
  try {
    g_last_error.clear();
    f();
    return NSP_OK;
  } catch (const nsp::Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return NSP_ERR_NOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return NSP_ERR_HIP;
  } catch (...) {
    g_last_error = "unknown error";
    return NSP_ERR_HIP;
  }
}

// Order the library's stream after the caller's stream (call entry) and the
// caller's stream after the library's (call exit).
void enter(nsp_ctx* c) {
  NSP_HIP(hipEventRecord(c->ev_in, c->user_stream));
  NSP_HIP(hipStreamWaitEvent(c->stream, c->ev_in, 0));
}
void leave(nsp_ctx* c) {
  NSP_HIP(hipEventRecord(c->ev_out, c->stream));
  NSP_HIP(hipStreamWaitEvent(c->user_stream, c->ev_out, 0));
}

void validate_params(const nsp_params* p, int64_t n) {
  NSP_REQUIRE(p != nullptr, "params must not be NULL");
  NSP_REQUIRE(std::isfinite(p->eps) && p->eps > 0.0, "eps must be finite and > 0");
  NSP_REQUIRE(p->d == 1 || p->d == 2 || p->d == 4 || p->d == 8, "d must be 1, 2, 4 or 8");
  NSP_REQUIRE(p->max_dim % p->d == 0, "max_dim must be a multiple of d");
  NSP_REQUIRE(p->max_dim >= 3 * p->d, "max_dim must be at least 3d");
  NSP_REQUIRE((int64_t)p->max_dim + p->d <= n, "max_dim + d must not exceed n");
  NSP_REQUIRE(p->max_dim <= 8192, "max_dim must be at most 8192");
  NSP_REQUIRE(p->max_matvec > 0, "max_matvec must be positive");
  NSP_REQUIRE(p->prec == NSP_PREC_FP64 || p->prec == NSP_PREC_MIXED, "unknown precision mode");
  NSP_REQUIRE(p->ro_tol >= 0.0 && p->ro_tol < 1.0, "ro_tol must be in [0, 1)");
  NSP_REQUIRE(p->tol_rel_resid >= 0.0 && p->tol_abs_resid >= 0.0 && p->tol_angle >= 0.0,
              "tolerances must be >= 0");
  NSP_REQUIRE(p->max_cycles >= 0, "max_cycles must be >= 0");
  NSP_REQUIRE(p->reorder == 0 || p->reorder == 1, "reorder must be 0 or 1");
  NSP_REQUIRE(p->op == NSP_OP_NORMAL || p->op == NSP_OP_SYM, "op must be NSP_OP_NORMAL or NSP_OP_SYM");
  NSP_REQUIRE(p->precond == NSP_PRECOND_NONE || p->precond == NSP_PRECOND_JACOBI ||
                  p->precond == NSP_PRECOND_IC,
              "precond must be NSP_PRECOND_NONE, NSP_PRECOND_JACOBI or NSP_PRECOND_IC");
  NSP_REQUIRE(std::isfinite(p->ic_droptol) && p->ic_droptol >= 0.0 && std::isfinite(p->ic_diagcomp) &&
                  p->ic_diagcomp >= 0.0,
              "ic_droptol and ic_diagcomp must be finite and >= 0");
}


// Rayleigh-Ritz step on T for testing (d x d blocks, see nullspace.h): a
// bound on ||T|| from host copies (largest absolute row sum), block-indexed
// device copies of Xi and Gamma, then the solver's eigensolver.
void ritz_eig_blocks(nsp_ctx* ctx, int32_t K, int32_t d, int32_t kk, const double* theta, const double* f,
                     const double* xib, const double* gamb, double* evals, double* evecs) {
  const int L = K / d, l0 = kk / d, nbk = L - l0;
  const size_t dd = (size_t)d * d;
  std::vector<double> ht(kk), hf((size_t)d * kk), hx(nbk * dd), hg(std::max(nbk - 1, 0) * dd);
  if (kk) {
    NSP_HIP(hipMemcpy(ht.data(), theta, sizeof(double) * kk, hipMemcpyDeviceToHost));
    NSP_HIP(hipMemcpy(hf.data(), f, sizeof(double) * d * kk, hipMemcpyDeviceToHost));
  }
  NSP_HIP(hipMemcpy(hx.data(), xib, sizeof(double) * hx.size(), hipMemcpyDeviceToHost));
  if (!hg.empty()) NSP_HIP(hipMemcpy(hg.data(), gamb, sizeof(double) * hg.size(), hipMemcpyDeviceToHost));
  double bound = 0.0;
  for (int i = 0; i < kk; ++i) {
    double r = std::fabs(ht[i]);
    for (int q = 0; q < d; ++q) r += std::fabs(hf[q + (size_t)i * d]);
    bound = std::max(bound, r);
  }
  for (int j = 0; j < nbk; ++j)
    for (int r = 0; r < d; ++r) {
      double sum = 0.0;
      for (int c2 = 0; c2 < d; ++c2) {
        sum += std::fabs(hx[j * dd + r + (size_t)c2 * d]);
        if (j > 0) sum += std::fabs(hg[(j - 1) * dd + r + (size_t)c2 * d]);      // T(blk j, blk j-1)
        if (j + 1 < nbk) sum += std::fabs(hg[j * dd + c2 + (size_t)r * d]);      // T(blk j, blk j+1)
      }
      if (j == 0)
        for (int i = 0; i < kk; ++i) sum += std::fabs(hf[r + (size_t)i * d]);
      bound = std::max(bound, sum);
    }
  nsp::DBuf xi, gam;
  xi.alloc(sizeof(double) * (size_t)(L + 2) * dd);
  gam.alloc(sizeof(double) * (size_t)(L + 2) * dd);
  NSP_HIP(hipMemsetAsync(xi.p, 0, sizeof(double) * (L + 2) * dd, ctx->stream));
  NSP_HIP(hipMemsetAsync(gam.p, 0, sizeof(double) * (L + 2) * dd, ctx->stream));
  NSP_HIP(hipMemcpyAsync(xi.as<double>() + (size_t)(l0 + 1) * dd, xib, sizeof(double) * nbk * dd,
                         hipMemcpyDeviceToDevice, ctx->stream));
  if (nbk > 1)
    NSP_HIP(hipMemcpyAsync(gam.as<double>() + (size_t)(l0 + 1) * dd, gamb, sizeof(double) * (nbk - 1) * dd,
                           hipMemcpyDeviceToDevice, ctx->stream));
  nsp::EigWork* w = nsp::eig_work_new();
  try {
    nsp::eig_restart(ctx, *w, K, d, kk, bound, theta, f, xi.as<double>(), gam.as<double>(), evals, evecs);
    NSP_HIP(hipStreamSynchronize(ctx->stream));
  } catch (...) {
    nsp::eig_work_delete(w);
    throw;
  }
  nsp::eig_work_delete(w);
}

}  // namespace

extern "C" {

void nsp_default_params(nsp_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->eps = 1e-3;
  p->d = 1;
  p->max_dim = 64;
  p->max_matvec = 10000000;
  p->ro_tol = 0.0;
  p->prec = NSP_PREC_FP64;
  p->refine = 1;
  p->tol_rel_resid = 1e-10;
  p->tol_abs_resid = 0.0;
  p->tol_angle = 1e-9;
  p->max_refine_iter = 1000000;
  p->max_cycles = 0;
  p->profile = 0;
  p->reorder = 1;
  p->op = NSP_OP_NORMAL;
  p->precond = NSP_PRECOND_NONE;
  p->seed = 20240704ull;
  p->ic_droptol = 1e-3;
  p->ic_diagcomp = 0.1;
}

nsp_status nullspace_init(nsp_ctx** out, int64_t m, int64_t n, int64_t nnz, const int64_t* rowptr,
                          const int32_t* colind, const double* vals, const double* D,
                          const double* Omega, const nsp_params* p, void* stream) {
  if (out) *out = nullptr;
  nsp_ctx* c = nullptr;
  nsp_status st = guarded([&] {
    NSP_REQUIRE(out != nullptr, "out must not be NULL");
    NSP_REQUIRE(m >= 1 && n >= 1, "m and n must be >= 1");
    NSP_REQUIRE(nnz >= 0 && nnz < 2147483647LL, "nnz must be in [0, 2^31)");
    NSP_REQUIRE(m < 2147483647LL && n < 2147483647LL, "m and n must be < 2^31");
    NSP_REQUIRE(rowptr != nullptr, "rowptr must not be NULL");
    NSP_REQUIRE(nnz == 0 || (colind != nullptr && vals != nullptr), "colind/vals must not be NULL");
    validate_params(p, n);
    NSP_REQUIRE(p->op != NSP_OP_SYM || m == n, "op = NSP_OP_SYM needs a square A (m == n)");
    c = new nsp_ctx();
    c->m = m;
    c->n = n;
    c->nnz = nnz;
    c->prm = *p;
    c->user_stream = static_cast<hipStream_t>(stream);
    NSP_HIP(hipGetDevice(&c->device));
    nsp::noalloc_setup();  // scratch of apply_op_noalloc on this device
    NSP_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
    NSP_HIP(hipEventCreateWithFlags(&c->ev_in, hipEventDisableTiming));
    NSP_HIP(hipEventCreateWithFlags(&c->ev_out, hipEventDisableTiming));
    c->pin_d = c->pind.ensure((size_t)p->max_dim + 16);
    c->pin_i = c->pini.ensure(64);
    // the caller's arrays may still be written on its stream
    NSP_HIP(hipStreamSynchronize(c->user_stream));
    NSP_BLAS(rocblas_create_handle(&c->blas));
    NSP_BLAS(rocblas_set_stream(c->blas, c->stream));
    // per-block partials of the step reductions (stream-ordered reuse)
    c->part_xi.alloc(sizeof(double) * (nsp::kStreamBlocks + 1) * nsp::kMaxD * nsp::kMaxD);
    c->part_g.alloc(sizeof(double) * nsp::kRedBlocks * nsp::kMaxD * nsp::kMaxD);
    c->part_g2.alloc(sizeof(double) * nsp::kRedBlocks * nsp::kMaxD * nsp::kMaxD);
    nsp::prepare_matrix(c, rowptr, colind, vals);
    nsp::init_random(c, D, Omega);
    nsp::matrix_norms(c);
    nsp::precondition(c);
    if (c->precond) nsp::matrix_norms(c);  // of the preconditioned matrix
    NSP_HIP(hipStreamSynchronize(c->stream));
  });
  if (st != NSP_OK) {
    if (c) nullspace_destroy(c);
    return st;
  }
  *out = c;
  return NSP_OK;
}

nsp_status apply_op(nsp_ctx* ctx, const double* X, int64_t ldx, double* Y, int64_t ldy,
                    int32_t ncols) {
  return guarded([&] {
    NSP_REQUIRE(ctx != nullptr, "ctx must not be NULL");
    NSP_REQUIRE(ncols >= 1, "ncols must be >= 1");
    NSP_REQUIRE(X != nullptr && Y != nullptr, "X and Y must not be NULL");
    NSP_REQUIRE(ldx >= ctx->n && ldy >= ctx->n, "leading dimensions must be >= n");
    if (!ctx->values_ok) throw nsp::Error(NSP_ERR_STATE, "the last nullspace_update_values failed");
    enter(ctx);
    nsp::apply_b_colmajor(ctx, X, ldx, Y, ldy, ncols);
    leave(ctx);
  });
}

nsp_status apply_op_noalloc(nsp_ctx* ctx, const double* X, int64_t ldx, double* Y, int64_t ldy,
                            int32_t ncols) {
  return guarded([&] {
    NSP_REQUIRE(ctx != nullptr, "ctx must not be NULL");
    NSP_REQUIRE(ncols >= 1, "ncols must be >= 1");
    NSP_REQUIRE(X != nullptr && Y != nullptr, "X and Y must not be NULL");
    NSP_REQUIRE(ldx >= ctx->n && ldy >= ctx->n, "leading dimensions must be >= n");
    if (!ctx->values_ok) throw nsp::Error(NSP_ERR_STATE, "the last nullspace_update_values failed");
    enter(ctx);
    nsp::apply_b_noalloc(ctx, X, ldx, Y, ldy, ncols);
    leave(ctx);
  });
}

nsp_status lanczos_run(nsp_ctx* ctx, nsp_stats* st) {
  nsp_status s = guarded([&] {
    NSP_REQUIRE(ctx != nullptr, "ctx must not be NULL");
    if (!ctx->values_ok) throw nsp::Error(NSP_ERR_STATE, "the last nullspace_update_values failed");
    enter(ctx);
    nsp::solve(ctx);
    leave(ctx);
  });
  if (ctx && st) *st = ctx->stats;
  if (s == NSP_OK && ctx && !ctx->stats.converged) {
    g_last_error = "matvec budget or cycle limit reached before the stopping rule fired";
    return NSP_ERR_NOCONV;
  }
  return s;
}

nsp_status nullspace_nullity(nsp_ctx* ctx, int32_t* nullity) {
  return guarded([&] {
    NSP_REQUIRE(ctx != nullptr && nullity != nullptr, "arguments must not be NULL");
    NSP_REQUIRE(ctx->state >= 1, "no basis yet: call lanczos_run first");
    *nullity = ctx->nullity;
  });
}

nsp_status extract_basis(nsp_ctx* ctx, double* V, int64_t ldv) {
  return guarded([&] {
    NSP_REQUIRE(ctx != nullptr, "ctx must not be NULL");
    if (ctx->state < 1) throw nsp::Error(NSP_ERR_STATE, "no basis yet: call lanczos_run first");
    if (ctx->nullity == 0) return;
    NSP_REQUIRE(V != nullptr && ldv >= ctx->n, "V must be non-NULL with ldv >= n");
    enter(ctx);
    nsp::scatter_rows(ctx, ctx->n, ctx->nullity, ctx->colperm.as<int32_t>(), ctx->V.as<double>(),
                      ctx->n, V, ldv);
    NSP_HIP(hipStreamSynchronize(ctx->stream));
  });
}

nsp_status nullspace_ritz_values(nsp_ctx* ctx, double* theta, int32_t cap, int32_t* count) {
  return guarded([&] {
    NSP_REQUIRE(ctx != nullptr && count != nullptr, "arguments must not be NULL");
    NSP_REQUIRE(cap >= 0 && (cap == 0 || theta != nullptr), "theta must hold cap values");
    const int32_t k = (int32_t)std::min<size_t>((size_t)cap, ctx->ritz.size());
    for (int32_t i = 0; i < k; ++i) theta[i] = ctx->ritz[i];
    *count = k;
  });
}

nsp_status nullspace_ritz_residuals(nsp_ctx* ctx, double* res, int32_t cap, int32_t* count) {
  return guarded([&] {
    NSP_REQUIRE(ctx != nullptr && count != nullptr, "arguments must not be NULL");
    NSP_REQUIRE(cap >= 0 && (cap == 0 || res != nullptr), "res must hold cap values");
    const int32_t k = (int32_t)std::min<size_t>((size_t)cap, ctx->ritz_res.size());
    for (int32_t i = 0; i < k; ++i) res[i] = ctx->ritz_res[i];
    *count = k;
  });
}

nsp_status nullspace_cycle_times(nsp_ctx* ctx, double* seconds, int32_t cap, int32_t* count) {
  return guarded([&] {
    NSP_REQUIRE(ctx != nullptr && count != nullptr, "arguments must not be NULL");
    NSP_REQUIRE(cap >= 0 && (cap == 0 || seconds != nullptr), "seconds must hold cap values");
    const int32_t k = (int32_t)std::min<size_t>((size_t)cap, ctx->cycle_s.size());
    for (int32_t i = 0; i < k; ++i) seconds[i] = ctx->cycle_s[i];
    *count = k;
  });
}


nsp_status nullspace_ritz_eig(nsp_ctx* ctx, int32_t K, int32_t kk, const double* theta,
                              const double* f, const double* alpha, const double* beta,
                              double* evals, double* evecs) {
  return guarded([&] {
    NSP_REQUIRE(ctx != nullptr, "ctx must not be NULL");
    NSP_REQUIRE(K >= 2 && kk >= 0 && kk <= K - 2, "need K >= 2 and 0 <= kk <= K-2");
    NSP_REQUIRE(alpha && beta && evals && evecs && (kk == 0 || (theta && f)), "NULL argument");
    enter(ctx);
    ritz_eig_blocks(ctx, K, 1, kk, theta, f, alpha, beta, evals, evecs);
    leave(ctx);
  });
}

nsp_status nullspace_ritz_eig_blocks(nsp_ctx* ctx, int32_t K, int32_t d, int32_t kk, const double* theta,
                                     const double* f, const double* xi, const double* gam, double* evals,
                                     double* evecs) {
  return guarded([&] {
    NSP_REQUIRE(ctx != nullptr, "ctx must not be NULL");
    NSP_REQUIRE(d == 1 || d == 2 || d == 4 || d == 8, "d must be 1, 2, 4 or 8");
    NSP_REQUIRE(K >= d && K % d == 0 && kk % d == 0 && kk >= 0 && (kk == 0 || kk <= K - 2 * d),
                "need K a multiple of d, kk a multiple of d, and kk = 0 or kk <= K - 2d");
    NSP_REQUIRE(K <= 4096, "K must not exceed 4096");
    NSP_REQUIRE(xi && evals && evecs && (K / d - kk / d < 2 || gam) && (kk == 0 || (theta && f)),
                "NULL argument");
    enter(ctx);
    ritz_eig_blocks(ctx, K, d, kk, theta, f, xi, gam, evals, evecs);
    leave(ctx);
  });
}

nsp_status nullspace_update_values(nsp_ctx* ctx, const double* vals) {
  return guarded([&] {
    NSP_REQUIRE(ctx != nullptr, "ctx must not be NULL");
    NSP_REQUIRE(vals != nullptr || ctx->nnz == 0, "vals must not be NULL");
    enter(ctx);
    // the previous basis and deflation space belong to the old values
    ctx->state = 0;
    ctx->nullity = 0;
    ctx->defl_r = 0;
    ctx->df_r = 0;
    ctx->ritz.clear();
    ctx->values_ok = false;
    nsp::refresh_values(ctx, vals);
    ctx->values_ok = true;
    leave(ctx);
  });
}

nsp_status backward(nsp_ctx* ctx, const double* dLdV, int64_t ld, double* grad_vals, double tol,
                    int64_t max_iter, int64_t* iters) {
  return guarded([&] {
    NSP_REQUIRE(ctx != nullptr, "ctx must not be NULL");
    if (ctx->state < 1) throw nsp::Error(NSP_ERR_STATE, "no basis yet: call lanczos_run first");
    NSP_REQUIRE(grad_vals != nullptr || ctx->nnz == 0, "grad_vals must not be NULL");
    NSP_REQUIRE(ctx->nullity == 0 || (dLdV != nullptr && ld >= ctx->n), "dLdV must be n x N, ld >= n");
    NSP_REQUIRE(tol > 0.0 && max_iter > 0, "tol and max_iter must be positive");
    NSP_REQUIRE(!(ctx->precond && ctx->sym),
                "backward does not support the preconditioned symmetric form");
    enter(ctx);
    nsp::run_backward(ctx, dLdV, ld, grad_vals, tol, max_iter, iters);
    leave(ctx);
  });
}

void nullspace_destroy(nsp_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->blas) (void)rocblas_destroy_handle(ctx->blas);
  if (ctx->ev_in) (void)hipEventDestroy(ctx->ev_in);
  if (ctx->ev_out) (void)hipEventDestroy(ctx->ev_out);
  hipStream_t s = ctx->stream;
  delete ctx;  // frees device buffers first
  if (s) (void)hipStreamDestroy(s);
}

const char* nullspace_last_error(void) { return g_last_error.c_str(); }

nsp_status nullspace_locality_order(int64_t m, int64_t n, const int64_t* rowptr,
                                    const int32_t* colind, int32_t* row_order,
                                    int32_t* col_order) {
  return guarded([&] {
    NSP_REQUIRE(m >= 1 && n >= 1 && m < 2147483647LL && n < 2147483647LL,
                "m and n must be in [1, 2^31)");
    NSP_REQUIRE(rowptr && row_order && col_order, "arguments must not be NULL");
    NSP_REQUIRE(rowptr[0] == 0 && rowptr[m] >= 0 && rowptr[m] < 2147483647LL,
                "rowptr[0] must be 0 and nnz < 2^31");
    NSP_REQUIRE(rowptr[m] == 0 || colind != nullptr, "colind must not be NULL");
    for (int64_t i = 0; i < m; ++i) NSP_REQUIRE(rowptr[i + 1] >= rowptr[i], "rowptr must be non-decreasing");
    for (int64_t p = 0; p < rowptr[m]; ++p) NSP_REQUIRE(colind[p] >= 0 && colind[p] < n, "colind out of range");
    nsp::locality_order(m, n, rowptr, colind, row_order, col_order);
  });
}

}  // extern "C"
