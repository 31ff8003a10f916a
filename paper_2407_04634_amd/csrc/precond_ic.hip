// Outer preconditioning with an incomplete Cholesky factor (Sec. 4.4, "Outer
// preconditioning"): P_R = L with L L^T ~ M + alpha diag(M), M = A (symmetric
// form) or M = A^T A (normal form).  The experiments of Sec. 5.1 precondition
// the graph Laplacians this way, with a threshold incomplete Cholesky and a
// diagonal compensation.  The Lanczos method then runs on
//     B_R = L^{-1} A^T A L^{-T} + eps D   or   L^{-1} A L^{-T} + eps D,
// which needs one solve with L^T and one with L per application.
//
// The factor is computed once on the host (left-looking, column by column,
// with the usual linked lists of the columns that reach each row) and stored
// twice on the device: L by rows (forward solve L y = b, diagonal last in each
// row) and L^T by rows (backward solve L^T y = b, diagonal first).  Each solve
// runs level by level: the rows of one level depend only on rows of earlier
// levels, so one launch solves a whole level, in place.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "common.h"
#include "device_util.h"
#include "kernels.h"

namespace nsp {

namespace {

// ---------------------------------------------------------------------------
// host: incomplete Cholesky
// ---------------------------------------------------------------------------
struct HostCsr {
  int64_t n = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
};

// M = A (the stored symmetric A) or A^T A from the stored A^T (rows = columns
// of A) and A, both in the library's order; column indices sorted.
HostCsr build_m(nsp_ctx* c) {
  auto down = [&](const Csr& a, std::vector<int32_t>& rp, std::vector<int32_t>& ci,
                  std::vector<double>& v) {
    rp.resize(a.rows + 1);
    NSP_HIP(hipMemcpy(rp.data(), a.rowptr, sizeof(int32_t) * (a.rows + 1), hipMemcpyDeviceToHost));
    ci.resize(a.nnz);
    v.resize(a.nnz);
    if (a.nnz) {
      NSP_HIP(hipMemcpy(ci.data(), a.colind, sizeof(int32_t) * a.nnz, hipMemcpyDeviceToHost));
      NSP_HIP(hipMemcpy(v.data(), a.val, sizeof(double) * a.nnz, hipMemcpyDeviceToHost));
    }
  };
  HostCsr m;
  m.n = c->n;
  std::vector<int32_t> arp, aci, trp, tci;
  std::vector<double> av, tv;
  NSP_HIP(hipStreamSynchronize(c->stream));
  down(c->A, arp, aci, av);
  if (c->sym) {
    m.rp.assign(arp.begin(), arp.end());
    m.ci = std::move(aci);
    m.v = std::move(av);
    return m;
  }
  // (A^T A)(i, :) = sum over the stored entries a_ri of row i of A^T of a_ri A(r, :)
  down(c->AT, trp, tci, tv);
  const int64_t n = c->n;
  std::vector<double> acc(n, 0.0);
  std::vector<int32_t> mark(n, -1), cols;
  m.rp.assign(1, 0);
  for (int64_t i = 0; i < n; ++i) {
    cols.clear();
    for (int32_t q = trp[i]; q < trp[i + 1]; ++q) {
      const int32_t r = tci[q];
      const double ari = tv[q];
      for (int32_t p = arp[r]; p < arp[r + 1]; ++p) {
        const int32_t j = aci[p];
        if (mark[j] != (int32_t)i) {
          mark[j] = (int32_t)i;
          acc[j] = 0.0;
          cols.push_back(j);
        }
        acc[j] += ari * av[p];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int32_t j : cols) {
      m.ci.push_back(j);
      m.v.push_back(acc[j]);
    }
    m.rp.push_back((int64_t)m.ci.size());
    if (m.ci.size() >= (size_t)INT32_MAX) throw Error(NSP_ERR_ARG, "A^T A has too many entries for IC");
  }
  return m;
}

struct HostLower {
  std::vector<int64_t> cp;  // column pointers
  std::vector<int32_t> ri;  // row indices (diagonal first, then ascending)
  std::vector<double> v;
};

// Left-looking incomplete Cholesky of Mc = M + alpha diag(M) (symmetric M, the
// upper part of row j = the lower part of column j).  Column j: w = Mc(j:n, j)
// - sum_k L(j:n, k) L(j, k) over the earlier columns k with L(j, k) != 0, then
// l_jj = sqrt(w_j) and l_ij = w_i / l_jj; droptol == 0 keeps l_ij only on M's
// pattern (IC(0)), droptol > 0 drops l_ij with |l_ij| < droptol ||Mc(j:n, j)||_1.
HostLower ict(const HostCsr& m, double alpha, double droptol, int64_t max_nnz) {
  const int64_t n = m.n;
  HostLower l;
  l.cp.assign(1, 0);
  std::vector<double> w(n, 0.0);
  std::vector<int32_t> mark(n, -1), onpat(n, -1), touched;
  std::vector<int64_t> next_pos(n, 0);     // next unused entry of column k
  std::vector<int32_t> head(n, -1), link(n, -1);  // columns k waiting at row r
  auto enqueue = [&](int32_t k) {
    const int64_t p = next_pos[k];
    if (p < l.cp[k + 1]) {
      const int32_t r = l.ri[p];
      link[k] = head[r];
      head[r] = k;
    }
  };
  for (int64_t j = 0; j < n; ++j) {
    touched.clear();
    double colnorm = 0.0;
    for (int64_t q = m.rp[j]; q < m.rp[j + 1]; ++q) {
      const int32_t i = m.ci[q];
      if (i < j) continue;
      double x = m.v[q];
      if (i == j) x *= 1.0 + alpha;
      w[i] = x;
      mark[i] = (int32_t)j;
      onpat[i] = (int32_t)j;
      touched.push_back(i);
      colnorm += std::fabs(x);
    }
    if (mark[j] != (int32_t)j) {  // empty diagonal: start from zero
      w[j] = 0.0;
      mark[j] = (int32_t)j;
      touched.push_back((int32_t)j);
    }
    int32_t k = head[j];
    head[j] = -1;
    while (k >= 0) {
      const int32_t nk = link[k];
      const int64_t p0 = next_pos[k];
      const double ljk = l.v[p0];
      for (int64_t p = p0; p < l.cp[k + 1]; ++p) {
        const int32_t i = l.ri[p];
        if (mark[i] != (int32_t)j) {
          mark[i] = (int32_t)j;
          w[i] = 0.0;
          touched.push_back(i);
        }
        w[i] -= l.v[p] * ljk;
      }
      next_pos[k] = p0 + 1;
      enqueue(k);
      k = nk;
    }
    double piv = w[j];
    // an unknown that M does not couple at all (an empty column of A, an
    // isolated vertex) keeps l_jj = 1
    if (colnorm == 0.0 && touched.size() == 1 && piv == 0.0) piv = 1.0;
    if (!(piv > 0.0) || !std::isfinite(piv))
      throw Error(NSP_ERR_ARG, "incomplete Cholesky: non-positive pivot at column " + std::to_string(j) +
                                   " (raise params.ic_diagcomp)");
    const double d = std::sqrt(piv);
    std::sort(touched.begin(), touched.end());
    l.ri.push_back((int32_t)j);
    l.v.push_back(d);
    for (int32_t i : touched) {
      if (i <= j) continue;
      const double x = w[i] / d;
      const bool keep = droptol > 0.0 ? std::fabs(x) >= droptol * colnorm : onpat[i] == (int32_t)j;
      if (keep && x != 0.0) {
        l.ri.push_back(i);
        l.v.push_back(x);
      }
    }
    l.cp.push_back((int64_t)l.ri.size());
    if ((int64_t)l.ri.size() > max_nnz)
      throw Error(NSP_ERR_ARG, "incomplete Cholesky: the factor exceeds " + std::to_string(max_nnz) +
                                   " entries (raise params.ic_droptol)");
    next_pos[j] = l.cp[j] + 1;  // first entry below the diagonal
    enqueue((int32_t)j);
  }
  return l;
}

// Level of every row for a triangular solve whose row i depends on the rows
// listed in its CSR (all earlier in the solve order ``ord``).
void levels(int64_t n, const std::vector<int32_t>& rp, const std::vector<int32_t>& ci, bool forward,
            std::vector<int32_t>& perm, std::vector<int32_t>& levptr) {
  std::vector<int32_t> lev(n, 0);
  int32_t nlev = 0;
  for (int64_t t = 0; t < n; ++t) {
    const int64_t i = forward ? t : n - 1 - t;
    int32_t lv = 0;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
      const int32_t j = ci[q];
      if (j != i) lv = std::max(lv, lev[j] + 1);
    }
    lev[i] = lv;
    nlev = std::max(nlev, lv + 1);
  }
  levptr.assign(nlev + 1, 0);
  for (int64_t i = 0; i < n; ++i) levptr[lev[i] + 1]++;
  std::partial_sum(levptr.begin(), levptr.end(), levptr.begin());
  perm.assign(n, 0);
  std::vector<int32_t> fill(levptr.begin(), levptr.end() - 1);
  for (int64_t i = 0; i < n; ++i) perm[fill[lev[i]]++] = (int32_t)i;
}

// ---------------------------------------------------------------------------
// device: one level of a triangular solve, in place, on a row-major n x k block
// ---------------------------------------------------------------------------
// DIAG_LAST: the row's diagonal is its last entry (L by rows), else its first
// (L^T by rows).  One thread per row for k == 1.
template <typename VT, bool DIAG_LAST>
__global__ void k_trsv_level1(int cnt, const int32_t* __restrict__ rows, const int32_t* __restrict__ rp,
                              const int32_t* __restrict__ ci, const double* __restrict__ v,
                              VT* __restrict__ y) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt) return;
  const int32_t i = rows[t];
  const int32_t q0 = rp[i], q1 = rp[i + 1];
  const int32_t qd = DIAG_LAST ? q1 - 1 : q0;
  double s = (double)y[i];
  for (int32_t q = DIAG_LAST ? q0 : q0 + 1; q < (DIAG_LAST ? q1 - 1 : q1); ++q)
    s = fma(-v[q], (double)y[ci[q]], s);
  y[i] = VT(s / v[qd]);
}

// k > 1 columns: one wavefront per row, lanes over the columns.
template <typename VT, bool DIAG_LAST>
__global__ void k_trsv_levelk(int cnt, int k, const int32_t* __restrict__ rows,
                              const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
                              const double* __restrict__ v, VT* __restrict__ y) {
  const int w = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int lane = threadIdx.x % kWave;
  if (w >= cnt) return;
  const int32_t i = rows[w];
  const int32_t q0 = rp[i], q1 = rp[i + 1];
  const int32_t qd = DIAG_LAST ? q1 - 1 : q0;
  const int32_t qa = DIAG_LAST ? q0 : q0 + 1, qb = DIAG_LAST ? q1 - 1 : q1;
  const double dinv = 1.0 / v[qd];
  for (int col = lane; col < k; col += kWave) {
    double s = (double)y[(int64_t)i * k + col];
    for (int32_t q = qa; q < qb; ++q) s = fma(-v[q], (double)y[(int64_t)ci[q] * k + col], s);
    y[(int64_t)i * k + col] = VT(s * dinv);
  }
}

// y = x + eps D x (k columns, row-major; the epilogue of apply_op)
__global__ void k_add_eps_dx(int64_t n, int k, double eps, const double* __restrict__ dv,
                             const double* __restrict__ x, double* __restrict__ y) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * k) return;
  y[t] = fma(eps * dv[t / k], x[t], y[t]);
}

// The Lanczos step's epilogue on P = B_R X without the perturbation (row-major
// n x D blocks): P += eps D X - Xp Gamma_prev^T, then per-block partials of
// Xi = X^T P over the stored (rounded) values, as the fused products write them.
template <typename VT, int D, bool PREV>
__global__ __launch_bounds__(kThreads) void k_step_epilogue(
    int64_t n, const VT* __restrict__ x, const double* __restrict__ dv, double eps,
    const VT* __restrict__ xp, const double* __restrict__ gprev, VT* __restrict__ p,
    double* __restrict__ part_xi) {
  constexpr int NV = D * D;
  __shared__ double gp[D * D];
  __shared__ double smem[(kThreads / kWave) * NV];
  if (PREV && threadIdx.x < D * D) gp[threadIdx.x] = gprev[threadIdx.x];
  __syncthreads();
  double dots[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) dots[i] = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    double s[D], xr[D];
    const double sd = eps * dv[r];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      xr[j] = (double)x[r * D + j];
      s[j] = fma(sd, xr[j], (double)p[r * D + j]);
    }
    if (PREV) {
      double pr[D];
#pragma unroll
      for (int j = 0; j < D; ++j) pr[j] = (double)xp[r * D + j];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double u = s[a];
#pragma unroll
        for (int q = 0; q < D; ++q) u = fma(-pr[q], gp[a + q * D], u);
        s[a] = u;
      }
    }
#pragma unroll
    for (int j = 0; j < D; ++j) {
      const VT o = VT(s[j]);
      p[r * D + j] = o;
      s[j] = (double)o;
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int q = 0; q < D; ++q) dots[a * D + q] += xr[a] * s[q];
  }
  block_sum<NV>(dots, smem);
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) part_xi[(size_t)blockIdx.x * NV + i] = dots[i];
}

void upload_tri(nsp_ctx* c, TriSolve& s, const std::vector<int32_t>& rp, const std::vector<int32_t>& ci,
                const std::vector<double>& v, bool forward) {
  std::vector<int32_t> perm;
  levels(c->n, rp, ci, forward, perm, s.levptr);
  s.rowptr.alloc(sizeof(int32_t) * rp.size());
  s.colind.alloc(sizeof(int32_t) * std::max<size_t>(ci.size(), 1));
  s.val.alloc(sizeof(double) * std::max<size_t>(v.size(), 1));
  s.perm.alloc(sizeof(int32_t) * std::max<size_t>(perm.size(), 1));
  NSP_HIP(hipMemcpy(s.rowptr.p, rp.data(), sizeof(int32_t) * rp.size(), hipMemcpyHostToDevice));
  NSP_HIP(hipMemcpy(s.colind.p, ci.data(), sizeof(int32_t) * ci.size(), hipMemcpyHostToDevice));
  NSP_HIP(hipMemcpy(s.val.p, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice));
  NSP_HIP(hipMemcpy(s.perm.p, perm.data(), sizeof(int32_t) * perm.size(), hipMemcpyHostToDevice));
  s.nnz = (int64_t)ci.size();
}

template <typename VT, bool DIAG_LAST>
void solve_levels(nsp_ctx* c, const TriSolve& s, int k, VT* y) {
  const int32_t* perm = s.perm.as<int32_t>();
  for (size_t lv = 0; lv + 1 < s.levptr.size(); ++lv) {
    const int cnt = s.levptr[lv + 1] - s.levptr[lv];
    if (cnt == 0) continue;
    if (k == 1)
      k_trsv_level1<VT, DIAG_LAST><<<(cnt + 255) / 256, 256, 0, c->stream>>>(
          cnt, perm + s.levptr[lv], s.rowptr.as<int32_t>(), s.colind.as<int32_t>(), s.val.as<double>(), y);
    else
      k_trsv_levelk<VT, DIAG_LAST><<<(cnt + 3) / 4, 256, 0, c->stream>>>(
          cnt, k, perm + s.levptr[lv], s.rowptr.as<int32_t>(), s.colind.as<int32_t>(), s.val.as<double>(), y);
  }
  NSP_HIP(hipGetLastError());
}

}  // namespace

template <typename VT>
void ic_solve_l(nsp_ctx* c, int k, VT* y) {
  solve_levels<VT, true>(c, c->ic.fwd, k, y);
}
template <typename VT>
void ic_solve_lt(nsp_ctx* c, int k, VT* y) {
  solve_levels<VT, false>(c, c->ic.bwd, k, y);
}
template void ic_solve_l<double>(nsp_ctx*, int, double*);
template void ic_solve_l<float>(nsp_ctx*, int, float*);
template void ic_solve_lt<double>(nsp_ctx*, int, double*);
template void ic_solve_lt<float>(nsp_ctx*, int, float*);

template <typename VT>
int step_epilogue(nsp_ctx* c, int d, const VT* x, const VT* xp, const double* gprev, VT* p,
                  double* part_xi) {
  const int64_t n = c->n;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kThreads - 1) / kThreads,
                                                                          kRedBlocks));
  const double* dv = c->Dv.as<double>();
  const double eps = c->prm.eps;
#define NSP_EPI(D)                                                                                  \
  case D:                                                                                           \
    if (xp) k_step_epilogue<VT, D, true><<<grid, kThreads, 0, c->stream>>>(n, x, dv, eps, xp, gprev, p, part_xi); \
    else k_step_epilogue<VT, D, false><<<grid, kThreads, 0, c->stream>>>(n, x, dv, eps, xp, gprev, p, part_xi);   \
    break;
  switch (d) {
    NSP_EPI(1) NSP_EPI(2) NSP_EPI(4) NSP_EPI(8)
    default: throw Error(NSP_ERR_ARG, "block size must be 1, 2, 4 or 8");
  }
#undef NSP_EPI
  NSP_HIP(hipGetLastError());
  return (int)grid;
}
template int step_epilogue<double>(nsp_ctx*, int, const double*, const double*, const double*, double*,
                                   double*);
template int step_epilogue<float>(nsp_ctx*, int, const float*, const float*, const double*, float*,
                                  double*);

void add_eps_dx(nsp_ctx* c, int k, const double* x, double* y) {
  const int64_t tot = c->n * (int64_t)k;
  if (tot == 0) return;
  k_add_eps_dx<<<(unsigned)((tot + 255) / 256), 256, 0, c->stream>>>(c->n, k, c->prm.eps,
                                                                    c->Dv.as<double>(), x, y);
  NSP_HIP(hipGetLastError());
}

void ic_setup(nsp_ctx* c) {
  const double alpha = c->prm.ic_diagcomp, droptol = c->prm.ic_droptol;
  HostCsr m = build_m(c);
  const int64_t mnnz = (int64_t)m.ci.size();
  const int64_t cap = std::min<int64_t>(INT32_MAX - 1, std::max<int64_t>(64 * mnnz, 1 << 20));
  HostLower l = ict(m, alpha, droptol, cap);
  const int64_t n = c->n, lnnz = (int64_t)l.ri.size();
  // L^T by rows = L by columns (diagonal first)
  std::vector<int32_t> brp(n + 1);
  for (int64_t j = 0; j <= n; ++j) brp[j] = (int32_t)l.cp[j];
  // L by rows (ascending columns, so the diagonal comes last)
  std::vector<int32_t> frp(n + 1, 0), fci(lnnz);
  std::vector<double> fv(lnnz);
  for (int64_t q = 0; q < lnnz; ++q) frp[l.ri[q] + 1]++;
  std::partial_sum(frp.begin(), frp.end(), frp.begin());
  std::vector<int32_t> fill(frp.begin(), frp.end() - 1);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t q = l.cp[j]; q < l.cp[j + 1]; ++q) {
      const int32_t i = l.ri[q];
      fci[fill[i]] = (int32_t)j;
      fv[fill[i]++] = l.v[q];
    }
  upload_tri(c, c->ic.fwd, frp, fci, fv, true);
  upload_tri(c, c->ic.bwd, brp, l.ri, l.v, false);
  c->ic.m_nnz = mnnz;
  c->precond = true;
  c->precond_ic = true;
}

}  // namespace nsp
