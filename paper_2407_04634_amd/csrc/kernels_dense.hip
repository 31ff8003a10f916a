// Dense kernels of the Lanczos step, the reorthogonalisation pair, the restart
// and the refinement / backward iterations.
//
// Layouts: the basis Z is column-major (n x cols, leading dimension ldz);
// Lanczos blocks in flight are row-interleaved (n x d row-major) so that the
// SpMM gathers read d contiguous values.  Small matrices (Xi, Gamma, R, H) are
// FP64 column-major.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "device_util.h"
#include "kernels.h"

namespace nsp {

static inline unsigned nblk(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }
static inline unsigned cap_grid(int64_t work, int per, int cap) {
  return std::max(1u, std::min<unsigned>(nblk(work, per), (unsigned)cap));
}

// ---------------------------------------------------------------------------
// small dense helpers (one thread)
// ---------------------------------------------------------------------------
// G (k x k, column-major, symmetric positive definite) = R^T R, R upper.
// Writes R and R^{-1}; returns false if a pivot is not positive relative to
// the largest diagonal entry (rank loss) or not finite.
// K is a template parameter so that the unrolled loops keep R and R^{-1} in
// registers (with a runtime size they go to per-lane scratch memory).
template <int K>
__device__ bool chol_upper_inv(const double* g, double* r, double* ri) {
  double gmax = 0.0;
#pragma unroll
  for (int i = 0; i < K; ++i) gmax = fmax(gmax, g[i + i * K]);
  bool ok = isfinite(gmax) && gmax > 0.0;
#pragma unroll
  for (int i = 0; i < K * K; ++i) { r[i] = 0.0; ri[i] = 0.0; }
#pragma unroll
  for (int j = 0; j < K; ++j) {
#pragma unroll
    for (int i = 0; i <= j; ++i) {
      double s = g[i + j * K];
#pragma unroll
      for (int l = 0; l < i; ++l) s -= r[l + i * K] * r[l + j * K];
      if (i == j) {
        if (!(s > 1e-24 * gmax) || !isfinite(s)) {
          ok = false;  // rank loss: finish with a dummy pivot, the result is replaced below
          s = 1.0;
        }
        r[j + j * K] = sqrt(s);
      } else {
        r[i + j * K] = s / r[i + i * K];
      }
    }
  }
  if (!ok) {
#pragma unroll
    for (int i = 0; i < K * K; ++i) { r[i] = 0.0; ri[i] = 0.0; }
#pragma unroll
    for (int i = 0; i < K; ++i) { r[i + i * K] = 1.0; ri[i + i * K] = 1.0; }
    return false;
  }
  // inverse of the upper triangular R, column by column
#pragma unroll
  for (int j = 0; j < K; ++j) {
    ri[j + j * K] = 1.0 / r[j + j * K];
#pragma unroll
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
#pragma unroll
      for (int l = i + 1; l <= j; ++l) s += r[i + l * K] * ri[l + j * K];
      ri[i + j * K] = -s / r[i + i * K];
    }
  }
  return true;
}

// chol_upper_inv by the threads of a block, in shared memory (for K = 16 R and
// R^{-1} do not fit one thread's registers, for K = 8 they take most of them):
// row i of R from rows 0..i-1 with its entries in parallel (each entry by the
// same formula and summation order as chol_upper_inv), then the columns of
// R^{-1} in parallel (each column as there).  g, r, ri: shared, K * K doubles;
// bad: shared int.  Every thread calls it; the result is valid in all threads.
template <int K>
__device__ bool chol_upper_inv_par(const double* g, double* r, double* ri, int* bad) {
  const int t = threadIdx.x;
  double gmax = 0.0;
  for (int i = 0; i < K; ++i) gmax = fmax(gmax, g[i + i * K]);
  const bool ok0 = isfinite(gmax) && gmax > 0.0;
  if (t == 0) *bad = ok0 ? 0 : 1;
  for (int i = t; i < K * K; i += blockDim.x) { r[i] = 0.0; ri[i] = 0.0; }
  __syncthreads();
  for (int i = 0; i < K; ++i) {
    if (t == 0) {
      double s = g[i + i * K];
      for (int l = 0; l < i; ++l) s -= r[l + i * K] * r[l + i * K];
      if (!(s > 1e-24 * gmax) || !isfinite(s)) {
        *bad = 1;  // rank loss: dummy pivot, the result is replaced below
        s = 1.0;
      }
      r[i + i * K] = sqrt(s);
    }
    __syncthreads();
    const int j = i + 1 + t;
    if (j < K) {
      double s = g[i + j * K];
      for (int l = 0; l < i; ++l) s -= r[l + i * K] * r[l + j * K];
      r[i + j * K] = s / r[i + i * K];
    }
    __syncthreads();
  }
  if (*bad) {
    __syncthreads();
    for (int i = t; i < K * K; i += blockDim.x) {
      const double e = (i % K == i / K) ? 1.0 : 0.0;
      r[i] = e;
      ri[i] = e;
    }
    __syncthreads();
    return false;
  }
  if (t < K) {
    const int j = t;
    ri[j + j * K] = 1.0 / r[j + j * K];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int l = i + 1; l <= j; ++l) s += r[i + l * K] * ri[l + j * K];
      ri[i + j * K] = -s / r[i + i * K];
    }
  }
  __syncthreads();
  return true;
}

template <int K>
__device__ double fro(const double* a) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < K * K; ++i) s += a[i] * a[i];
  return sqrt(s);
}

// ---------------------------------------------------------------------------
// W-recurrence (Sec. 4.2): column ell+1 of the bounds w_{k,j} >= ||Q_k^T Q_j||,
// blocks numbered from 1, W (ldw x ldw) column-major.  Executed by one block.
// Sets flags[0] = 1 (and counts the event in flags[3]) when a bound exceeds
// u_RO; the reorthogonalisation kernels that follow then run, and columns ell
// and ell+1 are reset to u_d here.
// ---------------------------------------------------------------------------
__device__ void wrec_block(const WArgs& a, double gi, double* red) {
  const int t = threadIdx.x, ell = a.ell, l0 = a.l0;
  const int lane = t % kWave, wid = t / kWave, nw = blockDim.x / kWave;
  const int ldw = a.ldw;
  // columns ell-1, ell (read) and ell+1 (written) of W are disjoint
  const double* __restrict__ wc = a.w + (int64_t)ell * ldw;
  const double* __restrict__ wp = a.w + (int64_t)(ell - 1) * ldw;
  double* __restrict__ wn = a.w + (int64_t)(ell + 1) * ldw;
  const double w_top = wc[l0 + 1], nxi_l = a.n_xi[ell], ngam_lm = a.n_gam[ell - 1];
  __shared__ double s_top[5];  // inputs of row l0+1, which needs the sum over the kept rows
  // Rows k = 1..ell, R per thread per pass: every load of a pass is issued
  // before the first store, so a pass costs one memory round trip.
  constexpr int R = 4;
  double sum_f = 0.0, mx = 0.0;
  for (int base = 1; base <= ell; base += R * (int)blockDim.x) {
    double wk[R], wkm[R], wkp[R], wpr[R], nt[R], nf[R], nx[R], ng[R], ngm[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int k = base + t + r * (int)blockDim.x;
      if (k <= ell) {
        wk[r] = wc[k]; wkm[r] = wc[k - 1]; wkp[r] = wc[k + 1]; wpr[r] = wp[k];
        nt[r] = a.n_theta[k]; nf[r] = a.n_f[k]; nx[r] = a.n_xi[k]; ng[r] = a.n_gam[k];
        ngm[r] = a.n_gam[k - 1];
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int k = base + t + r * (int)blockDim.x;
      if (k > ell) continue;
      double v;
      if (k == ell) {
        v = a.u_d;
      } else if (k <= l0) {
        sum_f += wk[r] * nf[r];
        v = gi * (wk[r] * (nt[r] + nxi_l) + w_top * nf[r] + wpr[r] * ngam_lm + 2.0 * a.u_d);
      } else if (k == l0 + 1) {
        s_top[0] = wk[r]; s_top[1] = nx[r]; s_top[2] = wkp[r]; s_top[3] = ng[r]; s_top[4] = wpr[r];
        continue;  // finished below, once sum_f is known
      } else {
        double acc = wk[r] * (nx[r] + nxi_l) + wkm[r] * ngm[r] + 2.0 * a.u_d;
        if (k < ell - 1) acc += wkp[r] * ng[r] + wpr[r] * ngam_lm;
        v = gi * acc;
      }
      wn[k] = v;
      if (k < ell) mx = (v == v) ? fmax(mx, v) : INFINITY;  // a NaN bound forces a reorthogonalisation
    }
  }
  sum_f = wave_sum(sum_f);
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, kWave));
  if (lane == 0) {
    red[wid] = sum_f;
    red[nw + wid] = mx;
  }
  __syncthreads();
  if (t == 0) {
    double sf = 0.0, m = 0.0;
    for (int q = 0; q < nw; ++q) {
      sf += red[q];
      m = fmax(m, red[nw + q]);
    }
    const int k = l0 + 1;
    if (k < ell) {
      double acc = s_top[0] * (s_top[1] + nxi_l) + sf + 2.0 * a.u_d;
      if (k < ell - 1) acc += s_top[2] * s_top[3] + s_top[4] * ngam_lm;
      const double v = gi * acc;
      wn[k] = v;
      m = (v == v) ? fmax(m, v) : INFINITY;
    }
    red[0] = m;
  }
  __syncthreads();
  const bool need = red[0] > a.u_ro;
  if (need) {
    double* wcw = a.w + (int64_t)ell * ldw;
    for (int k = 1 + t; k < ell; k += blockDim.x) wcw[k] = a.u_d;
    for (int k = 1 + t; k <= ell; k += blockDim.x) wn[k] = a.u_d;
  }
  if (t == 0) {
    a.flags[0] = need ? 1 : 0;
    if (need) a.flags[3] += 1;
    if (a.hist) a.hist[ell] = need ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// Lanczos step, QR part (no grid-wide synchronisation inside a kernel: each
// kernel reduces the per-block partials the previous kernel wrote, in block
// order, so results are deterministic and need no atomics or fences).
//
// k_sub_gram: [XI: Xi = sum of the Xi partials, symmetrised; block 0 stores Xi
//             and ||Xi||_F]; [SUB: P -= X Xi]; writes per-block partials of P^T P.
// ---------------------------------------------------------------------------
constexpr int kSmem = kThreads * 4;  // shared scratch doubles for block sums of <= 256 values

template <typename VT, int D, bool XI, bool SUB>
__global__ __launch_bounds__(kThreads) void k_sub_gram(int64_t n, VT* __restrict__ p,
                                                       const VT* __restrict__ x,
                                                       const double* __restrict__ part_xi,
                                                       int nparts_xi, double* xi_out,
                                                       double* nrm_xi, double* __restrict__ part_g) {
  constexpr int NV = D * D;
  __shared__ double smem[kSmem];
  __shared__ double res[NV];
  __shared__ double xs[NV];
  if constexpr (XI) {
    reduce_partials<NV>(part_xi, nparts_xi, res, smem);
    if (threadIdx.x < NV) {
      const int a = threadIdx.x % D, b = threadIdx.x / D;
      xs[threadIdx.x] = 0.5 * (res[a + b * D] + res[b + a * D]);
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      double f2 = 0.0;
      for (int i = 0; i < NV; ++i) { xi_out[i] = xs[i]; f2 += xs[i] * xs[i]; }
      if (nrm_xi) *nrm_xi = sqrt(f2);
    }
  }
  double g[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) g[i] = 0.0;
  // one row: FP64 arithmetic, one rounding to the working precision on store
  auto row = [&](int64_t r, double (&v)[D], const double (&xr)[D]) {
    if constexpr (SUB) {
      double w[D];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        double s = v[a];
#pragma unroll
        for (int b = 0; b < D; ++b) s = fma(-xr[b], xs[b + a * D], s);
        w[a] = s;
      }
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const VT o = VT(w[j]);
        p[r * D + j] = o;
        v[j] = (double)o;
      }
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) g[a + b * D] += v[a] * v[b];
  };
  // U rows per thread and pass, all their loads issued first (the rows are
  // then processed in the same order as one at a time, so the sums are too)
  constexpr int U = D <= 2 ? 4 : (D == 4 ? 2 : 1);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; r + (U - 1) * stride < n; r += U * stride) {
    double v[U][D], xr[U][D];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int j = 0; j < D; ++j) {
        v[u][j] = p[(r + u * stride) * D + j];
        xr[u][j] = SUB ? (double)x[(r + u * stride) * D + j] : 0.0;
      }
#pragma unroll
    for (int u = 0; u < U; ++u) row(r + u * stride, v[u], xr[u]);
  }
  for (; r < n; r += stride) {
    double v[D], xr[D];
#pragma unroll
    for (int j = 0; j < D; ++j) {
      v[j] = p[r * D + j];
      xr[j] = SUB ? (double)x[r * D + j] : 0.0;
    }
    row(r, v, xr);
  }
  block_sum<NV>(g, smem);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) part_g[(size_t)blockIdx.x * NV + i] = g[i];
  }
}

// k_sub_gram for block size 8 on the matrix cores: the same Xi, the same
// subtraction (per value, the same operations in the same order as k_sub_gram),
// and the Gram partials of P from g8_step with P's value as both operands.
// Grid-stride over 8-row groups, one group per wave and step; grid from
// g8_grid (at most 256 blocks).
template <typename VT, bool XI, bool SUB>
__global__ __launch_bounds__(kThreads) void k_sub_gram8(int64_t n, VT* __restrict__ p,
                                                        const VT* __restrict__ x,
                                                        const double* __restrict__ part_xi,
                                                        int nparts_xi, double* xi_out,
                                                        double* nrm_xi, double* __restrict__ part_g) {
  constexpr int D = 8, NV = D * D;
  __shared__ double smem[kSmem];
  __shared__ double res[NV];
  __shared__ double xs[NV];
  if constexpr (XI) {
    reduce_partials<NV>(part_xi, nparts_xi, res, smem);
    if (threadIdx.x < NV) {
      const int a = threadIdx.x % D, b = threadIdx.x / D;
      xs[threadIdx.x] = 0.5 * (res[a + b * D] + res[b + a * D]);
    }
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      double f2 = 0.0;
      for (int i = 0; i < NV; ++i) { xi_out[i] = xs[i]; f2 += xs[i] * xs[i]; }
      if (nrm_xi) *nrm_xi = sqrt(f2);
    }
  }
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  const int col = lane & 7, off = g8_off(lane);
  const int64_t nv = n * D;
  g8_acc acc = {0.0, 0.0, 0.0, 0.0};
  auto value = [&](int64_t idx, double v, const double (&xr)[D]) {
    if constexpr (SUB) {
      double s = v;
#pragma unroll
      for (int b = 0; b < D; ++b) s = fma(-xr[b], xs[b + col * D], s);
      const VT o = VT(s);
      p[idx] = o;
      v = (double)o;
    }
    return v;
  };
  constexpr int U = 2;  // groups per step, all loads first
  const int64_t ng = (n + 7) / 8, stride = (int64_t)gridDim.x * (kThreads / kWave);
  int64_t g = (int64_t)blockIdx.x * (kThreads / kWave) + wid;
  for (; g + (U - 1) * stride < ng; g += U * stride) {
    double v[U], xr[U][D];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t idx = (g + u * stride) * 64 + off;
      const bool in = idx < nv;
      v[u] = in ? (double)p[idx] : 0.0;
#pragma unroll
      for (int b = 0; b < D; ++b) xr[u][b] = SUB && in ? (double)x[idx - col + b] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t idx = (g + u * stride) * 64 + off;
      const double w = idx < nv ? value(idx, v[u], xr[u]) : 0.0;
      acc = g8_step(w, w, acc);
    }
  }
  for (; g < ng; g += stride) {
    const int64_t idx = g * 64 + off;
    double w = 0.0;
    if (idx < nv) {
      double xr[D];
#pragma unroll
      for (int b = 0; b < D; ++b) xr[b] = SUB ? (double)x[idx - col + b] : 0.0;
      w = value(idx, (double)p[idx], xr);
    }
    acc = g8_step(w, w, acc);
  }
  __syncthreads();  // smem is reused as the tile
  g8_finish(acc, smem, part_g + (size_t)blockIdx.x * NV);
}

// Xi partials for block size 8 (X^T P over the block's rows), on the matrix
// cores; the product kernel runs without its own Xi sums then.
template <typename VT>
__global__ __launch_bounds__(kThreads) void k_xi8(int64_t n, const VT* __restrict__ x,
                                                  const VT* __restrict__ p,
                                                  double* __restrict__ part) {
  __shared__ double tile[(kThreads / kWave) * 256];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  const int off = g8_off(lane);
  const int64_t nv = n * 8;
  g8_acc acc = {0.0, 0.0, 0.0, 0.0};
  constexpr int U = 4;
  const int64_t ng = (n + 7) / 8, stride = (int64_t)gridDim.x * (kThreads / kWave);
  int64_t g = (int64_t)blockIdx.x * (kThreads / kWave) + wid;
  for (; g + (U - 1) * stride < ng; g += U * stride) {
    double xv[U], pv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t idx = (g + u * stride) * 64 + off;
      xv[u] = idx < nv ? (double)x[idx] : 0.0;
      pv[u] = idx < nv ? (double)p[idx] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc = g8_step(xv[u], pv[u], acc);
  }
  for (; g < ng; g += stride) {
    const int64_t idx = g * 64 + off;
    acc = g8_step(idx < nv ? (double)x[idx] : 0.0, idx < nv ? (double)p[idx] : 0.0, acc);
  }
  g8_finish(acc, tile, part + (size_t)blockIdx.x * 64);
}

// Grid of the block-size-8 kernels above: one 8-row group per wave and step,
// at least 16 groups per wave and at most 256 blocks, so the next kernel's
// fixed-order sum of the partials (a few loads in flight per thread) stays
// short.
static unsigned g8_grid(int64_t n) {
  const int64_t groups = (n + 7) / 8, per_block = 16 * (kThreads / kWave);
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((groups + per_block - 1) / per_block, 256));
}

template <typename VT>
int xi8_parts(nsp_ctx* c, int64_t n, const VT* x, const VT* p, double* part) {
  const unsigned grid = g8_grid(n);
  k_xi8<VT><<<grid, kThreads, 0, c->stream>>>(n, x, p, part);
  NSP_HIP(hipGetLastError());
  return (int)grid;
}
template int xi8_parts<double>(nsp_ctx*, int64_t, const double*, const double*, double*);
template int xi8_parts<float>(nsp_ctx*, int64_t, const float*, const float*, double*);

// k_scale: G = sum of the Gram partials; Cholesky G = R^T R (every block, one
// thread); Xn = P R^{-1} written to the ring slot ``xn`` and, when zcol is not
// null, to D basis columns.  Block 0 stores R (the new Gamma), ||R||_F and
// ||R^{-1}||_F.  With GRAM it also writes the Gram partials of Xn for the
// second Cholesky-QR pass (k_scale2).
template <typename VT, int D, bool GRAM, bool WREC>
__global__ __launch_bounds__(kThreads) void k_scale(int64_t n, const VT* p,
                                                    const double* __restrict__ part_g, int nparts,
                                                    VT* xn, VT* __restrict__ zcol, int64_t ldz,
                                                    double* gam_out, double* nrm_gam,
                                                    double* nrm_ginv, double* __restrict__ part_g2,
                                                    int* flags, WArgs wa) {
  constexpr int NV = D * D;
  __shared__ double smem[kSmem];
  __shared__ double res[NV];
  __shared__ double ri[NV];
  __shared__ double gi_s;
  reduce_partials<NV>(part_g, nparts, res, smem);
  if (threadIdx.x == 0) {
    double r[NV], rv[NV];
    const bool ok = chol_upper_inv<D>(res, r, rv);
    for (int i = 0; i < NV; ++i) ri[i] = rv[i];
    gi_s = fro<D>(rv);
    if (blockIdx.x == 0) {
      if (!ok) atomicOr(flags + 1, 1);
      if (gam_out)
        for (int i = 0; i < NV; ++i) gam_out[i] = r[i];
      if (nrm_gam) *nrm_gam = fro<D>(r);
      if (nrm_ginv) *nrm_ginv = gi_s;
    }
  }
  __syncthreads();
  // the W-recurrence needs ||Gamma_ell^{-1}||; for d = 1 the QR is final here.
  // Block 0 runs it while the other blocks scale the rows.
  if constexpr (WREC) {
    if (blockIdx.x == 0) {
      wrec_block(wa, gi_s, smem);
      return;
    }
  }
  constexpr int NG = GRAM ? NV : 1;
  double g[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) g[i] = 0.0;
  const int b0 = WREC ? 1 : 0;
  // one row: FP64 arithmetic, one rounding on store
  auto row = [&](int64_t r, const double (&v)[D]) {
    double o[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b <= a; ++b) s = fma(v[b], ri[b + a * D], s);
      const VT q = VT(s);
      o[a] = (double)q;
      xn[r * D + a] = q;
      if (zcol) zcol[r + a * ldz] = q;
    }
    if constexpr (GRAM) {
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) g[a + b * D] += o[a] * o[b];
    }
  };
  // U rows per thread and pass with their loads issued first (same row order)
  constexpr int U = D <= 2 ? 4 : (D == 4 ? 2 : 1);
  const int64_t stride = (int64_t)(gridDim.x - b0) * blockDim.x;
  int64_t r = (int64_t)(blockIdx.x - b0) * blockDim.x + threadIdx.x;
  for (; r + (U - 1) * stride < n; r += U * stride) {
    double v[U][D];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int j = 0; j < D; ++j) v[u][j] = p[(r + u * stride) * D + j];
#pragma unroll
    for (int u = 0; u < U; ++u) row(r + u * stride, v[u]);
  }
  for (; r < n; r += stride) {
    double v[D];
#pragma unroll
    for (int j = 0; j < D; ++j) v[j] = p[r * D + j];
    row(r, v);
  }
  if constexpr (GRAM) {
    block_sum<NG>(g, smem);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < NG; ++i) part_g2[(size_t)blockIdx.x * NG + i] = g[i];
    }
  }
}

// k_scale for block size 8 with the Gram partials of Xn (first Cholesky-QR
// pass) on the matrix cores.  Lane l computes value (row, l % 8) of an 8-row
// group from the whole row (the same products in the same order as k_scale)
// and feeds it to g8_step as both operands.  P and Xn may be the same array: a
// row is read and written by one wave, the loads before the stores.
// Grid-stride over 8-row groups; grid from g8_grid (at most 256 blocks).
template <typename VT>
__global__ __launch_bounds__(kThreads) void k_scale8(int64_t n, const VT* p,
                                                     const double* __restrict__ part_g, int nparts,
                                                     VT* xn, VT* __restrict__ zcol, int64_t ldz,
                                                     double* gam_out, double* nrm_gam,
                                                     double* nrm_ginv, double* __restrict__ part_g2,
                                                     int* flags) {
  constexpr int D = 8, NV = D * D;
  __shared__ double smem[kSmem];
  __shared__ double res[NV];
  __shared__ double ri[NV];
  __shared__ double rs[NV];
  __shared__ int bad;
  reduce_partials<NV>(part_g, nparts, res, smem);
  const bool ok = chol_upper_inv_par<D>(res, rs, ri, &bad);
  if (blockIdx.x == 0) {
    if (gam_out && threadIdx.x < NV) gam_out[threadIdx.x] = rs[threadIdx.x];
    if (threadIdx.x == 0) {
      if (!ok) atomicOr(flags + 1, 1);
      if (nrm_gam) *nrm_gam = fro<D>(rs);
      if (nrm_ginv) *nrm_ginv = fro<D>(ri);
    }
  }
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  const int col = lane & 7, off = g8_off(lane);
  double rc[D];  // column ``col`` of R^{-1} (upper triangular)
#pragma unroll
  for (int b = 0; b < D; ++b) rc[b] = b <= col ? ri[b + col * D] : 0.0;
  const int64_t nv = n * D;
  g8_acc acc = {0.0, 0.0, 0.0, 0.0};
  const int64_t ng = (n + 7) / 8, stride = (int64_t)gridDim.x * (kThreads / kWave);
  for (int64_t g = (int64_t)blockIdx.x * (kThreads / kWave) + wid; g < ng; g += stride) {
    const int64_t idx = g * 64 + off;
    double o = 0.0;
    if (idx < nv) {
      double v[D];
#pragma unroll
      for (int b = 0; b < D; ++b) v[b] = (double)p[idx - col + b];
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < D; ++b)
        if (b <= col) s = fma(v[b], rc[b], s);
      const VT q = VT(s);
      o = (double)q;
      xn[idx] = q;
      if (zcol) zcol[idx / D + (int64_t)col * ldz] = q;
    }
    acc = g8_step(o, o, acc);
  }
  __syncthreads();  // smem is reused as the tile
  g8_finish(acc, smem, part_g2 + (size_t)blockIdx.x * NV);
}

// Second Cholesky-QR pass (d > 1): R2 from the Gram partials of Xn; Xn <- Xn R2^{-1};
// block 0 updates Gamma <- R2 Gamma and its norms.
template <typename VT, int D, bool WREC>
__global__ __launch_bounds__(kThreads) void k_scale2(int64_t n, const double* __restrict__ part_g2,
                                                     int nparts, VT* xn, VT* __restrict__ zcol,
                                                     int64_t ldz, double* gam, double* nrm_gam,
                                                     double* nrm_ginv, int* flags, WArgs wa) {
  constexpr int NV = D * D;
  __shared__ double smem[kSmem];
  __shared__ double res[NV];
  __shared__ double ri[NV];
  __shared__ double gi_s;
  reduce_partials<NV>(part_g2, nparts, res, smem);
  __shared__ double r2s[NV];
  if constexpr (D == 8) {
    __shared__ int bad;
    const bool ok = chol_upper_inv_par<D>(res, r2s, ri, &bad);
    if (blockIdx.x == 0 && threadIdx.x == 0 && !ok) atomicOr(flags + 1, 1);
  } else if (threadIdx.x == 0) {
    double r2[NV], r2i[NV];
    const bool ok = chol_upper_inv<D>(res, r2, r2i);
    for (int i = 0; i < NV; ++i) { ri[i] = r2i[i]; r2s[i] = r2[i]; }
    if (blockIdx.x == 0 && !ok) atomicOr(flags + 1, 1);
  }
  if (blockIdx.x == 0 && gam) {
    // Gamma <- R2 Gamma and its inverse Gamma^{-1} R2^{-1}: the inverse of the
    // old (upper triangular) Gamma by columns, then one thread per entry
    __shared__ double g0[NV], g0i[NV], gn[NV], gni[NV];
    __syncthreads();
    if (threadIdx.x < NV) { g0[threadIdx.x] = gam[threadIdx.x]; g0i[threadIdx.x] = 0.0; }
    __syncthreads();
    if (threadIdx.x < D) {
      const int j = threadIdx.x;
      g0i[j + j * D] = 1.0 / g0[j + j * D];
      for (int i = j - 1; i >= 0; --i) {
        double s = 0.0;
        for (int l = i + 1; l <= j; ++l) s += g0[i + l * D] * g0i[l + j * D];
        g0i[i + j * D] = -s / g0[i + i * D];
      }
    }
    __syncthreads();
    if (threadIdx.x < NV) {
      const int i = threadIdx.x % D, j = threadIdx.x / D;
      double s = 0.0, t = 0.0;
      for (int l = 0; l < D; ++l) {
        s += r2s[i + l * D] * g0[l + j * D];
        t += g0i[i + l * D] * ri[l + j * D];
      }
      gn[threadIdx.x] = s;
      gni[threadIdx.x] = t;
      gam[threadIdx.x] = s;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (nrm_gam) *nrm_gam = fro<D>(gn);
      gi_s = fro<D>(gni);
      if (nrm_ginv) *nrm_ginv = gi_s;
    }
  }
  __syncthreads();
  if constexpr (WREC) {
    if (blockIdx.x == 0) {
      wrec_block(wa, gi_s, smem);
      return;
    }
  }
  const int b0 = WREC ? 1 : 0;
  for (int64_t r = (int64_t)(blockIdx.x - b0) * blockDim.x + threadIdx.x; r < n;
       r += (int64_t)(gridDim.x - b0) * blockDim.x) {
    double v[D];  // FP64 arithmetic, one rounding on store
#pragma unroll
    for (int j = 0; j < D; ++j) v[j] = xn[r * D + j];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b <= a; ++b) s = fma(v[b], ri[b + a * D], s);
      const VT q = VT(s);
      xn[r * D + a] = q;
      if (zcol) zcol[r + a * ldz] = q;
    }
  }
}

// W columns col0 and col0+1 := u_d (rows above the diagonal), everything else of them zero
__global__ void k_w_reset(int col0, int ncols, double u_d, double* w, int ldw) {
  for (int c = col0; c < col0 + ncols; ++c)
    for (int k = 1 + threadIdx.x; k < ldw; k += blockDim.x) w[k + (int64_t)c * ldw] = k < c ? u_d : 0.0;
}

// ---------------------------------------------------------------------------
// Tall-skinny pair of the (partial) reorthogonalisation, classical
// Gram-Schmidt (Sec. 4.2):
//   H = Z^T C   (k x NC)  k_ts_tn writes per-row-chunk partials, k_reduce_cols sums them
//   C = C - Z H           k_ts_nn_v (NC <= 8, and 16 in FP64), k_ts_nn (16 in FP32)
// C is NC columns held as NA row-interleaved arrays of DA columns each
// (NC = NA * DA): for the reorthogonalisation of [Q_ell, Q_ell+1] NA = 2.
// When ``cond`` is non-null the kernels do nothing unless *cond != 0.
// ---------------------------------------------------------------------------
template <typename VT, int DA, int NA>
struct CPair {
  VT* a0;
  VT* a1;
  __device__ __forceinline__ VT get(int64_t r, int c) const {
    return (NA == 1 || c < DA) ? a0[r * DA + c] : a1[r * DA + (c - DA)];
  }
  __device__ __forceinline__ void set(int64_t r, int c, VT v) const {
    if (NA == 1 || c < DA) a0[r * DA + c] = v; else a1[r * DA + (c - DA)] = v;
  }
};

// Basis columns per wave (JW) and per block (JB) of the projection kernel.
// Each column is one 16-byte load per lane and row group, kept in its storage
// precision until its FMAs, so FP32 keeps as many loads in flight as FP64.
constexpr int ts_jw(int nc) { return nc >= 16 ? 4 : (nc >= 4 ? 4 : 8); }
constexpr int kTsWaves = 4;  // waves per block (8 measured slower: fewer, heavier blocks)
template <int NC, int ESIZE = 8> struct TsShape {
  static constexpr int JW = ts_jw(NC);
  static constexpr int NWT = kTsWaves;
  static constexpr int JB = NWT * JW;
};

// Rows one lane loads at once from a basis column: 16 bytes per load.
template <typename VT> struct RowVec;
template <> struct RowVec<double> { static constexpr int R = 2; using T = double2; };
template <> struct RowVec<float> { static constexpr int R = 4; using T = float4; };

// The DA values of one row of a row-interleaved block (16-byte loads where the
// row is a whole number of them; rows are 16-byte aligned then).
template <typename VT, int DA>
__device__ __forceinline__ void load_crow(const VT* __restrict__ p, double (&o)[DA]) {
  if constexpr (sizeof(VT) == 8 && DA % 2 == 0) {
#pragma unroll
    for (int q = 0; q < DA / 2; ++q) {
      const double2 t = reinterpret_cast<const double2*>(p)[q];
      o[2 * q] = t.x;
      o[2 * q + 1] = t.y;
    }
  } else if constexpr (sizeof(VT) == 4 && DA % 4 == 0) {
#pragma unroll
    for (int q = 0; q < DA / 4; ++q) {
      const float4 t = reinterpret_cast<const float4*>(p)[q];
      o[4 * q] = t.x;
      o[4 * q + 1] = t.y;
      o[4 * q + 2] = t.z;
      o[4 * q + 3] = t.w;
    }
  } else {
#pragma unroll
    for (int c = 0; c < DA; ++c) o[c] = (double)p[c];
  }
}

// RV consecutive rows of a column as one 16-byte vector (zeros past n)
template <typename VT>
__device__ __forceinline__ typename RowVec<VT>::T load_vec(const VT* __restrict__ p, int64_t r,
                                                           int64_t n) {
  using V = typename RowVec<VT>::T;
  constexpr int R = RowVec<VT>::R;
  if (r + R <= n) return *reinterpret_cast<const V*>(p + r);
  VT t[R];
#pragma unroll
  for (int i = 0; i < R; ++i) t[i] = r + i < n ? p[r + i] : VT(0);
  if constexpr (R == 2) return V{t[0], t[1]};
  else return V{t[0], t[1], t[2], t[3]};
}

template <typename V>
__device__ __forceinline__ double vec_elem(const V& v, int i) {
  if constexpr (sizeof(v.x) == 8) return i == 0 ? v.x : v.y;
  else return (double)(i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w);
}

template <typename VT>
__device__ __forceinline__ void load_rows(const VT* __restrict__ p, int64_t r, int64_t n,
                                          double (&v)[RowVec<VT>::R]) {
  constexpr int R = RowVec<VT>::R;
  if (r + R <= n) {
    const typename RowVec<VT>::T t = *reinterpret_cast<const typename RowVec<VT>::T*>(p + r);
    if constexpr (R == 2) {
      v[0] = t.x; v[1] = t.y;
    } else {
      v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
    }
  } else {
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = r + i < n ? (double)p[r + i] : 0.0;
  }
}

// grid (row chunks, column groups); wave w of a block owns JW columns, lanes stride rows
template <typename VT, int DA, int NA>
__global__ __launch_bounds__(kThreads) void k_ts_tn(const int* cond, int64_t n, int64_t chunk,
                                                    const VT* __restrict__ z, int64_t ldz, int k,
                                                    CPair<VT, DA, NA> cc, double* __restrict__ hpart) {
  constexpr int NC = DA * NA;
  constexpr int JW = TsShape<NC, sizeof(VT)>::JW;
  if (cond && *cond == 0) return;
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = min(n, r0 + chunk);
  const int j0 = blockIdx.y * TsShape<NC, sizeof(VT)>::JB + wid * JW;
  const int jn = max(0, min(JW, k - j0));
  double acc[JW][NC];
#pragma unroll
  for (int q = 0; q < JW; ++q)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[q][c] = 0.0;
  // lanes take RV consecutive rows each (one 16-byte load per basis column);
  // chunks start at multiples of 64 * RV rows, so the vector loads are aligned
  constexpr int RV = RowVec<VT>::R;
  if (jn > 0) {
    for (int64_t r = r0 + (int64_t)lane * RV; r < r1; r += kWave * RV) {
      double cv[RV][NC];
      if constexpr (DA == 1) {
        // C columns are plain vectors: the same 16-byte row loads as Z
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          double t[RV];
          load_rows<VT>(c == 0 ? cc.a0 : cc.a1, r, r1, t);
#pragma unroll
          for (int i = 0; i < RV; ++i) cv[i][c] = t[i];
        }
      } else {
#pragma unroll
        for (int i = 0; i < RV; ++i) {
          double t0[DA], t1[DA];
          if (r + i < r1) {
            load_crow<VT, DA>(cc.a0 + (r + i) * DA, t0);
            if constexpr (NA == 2) load_crow<VT, DA>(cc.a1 + (r + i) * DA, t1);
          } else {
#pragma unroll
            for (int c = 0; c < DA; ++c) { t0[c] = 0.0; t1[c] = 0.0; }
          }
#pragma unroll
          for (int c = 0; c < DA; ++c) {
            cv[i][c] = t0[c];
            if constexpr (NA == 2) cv[i][DA + c] = t1[c];
          }
        }
      }
      // the JW column loads are issued together and stay in the storage
      // precision (half the registers for FP32) until the FMAs
      typename RowVec<VT>::T zv[JW];
#pragma unroll
      for (int q = 0; q < JW; ++q) {
        if (q < jn) zv[q] = load_vec<VT>(z + (int64_t)(j0 + q) * ldz, r, r1);
        else zv[q] = typename RowVec<VT>::T{};
      }
#pragma unroll
      for (int q = 0; q < JW; ++q)
#pragma unroll
        for (int i = 0; i < RV; ++i) {
          const double zq = vec_elem(zv[q], i);
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[q][c] = fma(zq, cv[i][c], acc[q][c]);
        }
    }
  }
#pragma unroll
  for (int q = 0; q < JW; ++q)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double v = wave_sum(acc[q][c]);
      if (lane == 0 && q < jn) hpart[((int64_t)blockIdx.x * k + j0 + q) * NC + c] = v;
    }
}

// H = Z^T C for the 16-column FP64 pair (d = 8) on the matrix cores.  With 16
// columns of C the projection is a dense contraction: v_mfma_f64_16x16x4f64
// multiplies a 16 x 4 slice of Z^T (16 basis columns, 4 rows) by the 4 x 16
// slice of C on the same rows, so every C value a lane loads serves kMfTiles
// x 16 basis columns (the vector kernel reloads C for every 4 columns and
// keeps 64 accumulators per lane).  A block owns kMfCols basis columns and a
// row chunk; its 4 waves take interleaved 32-row steps of the chunk (lane
// group g = lane / 16 holds rows g*8 .. g*8+7 of the step, lane % 16 names the
// basis column in the A operand and the C column in the B operand) and their
// 16 x 16 tiles are summed in LDS in wave order.  Operand and output layout of
// the instruction (checked on the device with random operands): lane l gives
// A(l % 16, l / 16) and B(l / 16, l % 16); register v of lane l holds D(l / 16
// + 4 v, l % 16).
constexpr int kMfTiles = 4;               // 16-column tiles per block
constexpr int kMfCols = 16 * kMfTiles;    // basis columns per block
constexpr int kMfRows = 8;                // rows per lane group and step
typedef double mf_v4d __attribute__((ext_vector_type(4)));

template <int DA, int NA>
__global__ __launch_bounds__(kThreads) void k_ts_tn_mfma(const int* cond, int64_t n, int64_t chunk,
                                                         const double* __restrict__ z, int64_t ldz,
                                                         int k, CPair<double, DA, NA> cc,
                                                         double* __restrict__ hpart) {
  static_assert(DA * NA == 16 && NA == 2, "the 16-column pair");
  static_assert(kThreads == 4 * kWave, "four waves per block");
  constexpr int NC = 16;
  constexpr int STEP = 4 * kMfRows;  // rows per wave step
  if (cond && *cond == 0) return;
  __shared__ double red[4][kMfTiles][4][kWave];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  const int col = lane % 16, grp = lane / 16;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = min(n, r0 + chunk);
  const int j0 = blockIdx.y * kMfCols;
  mf_v4d acc[kMfTiles];
#pragma unroll
  for (int t = 0; t < kMfTiles; ++t) acc[t] = mf_v4d{0.0, 0.0, 0.0, 0.0};
  // the C column this lane feeds to the B operand
  const double* cp = col < DA ? cc.a0 + col : cc.a1 + (col - DA);
  const bool fullc = j0 + kMfCols <= k;  // all of the block's basis columns exist
  for (int64_t rb = r0 + (int64_t)wid * STEP; rb < r1; rb += 4 * STEP) {
    const int64_t rr = rb + grp * kMfRows;
    double b[kMfRows];
    double a[kMfTiles][kMfRows];
    if (fullc && rb + STEP <= r1) {
      // whole step: every load issued before the first product
#pragma unroll
      for (int s = 0; s < kMfRows; ++s) b[s] = cp[(rr + s) * DA];
#pragma unroll
      for (int t = 0; t < kMfTiles; ++t) {
        const double2* zp =
            reinterpret_cast<const double2*>(z + (int64_t)(j0 + 16 * t + col) * ldz + rr);
#pragma unroll
        for (int s = 0; s < kMfRows; s += 2) {
          const double2 v = zp[s / 2];
          a[t][s] = v.x;
          a[t][s + 1] = v.y;
        }
      }
    } else {
      // ragged step (rows past the chunk or columns past k read as zero)
#pragma unroll
      for (int s = 0; s < kMfRows; ++s) b[s] = rr + s < r1 ? cp[(rr + s) * DA] : 0.0;
#pragma unroll
      for (int t = 0; t < kMfTiles; ++t) {
        const int jj = j0 + 16 * t + col;
#pragma unroll
        for (int s = 0; s < kMfRows; s += 2) {
          double2 v = double2{0.0, 0.0};
          if (jj < k) v = load_vec<double>(z + (int64_t)jj * ldz, rr + s, r1);
          a[t][s] = v.x;
          a[t][s + 1] = v.y;
        }
      }
    }
#pragma unroll
    for (int s = 0; s < kMfRows; ++s)
#pragma unroll
      for (int t = 0; t < kMfTiles; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t][s], b[s], acc[t], 0, 0, 0);
  }
#pragma unroll
  for (int t = 0; t < kMfTiles; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wid][t][v][lane] = acc[t][v];
  __syncthreads();
  for (int e = threadIdx.x; e < kMfTiles * 4 * kWave; e += kThreads) {
    const int l = e % kWave, v = (e / kWave) % 4, t = e / (4 * kWave);
    const double sum = ((red[0][t][v][l] + red[1][t][v][l]) + red[2][t][v][l]) + red[3][t][v][l];
    const int j = j0 + 16 * t + l / 16 + 4 * v;
    if (j < k) hpart[((int64_t)blockIdx.x * k + j) * NC + (l % 16)] = sum;
  }
}

// out[v] = sum_b part[b * nv + v]  (fixed order); 32 values x 8 part-groups per block
__global__ __launch_bounds__(256) void k_reduce_cols(const int* cond, int nparts, int nv,
                                                     const double* __restrict__ part,
                                                     double* __restrict__ out) {
  if (cond && *cond == 0) return;
  __shared__ double sm[256];
  const int vl = threadIdx.x % 32, g = threadIdx.x / 32;
  const int v = blockIdx.x * 32 + vl;
  double s = 0.0;
  if (v < nv)
    for (int b = g; b < nparts; b += 8) s += part[(size_t)b * nv + v];
  sm[threadIdx.x] = s;
  __syncthreads();
  if (g == 0 && v < nv) {
    double r = 0.0;
    for (int q = 0; q < 8; ++q) r += sm[q * 32 + vl];
    out[v] = r;
  }
}

// C -= Z H for the 16-column FP32 pair (d = 8).  A block handles 64 rows;
// its 4 waves split the k columns and the partial sums are combined in LDS.
// With GRAM the block also writes the partial Gram matrix of the updated rows
// (for the final Cholesky QR).
template <typename VT, int DA, int NA, bool GRAM>
__global__ __launch_bounds__(kThreads) void k_ts_nn(const int* cond, int64_t n,
                                                    const VT* __restrict__ z, int64_t ldz, int k,
                                                    const double* __restrict__ h,
                                                    CPair<VT, DA, NA> cc,
                                                    double* __restrict__ part_c) {
  constexpr int NC = DA * NA;
  if (cond && *cond == 0) return;
  __shared__ double red[4][kWave][NC];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  const int64_t r = (int64_t)blockIdx.x * kWave + lane;
  const int per = (k + 3) / 4;
  const int jb = wid * per, je = min(k, jb + per);
  double acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0.0;
  if (r < n) {
    const VT* zr = z + r;
    // four column loads in flight, the products still in column order
    int j = jb;
    for (; j + 3 < je; j += 4) {
      double zv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) zv[u] = (double)zr[(int64_t)(j + u) * ldz];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = fma(zv[u], h[(int64_t)(j + u) * NC + c], acc[c]);
    }
    for (; j < je; ++j) {
      const double zv = (double)zr[(int64_t)j * ldz];
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] = fma(zv, h[(int64_t)j * NC + c], acc[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) red[wid][lane][c] = acc[c];
  __syncthreads();
  // the block's updated rows, for the Gram partials
  __shared__ double orow[GRAM ? kWave : 1][NC];
  if (wid == 0) {
    double o[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) o[c] = 0.0;
    if (r < n) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const double s = red[0][lane][c] + red[1][lane][c] + red[2][lane][c] + red[3][lane][c];
        o[c] = (double)VT((double)cc.get(r, c) - s);
        cc.set(r, c, VT(o[c]));
      }
    }
    if constexpr (GRAM) {
#pragma unroll
      for (int c = 0; c < NC; ++c) orow[lane][c] = o[c];
    }
  }
  if constexpr (GRAM) {
    // entry (a, b) of the block's partial Gram matrix per thread, summed over
    // the block's rows in order (no per-thread NC x NC accumulator)
    __syncthreads();
    constexpr int NG = NC * NC;
    for (int i = threadIdx.x; i < NG; i += blockDim.x) {
      const int a = i % NC, b = i / NC;
      double g = 0.0;
      for (int l = 0; l < kWave; ++l) g = fma(orow[l][a], orow[l][b], g);
      part_c[(size_t)blockIdx.x * NG + i] = g;
    }
  }
}

// Waves per block of the update kernel: 8, or 4 where the per-wave partial
// sums (NC x rows doubles each) would exceed 64 KB of LDS.
template <typename VT, int NC> constexpr int ts_nn_waves() {
  return 8 * NC * kWave * RowVec<VT>::R * 8 > 65536 ? 4 : 8;
}

// Whether the C -= Z H update of NC columns takes the vectorised kernel
// k_ts_nn_v: up to 8 columns, and the 16-column FP64 pair (its per-wave partial
// sums still fit 64 KB of LDS with 4 waves).
template <typename VT, int NC> constexpr bool ts_nn_vec() { return NC <= 8 || (NC == 16 && sizeof(VT) == 8); }

// C -= Z H, vectorised.  A block owns 64 * RV consecutive rows (RV rows per
// lane, one 16-byte load per basis column); its waves split the k columns,
// unrolled by 4 so every wave keeps several loads in flight, and combine the
// partial sums in LDS.  With GRAM it also writes the block's partial Gram
// matrix of the updated rows.
template <typename VT, int DA, int NA, bool GRAM>
__global__ __launch_bounds__(512) void k_ts_nn_v(const int* cond, int64_t n,
                                                 const VT* __restrict__ z, int64_t ldz, int k,
                                                 const double* __restrict__ h,
                                                 CPair<VT, DA, NA> cc,
                                                 double* __restrict__ part_c) {
  constexpr int NC = DA * NA;
  constexpr int RV = RowVec<VT>::R;
  constexpr int NW = ts_nn_waves<VT, NC>();
  constexpr int TR = kWave * RV;  // rows per block
  static_assert(ts_nn_vec<VT, NC>(), "other widths use k_ts_nn");
  if (cond && *cond == 0) return;
  __shared__ double red[NW][NC][TR];
  // the wave index is uniform: said explicitly, the column indices and the
  // H coefficients of a wave live in scalar registers (scalar loads)
  const int lane = threadIdx.x % kWave;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int64_t rb = (int64_t)blockIdx.x * TR;
  const int64_t r = rb + (int64_t)lane * RV;
  double acc[RV][NC];
#pragma unroll
  for (int i = 0; i < RV; ++i)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[i][c] = 0.0;
  // Columns go from the last to the first in groups of UN dealt round-robin
  // to the waves, so the whole grid sweeps Z downwards together: the
  // projection kernel just read Z upwards, and its most recent columns are the
  // ones still held in the memory-side cache.  UN loads in flight per wave.
  constexpr int UN = 4;
  if (r < n) {
    for (int g = wid;; g += NW) {
      const int jhi = k - UN * g;
      if (jhi <= 0) break;
      if (jhi >= UN) {
        const int j = jhi - UN;
        double zv[UN][RV];
#pragma unroll
        for (int u = 0; u < UN; ++u) load_rows<VT>(z + (int64_t)(j + u) * ldz, r, n, zv[u]);
#pragma unroll
        for (int u = 0; u < UN; ++u)
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const double hv = h[(int64_t)(j + u) * NC + c];
#pragma unroll
            for (int i = 0; i < RV; ++i) acc[i][c] = fma(zv[u][i], hv, acc[i][c]);
          }
      } else {
        for (int j = 0; j < jhi; ++j) {
          double zv[RV];
          load_rows<VT>(z + (int64_t)j * ldz, r, n, zv);
#pragma unroll
          for (int c = 0; c < NC; ++c) {
            const double hv = h[(int64_t)j * NC + c];
#pragma unroll
            for (int i = 0; i < RV; ++i) acc[i][c] = fma(zv[i], hv, acc[i][c]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < RV; ++i)
#pragma unroll
    for (int c = 0; c < NC; ++c) red[wid][c][lane * RV + i] = acc[i][c];
  __syncthreads();
  // thread t < TR finishes row rb + t
  constexpr bool GSMALL = GRAM && NC <= 4;  // Gram in registers; wider C goes through LDS
  constexpr int NG = GSMALL ? NC * NC : 1;
  double g[NG];
#pragma unroll
  for (int i = 0; i < NG; ++i) g[i] = 0.0;
  const int t = threadIdx.x;
  double o[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) o[c] = 0.0;
  if (t < TR && rb + t < n) {
    const int64_t row = rb + t;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double sum = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) sum += red[w][c][t];
      o[c] = (double)VT((double)cc.get(row, c) - sum);
      cc.set(row, c, VT(o[c]));
    }
    if constexpr (GSMALL) {
#pragma unroll
      for (int a = 0; a < NC; ++a)
#pragma unroll
        for (int b = 0; b < NC; ++b) g[a + b * NC] += o[a] * o[b];
    }
  }
  if constexpr (GSMALL) {
    __syncthreads();
    block_sum<NG>(g, &red[0][0][0]);  // reuses the LDS: needs NW * NG doubles
    if (threadIdx.x == 0)
#pragma unroll
      for (int i = 0; i < NG; ++i) part_c[(size_t)blockIdx.x * NG + i] = g[i];
  } else if constexpr (GRAM) {
    // the block's updated rows go to LDS (NC x TR), then thread (a, b) sums
    // entry (a, b) of their Gram matrix over the rows in order
    __syncthreads();
    double* ob = &red[0][0][0];
    if (t < TR)
#pragma unroll
      for (int c = 0; c < NC; ++c) ob[c * TR + t] = o[c];
    __syncthreads();
    if (t < NC * NC) {
      const int a = t % NC, b = t / NC;
      double sg = 0.0;
      for (int q = 0; q < TR; ++q) sg = fma(ob[a * TR + q], ob[b * TR + q], sg);
      part_c[(size_t)blockIdx.x * NC * NC + t] = sg;
    }
  }
}

// Partial reorthogonalisation is one classical Gram-Schmidt pass (Sec. 4.2),
// accepted by the Kahan-Parlett criterion: each projected column of the unit
// pair [Q_ell, Q_ell+1] must keep at least 1/sqrt(2) of its norm, i.e. the
// diagonal of its Gram matrix g must stay >= 1/2.  A flagged step starts from
// a loss of orthogonality just above sqrt(u), so this holds by a wide margin
// unless the W bound failed.
__device__ bool kahan_parlett_ok(int k, const double* g) {
  for (int i = 0; i < k; ++i)
    if (!(g[i + i * k] >= 0.5)) return false;
  return true;
}

// Rows per block of the C -= Z H kernel (and so the number of Gram partials).
template <typename VT, int NC> constexpr int ts_nn_rows() {
  return ts_nn_vec<VT, NC>() ? kWave * RowVec<VT>::R : kWave;
}

// Threads of k_ts_gramfin: 1024 for 16 columns (four groups of threads per
// Gram entry in the partial sums; the factor in parallel), else 256.
template <int NC> constexpr int ts_gramfin_threads() { return NC >= 16 ? 1024 : 256; }

// One block: Gram of C from the partials, Cholesky; writes R^{-1} then R (NC x NC each).
template <int NC>
__global__ __launch_bounds__(ts_gramfin_threads<NC>()) void k_ts_gramfin(
    const int* cond, int nparts, const double* __restrict__ part_c, double* rinv, int* flags) {
  constexpr int NV = NC * NC;
  constexpr int NT = ts_gramfin_threads<NC>();
  if (cond && *cond == 0) return;
  __shared__ double smem[NT];
  __shared__ double res[NV];
  reduce_partials<NV>(part_c, nparts, res, smem);
  if constexpr (NC >= 16) {
    __shared__ double r[NV], ri[NV];
    __shared__ int bad;
    const bool ok = chol_upper_inv_par<NC>(res, r, ri, &bad);
    if (threadIdx.x == 0) {
      if (!ok) atomicOr(flags + 1, 1);
      if (cond && !kahan_parlett_ok(NC, res)) atomicOr(flags + 1, 2);
    }
    for (int i = threadIdx.x; i < NV; i += NT) { rinv[i] = ri[i]; rinv[NV + i] = r[i]; }
  } else if (threadIdx.x == 0) {
    double r[NV], ri[NV];
    if (!chol_upper_inv<NC>(res, r, ri)) atomicOr(flags + 1, 1);
    if (cond && !kahan_parlett_ok(NC, res)) atomicOr(flags + 1, 2);
    for (int i = 0; i < NV; ++i) { rinv[i] = ri[i]; rinv[NV + i] = r[i]; }
  }
}

// C = C R^{-1} (NC columns), written back to the arrays and, if z0 is given,
// to NC consecutive basis columns starting at z0; R^{-1} comes from
// k_ts_gramfin (one block reduces the Gram partials and factors them once).
template <typename VT, int DA, int NA>
__global__ __launch_bounds__(kThreads) void k_ts_scale(const int* cond, int64_t n,
                                                       CPair<VT, DA, NA> cc,
                                                       const double* __restrict__ rinv,
                                                       VT* __restrict__ z0, int64_t ldz) {
  constexpr int NC = DA * NA;
  constexpr int NV = NC * NC;
  if (cond && *cond == 0) return;
  __shared__ double ri[NV];
  if (threadIdx.x < NV) ri[threadIdx.x] = rinv[threadIdx.x];
  __syncthreads();
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = (double)cc.get(r, c);
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b <= a; ++b) s = fma(v[b], ri[b + a * NC], s);
      cc.set(r, a, VT(s));
      if (z0) z0[r + (int64_t)a * ldz] = VT(s);
    }
  }
}

// k_ts_scale with the factor computed in the kernel: every block sums the Gram
// partials of k_ts_nn_v in the same fixed order (so all blocks hold the same
// R) and factors them; block 0 stores R^{-1} and R and raises the breakdown
// flags as k_ts_gramfin does.  One launch fewer per reorthogonalisation step
// where the partials are few enough for every block to read them all.
template <typename VT, int DA, int NA>
__global__ __launch_bounds__(kThreads) void k_ts_scale_fin(const int* cond, int64_t n,
                                                           CPair<VT, DA, NA> cc, int nparts,
                                                           const double* __restrict__ part_c,
                                                           double* __restrict__ rinv, int* flags,
                                                           VT* __restrict__ z0, int64_t ldz) {
  constexpr int NC = DA * NA;
  constexpr int NV = NC * NC;
  if (cond && *cond == 0) return;
  __shared__ double smem[kThreads];
  __shared__ double res[NV];
  __shared__ double ri[NV];
  reduce_partials<NV>(part_c, nparts, res, smem);
  if (threadIdx.x == 0) {
    double r[NV], rv[NV];
    const bool ok = chol_upper_inv<NC>(res, r, rv);
#pragma unroll
    for (int i = 0; i < NV; ++i) ri[i] = rv[i];
    if (blockIdx.x == 0) {
      if (!ok) atomicOr(flags + 1, 1);
      if (cond && !kahan_parlett_ok(NC, res)) atomicOr(flags + 1, 2);
#pragma unroll
      for (int i = 0; i < NV; ++i) { rinv[i] = rv[i]; rinv[NV + i] = r[i]; }
    }
  }
  __syncthreads();
  for (int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * blockDim.x) {
    double v[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) v[c] = (double)cc.get(row, c);
#pragma unroll
    for (int a = 0; a < NC; ++a) {
      double t = 0.0;
#pragma unroll
      for (int b = 0; b <= a; ++b) t = fma(v[b], ri[b + a * NC], t);
      cc.set(row, a, VT(t));
      if (z0) z0[row + (int64_t)a * ldz] = VT(t);
    }
  }
}

// ---------------------------------------------------------------------------
// restart and extraction helpers
// ---------------------------------------------------------------------------
// T (K x K, column-major): diag(Theta) for the kept part, F coupling, then the
// block tridiagonal Xi / Gamma blocks (Eq. "defT").
__global__ void k_assemble_t(int K, int d, int kk, const double* __restrict__ theta,
                             const double* __restrict__ f, const double* __restrict__ xi,
                             const double* __restrict__ gam, double* __restrict__ t) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)K * K) return;
  const int i = (int)(idx % K), j = (int)(idx / K);
  double v = 0.0;
  const int bi = i / d, bj = j / d;  // 0-based block indices; block b holds rows b*d..
  if (i < kk && j < kk) {
    v = (i == j) ? theta[i] : 0.0;
  } else if (i >= kk && i < kk + d && j < kk) {
    v = f[(i - kk) + (int64_t)j * d];
  } else if (j >= kk && j < kk + d && i < kk) {
    v = f[(j - kk) + (int64_t)i * d];
  } else if (i >= kk && j >= kk) {
    const int blk_i = bi + 1, blk_j = bj + 1;  // 1-based block numbers
    const int ii = i % d, jj = j % d;
    if (blk_i == blk_j) v = xi[(int64_t)blk_i * d * d + ii + jj * d];
    else if (blk_i == blk_j + 1) v = gam[(int64_t)blk_j * d * d + ii + jj * d];
    else if (blk_j == blk_i + 1) v = gam[(int64_t)blk_i * d * d + jj + ii * d];
  }
  t[idx] = v;
}

// Restart coupling block (reading R11): F = R Gamma_L V_Z(K-d:K, 0:kn), d x kn
// column-major, with R the triangular factor that re-orthonormalised Q_{L+1}
// (stored after R^{-1} in rinvc) and V_Z the eigenvectors of T (K x K).
__global__ void k_restart_f(int K, int d, int kn, const double* __restrict__ vz,
                            const double* __restrict__ gam_l, const double* __restrict__ rinvc,
                            double* __restrict__ f) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kn) return;
  const double* r = rinvc + d * d;
  for (int i = 0; i < d; ++i) {
    double s = 0.0;
    for (int l = 0; l < d; ++l) {
      double rg = 0.0;  // (R Gamma_L)[i, l]
      for (int q = 0; q < d; ++q) rg += r[i + q * d] * gam_l[q + l * d];
      s += rg * vz[(K - d + l) + (int64_t)j * K];
    }
    f[i + (int64_t)j * d] = s;
  }
}

// Block norms for the W-recurrence of the kept part: ||Theta_k|| (max |theta|)
// and ||F_k||_F for the blocks k = 1..nb of d kept Ritz vectors each.
__global__ void k_kept_norms(int nb, int d, const double* __restrict__ theta,
                             const double* __restrict__ f, double* __restrict__ n_theta,
                             double* __restrict__ n_f) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x + 1;
  if (k > nb) return;
  double mx = 0.0, s2 = 0.0;
  for (int j = (k - 1) * d; j < k * d; ++j) {
    mx = fmax(mx, fabs(theta[j]));
    for (int i = 0; i < d; ++i) s2 += f[i + (int64_t)j * d] * f[i + (int64_t)j * d];
  }
  n_theta[k] = mx;
  n_f[k] = sqrt(s2);
}

// column-major (ld) -> row-interleaved, with type conversion
template <typename SRC, typename DST>
__global__ void k_cm_to_ri(int64_t n, int d, const SRC* __restrict__ s, int64_t ld, DST* __restrict__ o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * d) return;
  o[i] = (DST)s[(i % d) * ld + i / d];
}

template <typename SRC, typename DST>
__global__ void k_convert(int64_t cnt, const SRC* __restrict__ s, DST* __restrict__ o) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) o[i] = (DST)s[i];
}

// copy a column-major panel (rows x cols) with leading dims, converting type
template <typename SRC, typename DST>
__global__ void k_copy_panel(int64_t rows, int cols, const SRC* __restrict__ s, int64_t lds,
                             DST* __restrict__ o, int64_t ldo) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * cols) return;
  const int64_t r = i % rows, c = i / rows;
  o[r + c * ldo] = (DST)s[r + c * lds];
}

// ---------------------------------------------------------------------------
// refinement / backward vector kernels (FP64, row-major n x k blocks)
// ---------------------------------------------------------------------------
// out[c] = sum_r a[r,c] * b[r,c]  (column dots), grid reduced in fixed order
__global__ __launch_bounds__(kThreads) void k_coldots_partial(int64_t rows, int k,
                                                              const double* __restrict__ a,
                                                              const double* __restrict__ b,
                                                              double* __restrict__ part,
                                                              int64_t rows_per_block) {
  // thread layout: threads over columns (k <= blockDim handled by looping), rows chunked
  const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t r1 = min(rows, r0 + rows_per_block);
  for (int c = threadIdx.x; c < k; c += blockDim.x) {
    double s = 0.0;
    for (int64_t r = r0; r < r1; ++r) s = fma(a[r * k + c], b[r * k + c], s);
    part[(int64_t)blockIdx.x * k + c] = s;
  }
}

// out[v] = sum_b part[b * nv + v]: vb values per block (1, 2, 4 or 8, fewer
// for small nv so that all 256 threads work), 256 / vb partial groups each
// with four independent sums (four loads in flight), then a fixed-order tree
// over the groups in LDS
__global__ __launch_bounds__(256) void k_reduce_parts(int nparts, int nv, int vb,
                                                      const double* __restrict__ part,
                                                      double* __restrict__ out) {
  __shared__ double sm[256];
  const int groups = 256 / vb;
  const int vl = (int)threadIdx.x % vb, g = (int)threadIdx.x / vb;
  const int v = (int)blockIdx.x * vb + vl;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (v < nv) {
    int b = g;
    for (; b + 3 * groups < nparts; b += 4 * groups) {
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += part[(size_t)(b + u * groups) * nv + v];
    }
    for (int u = 0; b < nparts; b += groups, ++u) acc[u & 3] += part[(size_t)b * nv + v];
  }
  sm[threadIdx.x] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  for (int h = groups / 2; h > 0; h >>= 1) {
    if (g < h) sm[threadIdx.x] += sm[threadIdx.x + h * vb];
    __syncthreads();
  }
  if (g == 0 && v < nv) out[v] = sm[vl];
}

// Elementwise updates of row-major blocks (rows x k).  A block's 256 threads
// cover kc = min(k, 256) consecutive columns (tile blockIdx.y) of 256 / kc
// rows at a time, kUpdRows such row steps per block: each thread's column and
// its coefficient are fixed (no 64-bit division per element), consecutive
// threads touch consecutive addresses, and narrow blocks (few columns) still
// use every thread.
constexpr int kUpdRows = 16;

struct UpdMap {
  int kc, rpt;  // columns per tile, rows per row step
  __host__ __device__ UpdMap(int k) : kc(k < 256 ? k : 256), rpt(256 / (k < 256 ? k : 256)) {}
};

// CGLS update: alpha_c = gamma_c / qq_c (0 for inactive columns)
//   x += alpha p (n rows) ; s -= alpha q (m rows)
__global__ __launch_bounds__(256) void k_cgls_xs(int64_t n, int64_t m, int k,
                                                 const double* __restrict__ gamma,
                                                 const double* __restrict__ qq,
                                                 const int* __restrict__ active, double* __restrict__ x,
                                                 const double* __restrict__ p, double* __restrict__ s,
                                                 const double* __restrict__ q) {
  const UpdMap mp(k);
  const int t = (int)threadIdx.x;
  if (t >= mp.rpt * mp.kc) return;
  const int c = (int)blockIdx.y * mp.kc + t % mp.kc;
  if (c >= k) return;
  const double al = (active[c] && qq[c] > 0.0) ? gamma[c] / qq[c] : 0.0;
  if (al == 0.0) return;
  const int64_t r0 = (int64_t)blockIdx.x * mp.rpt * kUpdRows + t / mp.kc;
#pragma unroll 4
  for (int u = 0; u < kUpdRows; ++u) {
    const int64_t row = r0 + (int64_t)u * mp.rpt;
    const int64_t i = row * k + c;
    if (row < n) x[i] = fma(al, p[i], x[i]);
    if (row < m) s[i] = fma(-al, q[i], s[i]);
  }
}

// CGLS direction: beta_c = gnew_c / gamma_c ; p = r + beta p (active columns only)
__global__ __launch_bounds__(256) void k_cgls_p(int64_t n, int k, const double* __restrict__ gnew,
                                                const double* __restrict__ gamma,
                                                const int* __restrict__ active,
                                                const double* __restrict__ r, double* __restrict__ p) {
  const UpdMap mp(k);
  const int t = (int)threadIdx.x;
  if (t >= mp.rpt * mp.kc) return;
  const int c = (int)blockIdx.y * mp.kc + t % mp.kc;
  if (c >= k || !active[c]) return;
  const double be = gamma[c] > 0.0 ? gnew[c] / gamma[c] : 0.0;
  const int64_t r0 = (int64_t)blockIdx.x * mp.rpt * kUpdRows + t / mp.kc;
#pragma unroll 4
  for (int u = 0; u < kUpdRows; ++u) {
    const int64_t row = r0 + (int64_t)u * mp.rpt;
    if (row >= n) break;
    const int64_t i = row * k + c;
    p[i] = fma(be, p[i], r[i]);
  }
}

// CG on A^T A: alpha = rr / pq ; w += alpha p ; r -= alpha q
__global__ __launch_bounds__(256) void k_cg_wr(int64_t n, int k, const double* __restrict__ rr,
                                               const double* __restrict__ pq,
                                               const int* __restrict__ active, double* __restrict__ w,
                                               const double* __restrict__ p, double* __restrict__ r,
                                               const double* __restrict__ q) {
  const UpdMap mp(k);
  const int t = (int)threadIdx.x;
  if (t >= mp.rpt * mp.kc) return;
  const int c = (int)blockIdx.y * mp.kc + t % mp.kc;
  if (c >= k) return;
  const double al = (active[c] && pq[c] > 0.0) ? rr[c] / pq[c] : 0.0;
  if (al == 0.0) return;
  const int64_t r0 = (int64_t)blockIdx.x * mp.rpt * kUpdRows + t / mp.kc;
#pragma unroll 4
  for (int u = 0; u < kUpdRows; ++u) {
    const int64_t row = r0 + (int64_t)u * mp.rpt;
    if (row >= n) break;
    const int64_t i = row * k + c;
    w[i] = fma(al, p[i], w[i]);
    r[i] = fma(-al, q[i], r[i]);
  }
}

// x -= y (elementwise)
__global__ void k_sub(int64_t cnt, double* __restrict__ x, const double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) x[i] -= y[i];
}

// x(i, :) /= s[i] or *= s[i] for a row-major rows x k block
__global__ void k_scale_rows(int64_t rows, int k, const double* __restrict__ s, bool divide,
                             double* __restrict__ x) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows * k) return;
  const double f = s[t / k];
  x[t] = divide ? x[t] / f : x[t] * f;
}

// ===========================================================================
// host launchers
// ===========================================================================
template <typename VT>
int sub_gram(nsp_ctx* c, int d, int64_t n, VT* p, const VT* x, const double* part_xi, int nparts_xi,
             double* xi_out, double* nrm_xi, double* part_g) {
  if (d == 8) {
    const unsigned g8 = g8_grid(n);
    if (part_xi && x)
      k_sub_gram8<VT, true, true><<<g8, kThreads, 0, c->stream>>>(n, p, x, part_xi, nparts_xi, xi_out,
                                                                  nrm_xi, part_g);
    else if (part_xi)
      k_sub_gram8<VT, true, false><<<g8, kThreads, 0, c->stream>>>(n, p, x, part_xi, nparts_xi, xi_out,
                                                                   nrm_xi, part_g);
    else
      k_sub_gram8<VT, false, false><<<g8, kThreads, 0, c->stream>>>(n, p, x, part_xi, nparts_xi,
                                                                    xi_out, nrm_xi, part_g);
    NSP_HIP(hipGetLastError());
    return (int)g8;
  }
  const unsigned grid = cap_grid(n, kThreads, kRedBlocks);
#define NSP_SG(D)                                                                              \
  case D:                                                                                      \
    if (part_xi && x)                                                                          \
      k_sub_gram<VT, D, true, true><<<grid, kThreads, 0, c->stream>>>(                         \
          n, p, x, part_xi, nparts_xi, xi_out, nrm_xi, part_g);                                \
    else if (part_xi)                                                                          \
      k_sub_gram<VT, D, true, false><<<grid, kThreads, 0, c->stream>>>(                        \
          n, p, x, part_xi, nparts_xi, xi_out, nrm_xi, part_g);                                \
    else                                                                                       \
      k_sub_gram<VT, D, false, false><<<grid, kThreads, 0, c->stream>>>(                       \
          n, p, x, part_xi, nparts_xi, xi_out, nrm_xi, part_g);                                \
    break;
  switch (d) { NSP_SG(1) NSP_SG(2) NSP_SG(4) default: throw Error(NSP_ERR_ARG, "d"); }
#undef NSP_SG
  NSP_HIP(hipGetLastError());
  return (int)grid;
}
template int sub_gram<double>(nsp_ctx*, int, int64_t, double*, const double*, const double*, int,
                              double*, double*, double*);
template int sub_gram<float>(nsp_ctx*, int, int64_t, float*, const float*, const double*, int,
                             double*, double*, double*);

template <typename VT>
int scale_block(nsp_ctx* c, int d, int64_t n, const VT* p, const double* part_g, int nparts,
                VT* xn, VT* zcol, int64_t ldz, double* gam_out, double* nrm_gam, double* nrm_ginv,
                double* part_g2, const WArgs* wa) {
  int* flags = c->flags.as<int>();
  if (d == 8 && part_g2 && !wa) {
    const unsigned g8 = g8_grid(n);
    k_scale8<VT><<<g8, kThreads, 0, c->stream>>>(n, p, part_g, nparts, xn, zcol, ldz, gam_out, nrm_gam,
                                                 nrm_ginv, part_g2, flags);
    NSP_HIP(hipGetLastError());
    return (int)g8;
  }
  const unsigned grid = cap_grid(n, kThreads, kRedBlocks);
  WArgs w{};
  if (wa) w = *wa;
#define NSP_SC(D)                                                                              \
  case D:                                                                                      \
    if (part_g2)                                                                               \
      k_scale<VT, D, true, false><<<grid, kThreads, 0, c->stream>>>(n, p, part_g, nparts, xn,  \
          zcol, ldz, gam_out, nrm_gam, nrm_ginv, part_g2, flags, w);                           \
    else if (wa) /* one extra block: block 0 runs the W-recurrence */                        \
      k_scale<VT, D, false, true><<<grid + 1, kThreads, 0, c->stream>>>(n, p, part_g, nparts, xn, \
          zcol, ldz, gam_out, nrm_gam, nrm_ginv, part_g2, flags, w);                           \
    else                                                                                       \
      k_scale<VT, D, false, false><<<grid, kThreads, 0, c->stream>>>(n, p, part_g, nparts, xn, \
          zcol, ldz, gam_out, nrm_gam, nrm_ginv, part_g2, flags, w);                           \
    break;
  switch (d) { NSP_SC(1) NSP_SC(2) NSP_SC(4) NSP_SC(8) default: throw Error(NSP_ERR_ARG, "d"); }
#undef NSP_SC
  NSP_HIP(hipGetLastError());
  return (int)grid;
}
template int scale_block<double>(nsp_ctx*, int, int64_t, const double*, const double*, int, double*,
                                 double*, int64_t, double*, double*, double*, double*, const WArgs*);
template int scale_block<float>(nsp_ctx*, int, int64_t, const float*, const double*, int, float*,
                                float*, int64_t, double*, double*, double*, double*, const WArgs*);

template <typename VT>
void scale_block2(nsp_ctx* c, int d, int64_t n, const double* part_g2, int nparts, VT* xn, VT* zcol,
                  int64_t ldz, double* gam, double* nrm_gam, double* nrm_ginv, const WArgs* wa) {
  const unsigned grid = cap_grid(n, kThreads, kRedBlocks);
  int* flags = c->flags.as<int>();
  WArgs w{};
  if (wa) w = *wa;
#define NSP_SC2(D)                                                                             \
  case D:                                                                                      \
    if (wa) /* one extra block: block 0 runs the W-recurrence */                               \
      k_scale2<VT, D, true><<<grid + 1, kThreads, 0, c->stream>>>(n, part_g2, nparts, xn, zcol, \
          ldz, gam, nrm_gam, nrm_ginv, flags, w);                                              \
    else                                                                                       \
      k_scale2<VT, D, false><<<grid, kThreads, 0, c->stream>>>(n, part_g2, nparts, xn, zcol,   \
          ldz, gam, nrm_gam, nrm_ginv, flags, w);                                              \
    break;
  switch (d) { NSP_SC2(1) NSP_SC2(2) NSP_SC2(4) NSP_SC2(8) default: throw Error(NSP_ERR_ARG, "d"); }
#undef NSP_SC2
  NSP_HIP(hipGetLastError());
}
template void scale_block2<double>(nsp_ctx*, int, int64_t, const double*, int, double*, double*,
                                   int64_t, double*, double*, double*, const WArgs*);
template void scale_block2<float>(nsp_ctx*, int, int64_t, const double*, int, float*, float*,
                                  int64_t, double*, double*, double*, const WArgs*);

void w_reset(nsp_ctx* c, int col0, int ncols, double u_d, double* w, int ldw) {
  k_w_reset<<<1, 256, 0, c->stream>>>(col0, ncols, u_d, w, ldw);
  NSP_HIP(hipGetLastError());
}

// Rows per chunk of the TN kernel: aim for ~1024 blocks in total with chunks of
// at least 1024 rows (so each lane accumulates >= 16 rows before the wave sum).
// Row chunk of the H = Z^T C kernel: about 2048 blocks over (chunks x column
// groups), at least 1024 rows, a multiple of 256 rows (aligned vector loads).
// Whether the projection of NC columns runs on the matrix cores (k_ts_tn_mfma).
constexpr bool ts_tn_mfma(int nc, int esize) { return nc == 16 && esize == 8; }

int64_t ts_chunk_rows(int64_t n, int k, int nc, int esize) {
  // basis columns per block: TsShape<NC, esize>::JB, or kMfCols on the matrix cores
  const int jb = ts_tn_mfma(nc, esize) ? kMfCols : kTsWaves * ts_jw(nc);
  const int64_t col_groups = std::max<int64_t>(1, (k + jb - 1) / jb);
  const int64_t chunks = std::max<int64_t>(1, 2048 / col_groups);
  int64_t rows = (n + chunks - 1) / chunks;
  rows = std::max<int64_t>(rows, 1024);
  return (rows + 255) / 256 * 256;
}

// Whether the factor of the reorthogonalised block's Gram matrix is computed
// inside k_ts_scale_fin (every block reads all partials of k_ts_nn_v: at most
// 4096 doubles, up to 4 columns) instead of by the one-block k_ts_gramfin.
template <typename VT, int NC>
static bool ts_fin_fused(int64_t n) {
  constexpr int TR = ts_nn_rows<VT, NC>();
  return NC <= 4 && ((n + TR - 1) / TR) * NC * NC <= 4096;
}

template <typename VT, int DA, int NA>
static void ts_proj_t(nsp_ctx* c, const int* cond, int64_t n, const VT* z, int64_t ldz, int k,
                      VT* a0, VT* a1, double* h, double* hpart, bool gram, double* part_c,
                      double* rinv, hipEvent_t ev_tn, hipEvent_t ev_red) {
  constexpr int NC = DA * NA;
  CPair<VT, DA, NA> cc{a0, a1};
  constexpr int TR = ts_nn_rows<VT, NC>();
  const unsigned nnblocks = (unsigned)((n + TR - 1) / TR);
  if (k > 0) {
    const int64_t chunk = ts_chunk_rows(n, k, NC, (int)sizeof(VT));
    const unsigned nchunks = (unsigned)((n + chunk - 1) / chunk);
    if constexpr (ts_tn_mfma(NC, sizeof(VT))) {
      const unsigned gy = (unsigned)((k + kMfCols - 1) / kMfCols);
      k_ts_tn_mfma<DA, NA><<<dim3(nchunks, gy), kThreads, 0, c->stream>>>(cond, n, chunk, z, ldz, k,
                                                                          cc, hpart);
    } else {
      const unsigned gy = (unsigned)((k + TsShape<NC, sizeof(VT)>::JB - 1) / TsShape<NC, sizeof(VT)>::JB);
      k_ts_tn<VT, DA, NA><<<dim3(nchunks, gy), TsShape<NC, sizeof(VT)>::NWT * kWave, 0, c->stream>>>(
          cond, n, chunk, z, ldz, k, cc, hpart);
    }
    if (ev_tn) NSP_HIP(hipEventRecord(ev_tn, c->stream));
    k_reduce_cols<<<nblk((int64_t)k * NC, 32), 256, 0, c->stream>>>(cond, (int)nchunks, k * NC,
                                                                    hpart, h);
  } else if (ev_tn) {
    NSP_HIP(hipEventRecord(ev_tn, c->stream));
  }
  if (ev_red) NSP_HIP(hipEventRecord(ev_red, c->stream));
  if constexpr (ts_nn_vec<VT, NC>()) {
    constexpr int nt = ts_nn_waves<VT, NC>() * kWave;
    if (gram) {
      k_ts_nn_v<VT, DA, NA, true><<<nnblocks, nt, 0, c->stream>>>(cond, n, z, ldz, k, h, cc, part_c);
      if (!ts_fin_fused<VT, NC>(n))
        k_ts_gramfin<NC><<<1, ts_gramfin_threads<NC>(), 0, c->stream>>>(cond, (int)nnblocks, part_c, rinv,
                                                                   c->flags.as<int>());
    } else if (k > 0)
      k_ts_nn_v<VT, DA, NA, false><<<nnblocks, nt, 0, c->stream>>>(cond, n, z, ldz, k, h, cc,
                                                                   nullptr);
  } else {
    if (gram) {
      k_ts_nn<VT, DA, NA, true><<<nnblocks, kThreads, 0, c->stream>>>(cond, n, z, ldz, k, h, cc, part_c);
      k_ts_gramfin<NC><<<1, ts_gramfin_threads<NC>(), 0, c->stream>>>(cond, (int)nnblocks, part_c, rinv,
                                                                 c->flags.as<int>());
    } else if (k > 0) {
      k_ts_nn<VT, DA, NA, false><<<nnblocks, kThreads, 0, c->stream>>>(cond, n, z, ldz, k, h, cc,
                                                                       nullptr);
    }
  }
  NSP_HIP(hipGetLastError());
}

int64_t ts_part_c_len(int64_t n, int nc) { return ((n + kWave - 1) / kWave) * nc * nc; }

// The projection and the update of the tall-skinny pair on their own, for a
// DA-column row-interleaved block C and two different bases (the deflated CG's
// directions are projected with one matrix and corrected with another):
// h (k x DA, basis-column major) = Z^T C, and C -= Z h.
int64_t ts_tn_parts_len(int64_t n, int k, int d) {
  const int64_t chunk = ts_chunk_rows(n, k, d, 8);
  return ((n + chunk - 1) / chunk) * (int64_t)k * d;
}

template <int DA>
static void ts_tn_only_t(nsp_ctx* c, int64_t n, const double* z, int64_t ldz, int k, const double* a0,
                         double* h, double* hpart) {
  CPair<double, DA, 1> cc{const_cast<double*>(a0), nullptr};
  const int64_t chunk = ts_chunk_rows(n, k, DA, 8);
  const unsigned nchunks = (unsigned)((n + chunk - 1) / chunk);
  const unsigned gy = (unsigned)((k + TsShape<DA, 8>::JB - 1) / TsShape<DA, 8>::JB);
  k_ts_tn<double, DA, 1><<<dim3(nchunks, gy), TsShape<DA, 8>::NWT * kWave, 0, c->stream>>>(
      nullptr, n, chunk, z, ldz, k, cc, hpart);
  k_reduce_cols<<<nblk((int64_t)k * DA, 32), 256, 0, c->stream>>>(nullptr, (int)nchunks, k * DA, hpart, h);
  NSP_HIP(hipGetLastError());
}

template <int DA>
static void ts_nn_only_t(nsp_ctx* c, int64_t n, const double* z, int64_t ldz, int k, const double* h,
                         double* a0) {
  CPair<double, DA, 1> cc{a0, nullptr};
  constexpr int TR = ts_nn_rows<double, DA>();
  constexpr int nt = ts_nn_waves<double, DA>() * kWave;
  k_ts_nn_v<double, DA, 1, false><<<(unsigned)((n + TR - 1) / TR), nt, 0, c->stream>>>(
      nullptr, n, z, ldz, k, h, cc, nullptr);
  NSP_HIP(hipGetLastError());
}

void ts_tn_only(nsp_ctx* c, int d, int64_t n, const double* z, int64_t ldz, int k, const double* a0,
                double* h, double* hpart) {
  switch (d) {
    case 1: ts_tn_only_t<1>(c, n, z, ldz, k, a0, h, hpart); break;
    case 2: ts_tn_only_t<2>(c, n, z, ldz, k, a0, h, hpart); break;
    case 4: ts_tn_only_t<4>(c, n, z, ldz, k, a0, h, hpart); break;
    case 8: ts_tn_only_t<8>(c, n, z, ldz, k, a0, h, hpart); break;
    default: throw Error(NSP_ERR_ARG, "ts_tn_only: d must be 1, 2, 4 or 8");
  }
}

void ts_nn_only(nsp_ctx* c, int d, int64_t n, const double* z, int64_t ldz, int k, const double* h,
                double* a0) {
  switch (d) {
    case 1: ts_nn_only_t<1>(c, n, z, ldz, k, h, a0); break;
    case 2: ts_nn_only_t<2>(c, n, z, ldz, k, h, a0); break;
    case 4: ts_nn_only_t<4>(c, n, z, ldz, k, h, a0); break;
    case 8: ts_nn_only_t<8>(c, n, z, ldz, k, h, a0); break;
    default: throw Error(NSP_ERR_ARG, "ts_nn_only: d must be 1, 2, 4 or 8");
  }
}

template <typename VT, int DA, int NA>
static void ts_scale_t(nsp_ctx* c, const int* cond, int64_t n, VT* a0, VT* a1, const double* part_c,
                       double* rinv, VT* z0, int64_t ldz) {
  constexpr int NC = DA * NA;
  CPair<VT, DA, NA> cc{a0, a1};
  const unsigned grid = cap_grid(n, kThreads, 2048);
  if constexpr (NC <= 4) {
    if (ts_fin_fused<VT, NC>(n)) {
      constexpr int TR = ts_nn_rows<VT, NC>();
      k_ts_scale_fin<VT, DA, NA><<<grid, kThreads, 0, c->stream>>>(
          cond, n, cc, (int)((n + TR - 1) / TR), part_c, rinv, c->flags.as<int>(), z0, ldz);
      NSP_HIP(hipGetLastError());
      return;
    }
  }
  // the Gram partials were reduced and factored by k_ts_gramfin
  k_ts_scale<VT, DA, NA><<<grid, kThreads, 0, c->stream>>>(cond, n, cc, rinv, z0, ldz);
  NSP_HIP(hipGetLastError());
}

// One CGS pass of C = [a0 (| a1)] against the first k basis columns; with gram
// also the Cholesky factor of the updated C's Gram matrix (R^{-1}, then R, in rinv).
template <typename VT>
void ts_project(nsp_ctx* c, const int* cond, int d, int na, int64_t n, const VT* z, int64_t ldz,
                int k, VT* a0, VT* a1, double* h, double* hpart, bool gram, double* part_c,
                double* rinv, hipEvent_t ev_tn, hipEvent_t ev_red) {
  k = std::max(k, 0);
#define NSP_TP(D)                                                                              \
  case D:                                                                                      \
    if (na == 1) ts_proj_t<VT, D, 1>(c, cond, n, z, ldz, k, a0, a1, h, hpart, gram, part_c, rinv, ev_tn, ev_red); \
    else ts_proj_t<VT, D, 2>(c, cond, n, z, ldz, k, a0, a1, h, hpart, gram, part_c, rinv, ev_tn, ev_red);          \
    break;
  switch (d) { NSP_TP(1) NSP_TP(2) NSP_TP(4) NSP_TP(8) default: throw Error(NSP_ERR_ARG, "d"); }
#undef NSP_TP
}
template void ts_project<double>(nsp_ctx*, const int*, int, int, int64_t, const double*, int64_t,
                                 int, double*, double*, double*, double*, bool, double*, double*,
                                 hipEvent_t, hipEvent_t);
template void ts_project<float>(nsp_ctx*, const int*, int, int, int64_t, const float*, int64_t, int,
                                float*, float*, double*, double*, bool, double*, double*, hipEvent_t,
                                hipEvent_t);

template <typename VT>
void ts_scale(nsp_ctx* c, const int* cond, int d, int na, int64_t n, VT* a0, VT* a1,
              const double* part_c, double* rinv, VT* z0, int64_t ldz) {
#define NSP_TS(D)                                                                              \
  case D:                                                                                      \
    if (na == 1) ts_scale_t<VT, D, 1>(c, cond, n, a0, a1, part_c, rinv, z0, ldz);              \
    else ts_scale_t<VT, D, 2>(c, cond, n, a0, a1, part_c, rinv, z0, ldz);                      \
    break;
  switch (d) { NSP_TS(1) NSP_TS(2) NSP_TS(4) NSP_TS(8) default: throw Error(NSP_ERR_ARG, "d"); }
#undef NSP_TS
}
template void ts_scale<double>(nsp_ctx*, const int*, int, int, int64_t, double*, double*,
                               const double*, double*, double*, int64_t);
template void ts_scale<float>(nsp_ctx*, const int*, int, int, int64_t, float*, float*,
                              const double*, double*, float*, int64_t);

void restart_coupling(nsp_ctx* c, int K, int d, int kn, const double* vz, const double* gam_l,
                      const double* rinvc, const double* evals, double* f, double* theta_kept,
                      double* n_theta, double* n_f) {
  k_restart_f<<<nblk(kn, 256), 256, 0, c->stream>>>(K, d, kn, vz, gam_l, rinvc, f);
  NSP_HIP(hipMemcpyAsync(theta_kept, evals, sizeof(double) * kn, hipMemcpyDeviceToDevice, c->stream));
  k_kept_norms<<<nblk(kn / d, 256), 256, 0, c->stream>>>(kn / d, d, evals, f, n_theta, n_f);
  NSP_HIP(hipGetLastError());
}

void assemble_t(nsp_ctx* c, int K, int d, int kk, const double* theta, const double* f,
                const double* xi, const double* gam, double* t) {
  k_assemble_t<<<nblk((int64_t)K * K, 256), 256, 0, c->stream>>>(K, d, kk, theta, f, xi, gam, t);
  NSP_HIP(hipGetLastError());
}

template <typename SRC, typename DST>
void cm_to_ri(nsp_ctx* c, int64_t n, int d, const SRC* s, int64_t ld, DST* o) {
  k_cm_to_ri<SRC, DST><<<nblk(n * d, 256), 256, 0, c->stream>>>(n, d, s, ld, o);
  NSP_HIP(hipGetLastError());
}
template void cm_to_ri<double, double>(nsp_ctx*, int64_t, int, const double*, int64_t, double*);
template void cm_to_ri<double, float>(nsp_ctx*, int64_t, int, const double*, int64_t, float*);
template void cm_to_ri<float, float>(nsp_ctx*, int64_t, int, const float*, int64_t, float*);

template <typename SRC, typename DST>
void convert(nsp_ctx* c, int64_t cnt, const SRC* s, DST* o) {
  if (cnt <= 0) return;
  k_convert<SRC, DST><<<nblk(cnt, 256), 256, 0, c->stream>>>(cnt, s, o);
  NSP_HIP(hipGetLastError());
}
template void convert<double, float>(nsp_ctx*, int64_t, const double*, float*);
template void convert<float, double>(nsp_ctx*, int64_t, const float*, double*);

template <typename SRC, typename DST>
void copy_panel(nsp_ctx* c, int64_t rows, int cols, const SRC* s, int64_t lds, DST* o, int64_t ldo) {
  if (rows * cols <= 0) return;
  k_copy_panel<SRC, DST><<<nblk(rows * cols, 256), 256, 0, c->stream>>>(rows, cols, s, lds, o, ldo);
  NSP_HIP(hipGetLastError());
}
template void copy_panel<double, double>(nsp_ctx*, int64_t, int, const double*, int64_t, double*, int64_t);
template void copy_panel<float, float>(nsp_ctx*, int64_t, int, const float*, int64_t, float*, int64_t);
template void copy_panel<float, double>(nsp_ctx*, int64_t, int, const float*, int64_t, double*, int64_t);

// column dots of two row-major (rows x k) blocks -> out[k] (fixed-order reduction)
void coldots(nsp_ctx* c, int64_t rows, int k, const double* a, const double* b, double* out,
             double* part) {
  const int64_t rpb = std::max<int64_t>(64, (rows + 1023) / 1024);
  const unsigned nb = (unsigned)((rows + rpb - 1) / rpb);
  const int thr = k >= 256 ? 256 : std::max(64, (k + 63) / 64 * 64);
  k_coldots_partial<<<nb, thr, 0, c->stream>>>(rows, k, a, b, part, rpb);
  reduce_parts(c, (int)nb, k, part, out);
}

void reduce_parts(nsp_ctx* c, int nparts, int nv, const double* part, double* out) {
  if (nv <= 0) return;
  const int vb = nv >= 8 ? 8 : nv >= 4 ? 4 : nv >= 2 ? 2 : 1;
  k_reduce_parts<<<nblk(nv, vb), 256, 0, c->stream>>>(nparts, nv, vb, part, out);
  NSP_HIP(hipGetLastError());
}

int64_t coldots_parts(int64_t rows) {
  const int64_t rpb = std::max<int64_t>(64, (rows + 1023) / 1024);
  return std::max<int64_t>((rows + rpb - 1) / rpb, kWideBlocks);
}

void cgls_xs(nsp_ctx* c, int64_t n, int64_t m, int k, const double* gamma, const double* qq,
             const int* active, double* x, const double* p, double* s, const double* q) {
  if (k <= 0) return;
  const UpdMap mp(k);
  const int64_t rows_per_block = (int64_t)mp.rpt * kUpdRows;
  const dim3 grid((unsigned)((std::max(n, m) + rows_per_block - 1) / rows_per_block),
                  (unsigned)((k + mp.kc - 1) / mp.kc));
  k_cgls_xs<<<grid, 256, 0, c->stream>>>(n, m, k, gamma, qq, active, x, p, s, q);
  NSP_HIP(hipGetLastError());
}

void cgls_p(nsp_ctx* c, int64_t n, int k, const double* gnew, const double* gamma, const int* active,
            const double* r, double* p) {
  if (k <= 0 || n <= 0) return;
  const UpdMap mp(k);
  const int64_t rows_per_block = (int64_t)mp.rpt * kUpdRows;
  const dim3 grid((unsigned)((n + rows_per_block - 1) / rows_per_block), (unsigned)((k + mp.kc - 1) / mp.kc));
  k_cgls_p<<<grid, 256, 0, c->stream>>>(n, k, gnew, gamma, active, r, p);
  NSP_HIP(hipGetLastError());
}

void cg_wr(nsp_ctx* c, int64_t n, int k, const double* rr, const double* pq, const int* active,
           double* w, const double* p, double* r, const double* q) {
  if (k <= 0 || n <= 0) return;
  const UpdMap mp(k);
  const int64_t rows_per_block = (int64_t)mp.rpt * kUpdRows;
  const dim3 grid((unsigned)((n + rows_per_block - 1) / rows_per_block), (unsigned)((k + mp.kc - 1) / mp.kc));
  k_cg_wr<<<grid, 256, 0, c->stream>>>(n, k, rr, pq, active, w, p, r, q);
  NSP_HIP(hipGetLastError());
}

void sub_inplace(nsp_ctx* c, int64_t cnt, double* x, const double* y) {
  if (cnt <= 0) return;
  k_sub<<<nblk(cnt, 256), 256, 0, c->stream>>>(cnt, x, y);
  NSP_HIP(hipGetLastError());
}

void scale_rows(nsp_ctx* c, int64_t rows, int k, const double* s, bool divide, double* x) {
  if (rows * k <= 0) return;
  k_scale_rows<<<nblk(rows * k, 256), 256, 0, c->stream>>>(rows, k, s, divide, x);
  NSP_HIP(hipGetLastError());
}

}  // namespace nsp
