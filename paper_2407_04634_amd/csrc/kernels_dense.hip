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
__device__ bool chol_upper_inv(int k, const double* g, double* r, double* ri) {
  double gmax = 0.0;
  for (int i = 0; i < k; ++i) gmax = fmax(gmax, g[i + i * k]);
  bool ok = isfinite(gmax) && gmax > 0.0;
  for (int i = 0; i < k * k; ++i) { r[i] = 0.0; ri[i] = 0.0; }
  for (int j = 0; j < k && ok; ++j) {
    for (int i = 0; i <= j; ++i) {
      double s = g[i + j * k];
      for (int l = 0; l < i; ++l) s -= r[l + i * k] * r[l + j * k];
      if (i == j) {
        if (!(s > 1e-24 * gmax) || !isfinite(s)) { ok = false; break; }
        r[j + j * k] = sqrt(s);
      } else {
        r[i + j * k] = s / r[i + i * k];
      }
    }
  }
  if (!ok) {
    for (int i = 0; i < k * k; ++i) { r[i] = 0.0; ri[i] = 0.0; }
    for (int i = 0; i < k; ++i) { r[i + i * k] = 1.0; ri[i + i * k] = 1.0; }
    return false;
  }
  // inverse of the upper triangular R, column by column
  for (int j = 0; j < k; ++j) {
    ri[j + j * k] = 1.0 / r[j + j * k];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int l = i + 1; l <= j; ++l) s += r[i + l * k] * ri[l + j * k];
      ri[i + j * k] = -s / r[i + i * k];
    }
  }
  return true;
}

__device__ double fro(int k, const double* a) {
  double s = 0.0;
  for (int i = 0; i < k * k; ++i) s += a[i] * a[i];
  return sqrt(s);
}

// ---------------------------------------------------------------------------
// Lanczos step, QR part.
// k_sub_gram:  P -= X Xi (if SUB) ; G = P^T P reduced ; last block: Cholesky
//              G = R^T R, stores R (gam_out), R^{-1} (rinv), ||R||_F, ||R^-1||_F.
// ---------------------------------------------------------------------------
template <typename VT, int D, bool SUB>
__global__ __launch_bounds__(kThreads) void k_sub_gram(int64_t n, VT* __restrict__ p,
                                                       const VT* __restrict__ x,
                                                       const double* __restrict__ xi,
                                                       double* partials, unsigned* counter,
                                                       double* gam_out, double* rinv,
                                                       double* nrm_gam, double* nrm_ginv,
                                                       int* flags) {
  constexpr int NV = D * D;
  __shared__ double smem[kThreads > NV * (kThreads / kWave) ? kThreads : NV * (kThreads / kWave)];
  __shared__ double xs[NV];
  if (SUB) {
    if (threadIdx.x < NV) xs[threadIdx.x] = xi[threadIdx.x];
    __syncthreads();
  }
  double g[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) g[i] = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    VT v[D];
#pragma unroll
    for (int j = 0; j < D; ++j) v[j] = p[r * D + j];
    if (SUB) {
      VT xr[D];
#pragma unroll
      for (int j = 0; j < D; ++j) xr[j] = x[r * D + j];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        VT s = v[a];
#pragma unroll
        for (int b = 0; b < D; ++b) s = fma(-xr[b], VT(xs[b + a * D]), s);
        v[a] = s;
      }
#pragma unroll
      for (int j = 0; j < D; ++j) p[r * D + j] = v[j];
    }
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int b = 0; b < D; ++b) g[a + b * D] += (double)v[a] * (double)v[b];
  }
  block_sum<NV>(g, smem);
  __shared__ double res[NV];
  if (grid_sum_last<NV>(g, partials, counter, res, smem)) {
    if (threadIdx.x == 0) {
      double r[NV], ri[NV];
      const bool ok = chol_upper_inv(D, res, r, ri);
      if (!ok) atomicOr(flags + 1, 1);
      for (int i = 0; i < NV; ++i) { gam_out[i] = r[i]; rinv[i] = ri[i]; }
      if (nrm_gam) *nrm_gam = fro(D, r);
      if (nrm_ginv) *nrm_ginv = fro(D, ri);
    }
  }
}

// k_scale: Xn = P R^{-1}; written to the ring slot ``xn`` and, when zcol is not
// null, to D columns of the column-major basis.  With GRAM, also reduces the
// Gram matrix of Xn and (last block) refines: R2 from Cholesky, stores
// R2^{-1} in rinv2 and Gamma <- R2 Gamma.
template <typename VT, int D, bool GRAM>
__global__ __launch_bounds__(kThreads) void k_scale(int64_t n, const VT* __restrict__ p,
                                                    const double* __restrict__ rinv,
                                                    VT* __restrict__ xn, VT* __restrict__ zcol,
                                                    int64_t ldz, double* partials,
                                                    unsigned* counter, double* gam, double* rinv2,
                                                    double* nrm_gam, double* nrm_ginv, int* flags) {
  constexpr int NV = GRAM ? D * D : 1;
  __shared__ double smem[kThreads > NV * (kThreads / kWave) ? kThreads : NV * (kThreads / kWave)];
  __shared__ double ri[D * D];
  if (threadIdx.x < D * D) ri[threadIdx.x] = rinv[threadIdx.x];
  __syncthreads();
  double g[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) g[i] = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
    VT v[D], o[D];
#pragma unroll
    for (int j = 0; j < D; ++j) v[j] = p[r * D + j];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      VT s = VT(0);
#pragma unroll
      for (int b = 0; b <= a; ++b) s = fma(v[b], VT(ri[b + a * D]), s);
      o[a] = s;
    }
#pragma unroll
    for (int j = 0; j < D; ++j) xn[r * D + j] = o[j];
    if (zcol) {
#pragma unroll
      for (int j = 0; j < D; ++j) zcol[r + j * ldz] = o[j];
    }
    if constexpr (GRAM) {
#pragma unroll
      for (int a = 0; a < D; ++a)
#pragma unroll
        for (int b = 0; b < D; ++b) g[a + b * D] += (double)o[a] * (double)o[b];
    }
  }
  if constexpr (GRAM) {
    block_sum<NV>(g, smem);
    __shared__ double res[NV];
    if (grid_sum_last<NV>(g, partials, counter, res, smem)) {
      if (threadIdx.x == 0) {
        double r2[NV], r2i[NV], gn[NV], rin[NV];
        const bool ok = chol_upper_inv(D, res, r2, r2i);
        if (!ok) atomicOr(flags + 1, 1);
        // Gamma <- R2 Gamma ; (R2 Gamma)^{-1} = Gamma^{-1} R2^{-1}
        for (int i = 0; i < D; ++i)
          for (int j = 0; j < D; ++j) {
            double s = 0.0, t = 0.0;
            for (int l = 0; l < D; ++l) {
              s += r2[i + l * D] * gam[l + j * D];
              t += rinv[i + l * D] * r2i[l + j * D];
            }
            gn[i + j * D] = s;
            rin[i + j * D] = t;
          }
        for (int i = 0; i < NV; ++i) { gam[i] = gn[i]; rinv2[i] = r2i[i]; }
        if (nrm_gam) *nrm_gam = fro(D, gn);
        if (nrm_ginv) *nrm_ginv = fro(D, rin);
      }
    }
  }
}

// ---------------------------------------------------------------------------
// W-recurrence (Sec. 4.2): column ell+1 of the bounds w_{k,j} >= ||Q_k^T Q_j||.
// One block.  W is (ldw x ldw) column-major, blocks numbered from 1.  Sets
// flags[0] = 1 (and counts the event in flags[3]) when a bound exceeds u_RO,
// in which case the caller's reorthogonalisation kernels run and the columns
// ell and ell+1 are reset to u_d here.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_wrec(int ell, int l0, double u_d, double u_ro,
                                              const double* __restrict__ n_xi,
                                              const double* __restrict__ n_gam,
                                              const double* __restrict__ n_ginv,
                                              const double* __restrict__ n_theta,
                                              const double* __restrict__ n_f, double* w, int ldw,
                                              int* flags) {
  __shared__ double red[256];
  __shared__ double sum_f_s;
  const int t = threadIdx.x;
  auto W = [&](int k, int j) -> double& { return w[k + (int64_t)j * ldw]; };
  // sum_{i <= l0} w_{i,ell} ||F_i||
  double s = 0.0;
  for (int i = 1 + t; i <= l0; i += blockDim.x) s += W(i, ell) * n_f[i];
  red[t] = s;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) red[t] += red[t + off];
    __syncthreads();
  }
  if (t == 0) sum_f_s = red[0];
  __syncthreads();
  const double sum_f = sum_f_s;
  const double gi = n_ginv[ell];
  double mx = 0.0;
  for (int k = 1 + t; k <= ell; k += blockDim.x) {
    double v;
    if (k == ell) {
      v = u_d;
    } else if (k <= l0) {
      v = gi * (W(k, ell) * (n_theta[k] + n_xi[ell]) + W(l0 + 1, ell) * n_f[k] +
                W(k, ell - 1) * n_gam[ell - 1] + 2.0 * u_d);
    } else if (k == l0 + 1) {
      double acc = W(k, ell) * (n_xi[k] + n_xi[ell]) + sum_f + 2.0 * u_d;
      if (k < ell - 1) acc += W(k + 1, ell) * n_gam[k] + W(k, ell - 1) * n_gam[ell - 1];
      v = gi * acc;
    } else {
      double acc = W(k, ell) * (n_xi[k] + n_xi[ell]) + W(k - 1, ell) * n_gam[k - 1] + 2.0 * u_d;
      if (k < ell - 1) acc += W(k + 1, ell) * n_gam[k] + W(k, ell - 1) * n_gam[ell - 1];
      v = gi * acc;
    }
    W(k, ell + 1) = v;
    if (k < ell) mx = fmax(mx, v);
  }
  red[t] = mx;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) red[t] = fmax(red[t], red[t + off]);
    __syncthreads();
  }
  const bool need = red[0] > u_ro || !(red[0] == red[0]);
  __syncthreads();
  if (need) {
    for (int k = 1 + t; k < ell; k += blockDim.x) W(k, ell) = u_d;
    for (int k = 1 + t; k <= ell; k += blockDim.x) W(k, ell + 1) = u_d;
  }
  if (t == 0) {
    flags[0] = need ? 1 : 0;
    if (need) flags[3] += 1;
  }
}

// W columns col0 and col0+1 := u_d (rows above the diagonal), everything else of them zero
__global__ void k_w_reset(int col0, int ncols, double u_d, double* w, int ldw) {
  for (int c = col0; c < col0 + ncols; ++c)
    for (int k = 1 + threadIdx.x; k < ldw; k += blockDim.x) w[k + (int64_t)c * ldw] = k < c ? u_d : 0.0;
}

// ---------------------------------------------------------------------------
// Tall-skinny pair of the (partial) reorthogonalisation, CGS (Sec. 4.2):
//   H = Z^T C       (k x NC, split over row chunks, partials then reduce)
//   C = C - Z H
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

constexpr int kTnRows = 256;  // rows per LDS sub-tile

template <typename VT, int DA, int NA>
__global__ __launch_bounds__(kThreads) void k_ts_tn(const int* cond, int64_t n, int64_t chunk,
                                                    const VT* __restrict__ z, int64_t ldz, int k,
                                                    CPair<VT, DA, NA> cc, double* __restrict__ hpart) {
  constexpr int NC = DA * NA;
  constexpr int JW = NC >= 32 ? 1 : 32 / NC;  // columns per wave
  if (cond && *cond == 0) return;
  __shared__ VT cs[kTnRows * NC];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  const int nw = blockDim.x / kWave;
  const int64_t r0 = (int64_t)blockIdx.x * chunk;
  const int64_t r1 = min(n, r0 + chunk);
  const int jbase = blockIdx.y * (nw * JW) + wid * JW;
  double acc[JW][NC];
#pragma unroll
  for (int q = 0; q < JW; ++q)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[q][c] = 0.0;
  for (int64_t t0 = r0; t0 < r1; t0 += kTnRows) {
    const int rows = (int)min((int64_t)kTnRows, r1 - t0);
    __syncthreads();
    for (int i = threadIdx.x; i < rows * NC; i += blockDim.x)
      cs[i] = cc.get(t0 + i / NC, i % NC);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < JW; ++q) {
      const int j = jbase + q;
      if (j >= k) break;
      const VT* zc = z + (int64_t)j * ldz + t0;
      for (int i = lane; i < rows; i += kWave) {
        const double zv = (double)zc[i];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[q][c] = fma(zv, (double)cs[i * NC + c], acc[q][c]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < JW; ++q) {
    const int j = jbase + q;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double v = wave_sum(acc[q][c]);
      if (lane == 0 && j < k) hpart[((int64_t)blockIdx.x * k + j) * NC + c] = v;
    }
  }
}

// H[j][c] = sum over chunks of the partials (fixed order)
__global__ void k_ts_reduce(const int* cond, int nchunks, int kc, const double* __restrict__ hpart,
                            double* __restrict__ h) {
  if (cond && *cond == 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kc) return;
  double s = 0.0;
  for (int b = 0; b < nchunks; ++b) s += hpart[(int64_t)b * kc + i];
  h[i] = s;
}

// C -= Z H ; with GRAM also reduces C^T C and (last block) stores R^{-1} of its
// Cholesky factor in rinv (NC x NC) for the final re-orthonormalisation.
constexpr int kNnJ = 256;  // H rows staged in LDS per pass

template <typename VT, int DA, int NA, bool GRAM>
__global__ __launch_bounds__(kThreads) void k_ts_nn(const int* cond, int64_t n,
                                                    const VT* __restrict__ z, int64_t ldz, int k,
                                                    const double* __restrict__ h,
                                                    CPair<VT, DA, NA> cc, double* partials,
                                                    unsigned* counter, double* rinv, int* flags) {
  constexpr int NC = DA * NA;
  constexpr int NV = GRAM ? NC * NC : 1;
  if (cond && *cond == 0) return;
  __shared__ double hs[kNnJ * NC];
  __shared__ double smem[kThreads > NV * (kThreads / kWave) ? kThreads : NV * (kThreads / kWave)];
  double g[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) g[i] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t rbeg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  // every thread of the block walks the same number of row iterations so the
  // __syncthreads around the LDS staging stay uniform
  const int64_t iters = (n + stride - 1) / stride;
  for (int64_t it = 0; it < iters; ++it) {
    const int64_t r = rbeg + it * stride;
    const bool valid = r < n;
    double acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = 0.0;
    for (int j0 = 0; j0 < k; j0 += kNnJ) {
      const int jn = min(kNnJ, k - j0);
      __syncthreads();
      for (int i = threadIdx.x; i < jn * NC; i += blockDim.x) hs[i] = h[(int64_t)j0 * NC + i];
      __syncthreads();
      if (valid) {
        const VT* zr = z + r + (int64_t)j0 * ldz;
        for (int j = 0; j < jn; ++j) {
          const double zv = (double)zr[(int64_t)j * ldz];
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[c] = fma(zv, hs[j * NC + c], acc[c]);
        }
      }
    }
    if (valid) {
      VT o[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        o[c] = VT((double)cc.get(r, c) - acc[c]);
        cc.set(r, c, o[c]);
      }
      if constexpr (GRAM) {
#pragma unroll
        for (int a = 0; a < NC; ++a)
#pragma unroll
          for (int b = 0; b < NC; ++b) g[a + b * NC] += (double)o[a] * (double)o[b];
      }
    }
  }
  if constexpr (GRAM) {
    block_sum<NV>(g, smem);
    __shared__ double res[NV];
    if (grid_sum_last<NV>(g, partials, counter, res, smem)) {
      if (threadIdx.x == 0) {
        double r[NV], ri[NV];
        if (!chol_upper_inv(NC, res, r, ri)) atomicOr(flags + 1, 1);
        // rinv holds R^{-1} followed by R
        for (int i = 0; i < NV; ++i) { rinv[i] = ri[i]; rinv[NV + i] = r[i]; }
      }
    }
  }
}

// C = C R^{-1} (NC columns), written back to the arrays and, if z0 is given,
// to NC consecutive basis columns starting at z0.
template <typename VT, int DA, int NA>
__global__ __launch_bounds__(kThreads) void k_ts_scale(const int* cond, int64_t n,
                                                       CPair<VT, DA, NA> cc,
                                                       const double* __restrict__ rinv,
                                                       VT* __restrict__ z0, int64_t ldz) {
  constexpr int NC = DA * NA;
  if (cond && *cond == 0) return;
  __shared__ double ri[NC * NC];
  if (threadIdx.x < NC * NC) ri[threadIdx.x] = rinv[threadIdx.x];
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

__global__ void k_sum_parts(int nparts, int k, const double* __restrict__ part, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= k) return;
  double s = 0.0;
  for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * k + c];
  out[c] = s;
}

// CGLS update: alpha_c = gamma_c / qq_c (0 for inactive columns)
//   x += alpha p ; s -= alpha q
__global__ void k_cgls_xs(int64_t n, int64_t m, int k, const double* __restrict__ gamma,
                          const double* __restrict__ qq, const int* __restrict__ active,
                          double* __restrict__ x, const double* __restrict__ p,
                          double* __restrict__ s, const double* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t tot = (n > m ? n : m) * k;
  if (i >= tot) return;
  const int c = (int)(i % k);
  const double al = (active[c] && qq[c] > 0.0) ? gamma[c] / qq[c] : 0.0;
  if (al == 0.0) return;
  if (i < n * k) x[i] = fma(al, p[i], x[i]);
  if (i < m * k) s[i] = fma(-al, q[i], s[i]);
}

// CGLS direction: beta_c = gnew_c / gamma_c ; p = r + beta p (active columns only)
__global__ void k_cgls_p(int64_t n, int k, const double* __restrict__ gnew,
                         const double* __restrict__ gamma, const int* __restrict__ active,
                         const double* __restrict__ r, double* __restrict__ p) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * k) return;
  const int c = (int)(i % k);
  if (!active[c]) return;
  const double be = gamma[c] > 0.0 ? gnew[c] / gamma[c] : 0.0;
  p[i] = fma(be, p[i], r[i]);
}

// CG on A^T A: alpha = rr / pq ; w += alpha p ; r -= alpha q
__global__ void k_cg_wr(int64_t n, int k, const double* __restrict__ rr, const double* __restrict__ pq,
                        const int* __restrict__ active, double* __restrict__ w,
                        const double* __restrict__ p, double* __restrict__ r,
                        const double* __restrict__ q) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * k) return;
  const int c = (int)(i % k);
  const double al = (active[c] && pq[c] > 0.0) ? rr[c] / pq[c] : 0.0;
  if (al == 0.0) return;
  w[i] = fma(al, p[i], w[i]);
  r[i] = fma(-al, q[i], r[i]);
}

// x -= y (elementwise)
__global__ void k_sub(int64_t cnt, double* __restrict__ x, const double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) x[i] -= y[i];
}

// ===========================================================================
// host launchers
// ===========================================================================
template <typename VT>
void sub_gram(nsp_ctx* c, int d, int64_t n, VT* p, const VT* x, const double* xi, double* gam_out,
              double* rinv, double* nrm_gam, double* nrm_ginv) {
  const unsigned grid = cap_grid(n, kThreads, kRedBlocks);
  int* flags = c->flags.as<int>();
#define NSP_SG(D)                                                                              \
  case D:                                                                                      \
    if (xi)                                                                                    \
      k_sub_gram<VT, D, true><<<grid, kThreads, 0, c->stream>>>(n, p, x, xi, c->red.partials,  \
          c->red.counter, gam_out, rinv, nrm_gam, nrm_ginv, flags);                            \
    else                                                                                       \
      k_sub_gram<VT, D, false><<<grid, kThreads, 0, c->stream>>>(n, p, x, xi, c->red.partials, \
          c->red.counter, gam_out, rinv, nrm_gam, nrm_ginv, flags);                            \
    break;
  switch (d) { NSP_SG(1) NSP_SG(2) NSP_SG(4) NSP_SG(8) default: throw Error(NSP_ERR_ARG, "d"); }
#undef NSP_SG
  NSP_HIP(hipGetLastError());
}
template void sub_gram<double>(nsp_ctx*, int, int64_t, double*, const double*, const double*,
                               double*, double*, double*, double*);
template void sub_gram<float>(nsp_ctx*, int, int64_t, float*, const float*, const double*, double*,
                              double*, double*, double*);

template <typename VT>
void scale_block(nsp_ctx* c, int d, int64_t n, const VT* p, const double* rinv, VT* xn, VT* zcol,
                 int64_t ldz, bool gram, double* gam, double* rinv2, double* nrm_gam,
                 double* nrm_ginv) {
  const unsigned grid = cap_grid(n, kThreads, kRedBlocks);
  int* flags = c->flags.as<int>();
#define NSP_SC(D)                                                                              \
  case D:                                                                                      \
    if (gram)                                                                                  \
      k_scale<VT, D, true><<<grid, kThreads, 0, c->stream>>>(n, p, rinv, xn, zcol, ldz,        \
          c->red.partials, c->red.counter, gam, rinv2, nrm_gam, nrm_ginv, flags);              \
    else                                                                                       \
      k_scale<VT, D, false><<<grid, kThreads, 0, c->stream>>>(n, p, rinv, xn, zcol, ldz,       \
          c->red.partials, c->red.counter, gam, rinv2, nrm_gam, nrm_ginv, flags);              \
    break;
  switch (d) { NSP_SC(1) NSP_SC(2) NSP_SC(4) NSP_SC(8) default: throw Error(NSP_ERR_ARG, "d"); }
#undef NSP_SC
  NSP_HIP(hipGetLastError());
}
template void scale_block<double>(nsp_ctx*, int, int64_t, const double*, const double*, double*,
                                  double*, int64_t, bool, double*, double*, double*, double*);
template void scale_block<float>(nsp_ctx*, int, int64_t, const float*, const double*, float*,
                                 float*, int64_t, bool, double*, double*, double*, double*);

void wrec(nsp_ctx* c, int ell, int l0, double u_d, double u_ro, const double* n_xi,
          const double* n_gam, const double* n_ginv, const double* n_theta, const double* n_f,
          double* w, int ldw) {
  k_wrec<<<1, 256, 0, c->stream>>>(ell, l0, u_d, u_ro, n_xi, n_gam, n_ginv, n_theta, n_f, w, ldw,
                                   c->flags.as<int>());
  NSP_HIP(hipGetLastError());
}

void w_reset(nsp_ctx* c, int col0, int ncols, double u_d, double* w, int ldw) {
  k_w_reset<<<1, 256, 0, c->stream>>>(col0, ncols, u_d, w, ldw);
  NSP_HIP(hipGetLastError());
}

// Workspace need of the TN partials: nchunks * k * NC doubles.
int64_t ts_chunk_rows(int64_t n, int k, int nc) {
  const int jw = nc >= 32 ? 1 : 32 / nc;
  const int64_t col_groups = (k + 4 * jw - 1) / (4 * jw);
  // aim for ~2048 blocks in total, chunks of at least 256 rows
  int64_t chunks = std::max<int64_t>(1, 2048 / std::max<int64_t>(1, col_groups));
  int64_t rows = (n + chunks - 1) / chunks;
  rows = std::max<int64_t>(rows, kTnRows);
  rows = (rows + kTnRows - 1) / kTnRows * kTnRows;
  return rows;
}

template <typename VT, int DA, int NA>
static void ts_proj_t(nsp_ctx* c, const int* cond, int64_t n, const VT* z, int64_t ldz, int k,
                      VT* a0, VT* a1, double* h, double* hpart, bool gram, double* rinv) {
  constexpr int NC = DA * NA;
  constexpr int JW = NC >= 32 ? 1 : 32 / NC;
  CPair<VT, DA, NA> cc{a0, a1};
  const int64_t chunk = ts_chunk_rows(n, k, NC);
  const unsigned nchunks = (unsigned)((n + chunk - 1) / chunk);
  const unsigned gy = (unsigned)((k + 4 * JW - 1) / (4 * JW));
  if (k > 0) {
    dim3 grid(nchunks, gy);
    k_ts_tn<VT, DA, NA><<<grid, kThreads, 0, c->stream>>>(cond, n, chunk, z, ldz, k, cc, hpart);
    k_ts_reduce<<<nblk((int64_t)k * NC, 256), 256, 0, c->stream>>>(cond, (int)nchunks, k * NC, hpart, h);
  }
  const unsigned g2 = cap_grid(n, kThreads, 2048);
  if (gram)
    k_ts_nn<VT, DA, NA, true><<<std::min<unsigned>(g2, kRedBlocks), kThreads, 0, c->stream>>>(
        cond, n, z, ldz, k, h, cc, c->red.partials, c->red.counter, rinv, c->flags.as<int>());
  else
    k_ts_nn<VT, DA, NA, false><<<g2, kThreads, 0, c->stream>>>(cond, n, z, ldz, k, h, cc, nullptr,
                                                               nullptr, nullptr, c->flags.as<int>());
  NSP_HIP(hipGetLastError());
}

template <typename VT, int DA, int NA>
static void ts_scale_t(nsp_ctx* c, const int* cond, int64_t n, VT* a0, VT* a1, const double* rinv,
                       VT* z0, int64_t ldz) {
  CPair<VT, DA, NA> cc{a0, a1};
  k_ts_scale<VT, DA, NA><<<cap_grid(n, kThreads, 2048), kThreads, 0, c->stream>>>(cond, n, cc, rinv,
                                                                                  z0, ldz);
  NSP_HIP(hipGetLastError());
}

// One CGS pass of C = [a0 (| a1)] against the first k basis columns.
template <typename VT>
void ts_project(nsp_ctx* c, const int* cond, int d, int na, int64_t n, const VT* z, int64_t ldz,
                int k, VT* a0, VT* a1, double* h, double* hpart, bool gram, double* rinv) {
  if (k <= 0) {
    if (!gram) return;
  }
#define NSP_TP(D)                                                                              \
  case D:                                                                                      \
    if (na == 1) ts_proj_t<VT, D, 1>(c, cond, n, z, ldz, std::max(k, 0), a0, a1, h, hpart, gram, rinv); \
    else ts_proj_t<VT, D, 2>(c, cond, n, z, ldz, std::max(k, 0), a0, a1, h, hpart, gram, rinv);          \
    break;
  switch (d) { NSP_TP(1) NSP_TP(2) NSP_TP(4) NSP_TP(8) default: throw Error(NSP_ERR_ARG, "d"); }
#undef NSP_TP
}
template void ts_project<double>(nsp_ctx*, const int*, int, int, int64_t, const double*, int64_t,
                                 int, double*, double*, double*, double*, bool, double*);
template void ts_project<float>(nsp_ctx*, const int*, int, int, int64_t, const float*, int64_t, int,
                                float*, float*, double*, double*, bool, double*);

template <typename VT>
void ts_scale(nsp_ctx* c, const int* cond, int d, int na, int64_t n, VT* a0, VT* a1,
              const double* rinv, VT* z0, int64_t ldz) {
#define NSP_TS(D)                                                                              \
  case D:                                                                                      \
    if (na == 1) ts_scale_t<VT, D, 1>(c, cond, n, a0, a1, rinv, z0, ldz);                      \
    else ts_scale_t<VT, D, 2>(c, cond, n, a0, a1, rinv, z0, ldz);                              \
    break;
  switch (d) { NSP_TS(1) NSP_TS(2) NSP_TS(4) NSP_TS(8) default: throw Error(NSP_ERR_ARG, "d"); }
#undef NSP_TS
}
template void ts_scale<double>(nsp_ctx*, const int*, int, int, int64_t, double*, double*,
                               const double*, double*, int64_t);
template void ts_scale<float>(nsp_ctx*, const int*, int, int, int64_t, float*, float*,
                              const double*, float*, int64_t);

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
  k_sum_parts<<<nblk(k, 256), 256, 0, c->stream>>>((int)nb, k, part, out);
  NSP_HIP(hipGetLastError());
}

int64_t coldots_parts(int64_t rows) {
  const int64_t rpb = std::max<int64_t>(64, (rows + 1023) / 1024);
  return (rows + rpb - 1) / rpb;
}

void cgls_xs(nsp_ctx* c, int64_t n, int64_t m, int k, const double* gamma, const double* qq,
             const int* active, double* x, const double* p, double* s, const double* q) {
  const int64_t tot = std::max(n, m) * k;
  k_cgls_xs<<<nblk(tot, 256), 256, 0, c->stream>>>(n, m, k, gamma, qq, active, x, p, s, q);
  NSP_HIP(hipGetLastError());
}

void cgls_p(nsp_ctx* c, int64_t n, int k, const double* gnew, const double* gamma, const int* active,
            const double* r, double* p) {
  k_cgls_p<<<nblk(n * k, 256), 256, 0, c->stream>>>(n, k, gnew, gamma, active, r, p);
  NSP_HIP(hipGetLastError());
}

void cg_wr(nsp_ctx* c, int64_t n, int k, const double* rr, const double* pq, const int* active,
           double* w, const double* p, double* r, const double* q) {
  k_cg_wr<<<nblk(n * k, 256), 256, 0, c->stream>>>(n, k, rr, pq, active, w, p, r, q);
  NSP_HIP(hipGetLastError());
}

void sub_inplace(nsp_ctx* c, int64_t cnt, double* x, const double* y) {
  if (cnt <= 0) return;
  k_sub<<<nblk(cnt, 256), 256, 0, c->stream>>>(cnt, x, y);
  NSP_HIP(hipGetLastError());
}

}  // namespace nsp
