// Sparse kernels: CSR SpMM (y = A x), the fused transposed product of one
// Lanczos step (z = A^T y + eps D x - X_prev Gamma^T, with the Xi dots),
// wide SpMM for many right-hand sides, SDDMM, and the set-up work of
// nullspace_init (stored transpose, random draws, norms).
//
// The operator B = A^T A + eps D is applied matrix-free exactly as in Sec. 1.2
// of the paper: one CSR product with A, one with the stored CSR of A^T.
// Row-interleaved blocks: a block of d columns is stored n x d row-major so a
// gather of row c of the block reads d contiguous values.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "common.h"
#include "device_util.h"
#include "kernels.h"

namespace nsp {

// ---------------------------------------------------------------------------
// y(rows x D) = A x, narrow blocks (D <= 8); LPR lanes cooperate on one row.
// ---------------------------------------------------------------------------
template <typename VT, int D, int LPR>
__global__ __launch_bounds__(kThreads) void k_spmm(int64_t nrows, const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ ci,
                                                   const VT* __restrict__ av,
                                                   const VT* __restrict__ x, VT* __restrict__ y) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = g / LPR;
  const int lane = threadIdx.x % LPR;
  double acc[D];  // FP64 accumulation also for FP32 operands
#pragma unroll
  for (int j = 0; j < D; ++j) acc[j] = 0.0;
  if (row < nrows) {
    const int beg = rp[row], end = rp[row + 1];
    for (int p = beg + lane; p < end; p += LPR) {
      const double a = av[p];
      const VT* xr = x + (int64_t)ci[p] * D;
#pragma unroll
      for (int j = 0; j < D; ++j) acc[j] = fma(a, (double)xr[j], acc[j]);
    }
  }
#pragma unroll
  for (int j = 0; j < D; ++j) acc[j] = group_sum<double, LPR>(acc[j]);
  if (row < nrows && lane == 0) {
#pragma unroll
    for (int j = 0; j < D; ++j) y[row * D + j] = VT(acc[j]);
  }
}

// ---------------------------------------------------------------------------
// One Lanczos step's second product, fused (Alg. 2 inner loop):
//   P = A^T Y + eps D X  [- Xp Gamma_prev^T]            (three-term recurrence)
//   per-block partials of Xi = X^T P (D x D) when XI is set; the QR kernel
//   that follows reduces them in block order (deterministic)
// Y (m x D), X, Xp, P (n x D) row-interleaved.  Gamma_prev is D x D column-major.
// ---------------------------------------------------------------------------
template <typename VT, int D, int LPR, bool PREV, bool XI>
__global__ __launch_bounds__(kThreads) void k_spmmT_step(
    int64_t nrows, const int32_t* __restrict__ rp, const int32_t* __restrict__ ci,
    const VT* __restrict__ av, const VT* __restrict__ y, const VT* __restrict__ x,
    const double* __restrict__ dv, double eps, const VT* __restrict__ xp,
    const double* __restrict__ gprev, VT* __restrict__ out, double* __restrict__ part_xi) {
  __shared__ double smem[kThreads > D * D * (kThreads / kWave) ? kThreads : D * D * (kThreads / kWave)];
  __shared__ double gp[D * D];
  if (PREV) {
    if (threadIdx.x < D * D) gp[threadIdx.x] = gprev[threadIdx.x];
    __syncthreads();
  }
  constexpr int NV = XI ? D * D : 1;
  double dots[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) dots[i] = 0.0;
  const int lane = threadIdx.x % LPR;
  const int64_t rows_per_grid = (int64_t)gridDim.x * (blockDim.x / LPR);
  // grid-stride over rows; the LPR lanes of a group always share ``row``
  for (int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / LPR; row < nrows;
       row += rows_per_grid) {
    double acc[D];  // FP64 accumulation also for FP32 operands
#pragma unroll
    for (int j = 0; j < D; ++j) acc[j] = 0.0;
    const int beg = rp[row], end = rp[row + 1];
    for (int p = beg + lane; p < end; p += LPR) {
      const double a = av[p];
      const VT* yr = y + (int64_t)ci[p] * D;
#pragma unroll
      for (int j = 0; j < D; ++j) acc[j] = fma(a, (double)yr[j], acc[j]);
    }
#pragma unroll
    for (int j = 0; j < D; ++j) acc[j] = group_sum<double, LPR>(acc[j]);
    if (lane == 0) {
      const double sd = eps * dv[row];
      double xr[D];
#pragma unroll
      for (int j = 0; j < D; ++j) xr[j] = x[row * D + j];
#pragma unroll
      for (int j = 0; j < D; ++j) acc[j] = fma(sd, xr[j], acc[j]);
      if (PREV) {
        double pr[D];
#pragma unroll
        for (int j = 0; j < D; ++j) pr[j] = xp[row * D + j];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          double s = acc[a];
#pragma unroll
          for (int b = 0; b < D; ++b) s = fma(-pr[b], gp[a + b * D], s);
          acc[a] = s;
        }
      }
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const VT o = VT(acc[j]);
        out[row * D + j] = o;
        acc[j] = (double)o;  // the Xi sums see the stored values
      }
      if constexpr (XI) {
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int b = 0; b < D; ++b) dots[a * D + b] += xr[a] * acc[b];
      }
    }
  }
  if constexpr (XI) {
    // per-block partial of X^T P; the next kernel reduces the partials
    block_sum<NV>(dots, smem);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i) part_xi[(size_t)blockIdx.x * NV + i] = dots[i];
    }
  }
}

// Y (rows x k, row-major) = A X (X: cols x k, row-major), many right-hand
// sides.  One wavefront per row, grid-stride over rows; lane l owns columns
// 4l .. 4l+3 of each 256-column panel, read as two 16-byte loads when k is even.
// With RED = 1 every block also writes partial column sums of Y^2, with RED = 2
// of Y .* X(row, :) (square A: the operand's own row), part[block * k + c],
// summed in block order by reduce_parts.
template <bool VEC, int RED>
__global__ __launch_bounds__(kThreads) void k_spmm_wide(int64_t nrows, int k,
                                                        const int32_t* __restrict__ rp,
                                                        const int32_t* __restrict__ ci,
                                                        const double* __restrict__ av,
                                                        const double* __restrict__ x,
                                                        double* __restrict__ y,
                                                        double* __restrict__ part) {
  constexpr int CPL = 4;
  constexpr int NWB = kThreads / kWave;
  constexpr bool SQ = RED != 0;
  __shared__ double red[SQ ? NWB : 1][SQ ? kWave * CPL : 1];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  const int64_t gw = (int64_t)blockIdx.x * NWB + wid;
  const int64_t nw = (int64_t)gridDim.x * NWB;
  for (int c0 = 0; c0 < k; c0 += kWave * CPL) {
    const int cb = c0 + lane * CPL;
    const bool full = cb + CPL <= k;
    double sq[CPL];
#pragma unroll
    for (int t = 0; t < CPL; ++t) sq[t] = 0.0;
    for (int64_t row = gw; row < nrows; row += nw) {
      const int beg = rp[row], end = rp[row + 1];
      double acc[CPL];
#pragma unroll
      for (int t = 0; t < CPL; ++t) acc[t] = 0.0;
      if (cb < k) {
        for (int p = beg; p < end; ++p) {
          const double a = av[p];
          const double* xr = x + (int64_t)ci[p] * k + cb;
          if (VEC && full) {
            const double2 u = *reinterpret_cast<const double2*>(xr);
            const double2 v = *reinterpret_cast<const double2*>(xr + 2);
            acc[0] = fma(a, u.x, acc[0]);
            acc[1] = fma(a, u.y, acc[1]);
            acc[2] = fma(a, v.x, acc[2]);
            acc[3] = fma(a, v.y, acc[3]);
          } else {
#pragma unroll
            for (int t = 0; t < CPL; ++t)
              if (cb + t < k) acc[t] = fma(a, xr[t], acc[t]);
          }
        }
        double* yr = y + row * k + cb;
        if (VEC && full) {
          *reinterpret_cast<double2*>(yr) = make_double2(acc[0], acc[1]);
          *reinterpret_cast<double2*>(yr + 2) = make_double2(acc[2], acc[3]);
        } else {
#pragma unroll
          for (int t = 0; t < CPL; ++t)
            if (cb + t < k) yr[t] = acc[t];
        }
        if constexpr (RED == 1) {
#pragma unroll
          for (int t = 0; t < CPL; ++t) sq[t] = fma(acc[t], acc[t], sq[t]);
        } else if constexpr (RED == 2) {
          const double* xo = x + row * k + cb;
#pragma unroll
          for (int t = 0; t < CPL; ++t)
            if (cb + t < k) sq[t] = fma(acc[t], xo[t], sq[t]);
        }
      }
    }
    if constexpr (SQ) {
#pragma unroll
      for (int t = 0; t < CPL; ++t) red[wid][lane * CPL + t] = sq[t];
      __syncthreads();
      const int j = threadIdx.x;  // kThreads == kWave * CPL columns of the panel
      if (c0 + j < k) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NWB; ++w) s += red[w][j];
        part[(int64_t)blockIdx.x * k + c0 + j] = s;
      }
      __syncthreads();
    }
  }
}

// SDDMM on A's pattern: grad[p] = -2 <U_i, V_j> for p = (i, j); U (m x k), V (n x k) row-major.
__global__ __launch_bounds__(kThreads) void k_sddmm(int64_t nrows, int k, const int32_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci,
                                                    const double* __restrict__ u,
                                                    const double* __restrict__ v,
                                                    double* __restrict__ grad) {
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (row >= nrows) return;
  const int beg = rp[row], end = rp[row + 1];
  for (int p = beg; p < end; ++p) {
    const int64_t col = ci[p];
    double s = 0.0;
    for (int c = lane; c < k; c += kWave) s = fma(u[row * k + c], v[col * k + c], s);
    s = wave_sum(s);
    if (lane == 0) grad[p] = -2.0 * s;
  }
}

// k_spmm_wide for narrow blocks (k <= 4 LPR columns): LPR lanes per row with
// 4 columns each, 64 / LPR rows per wavefront, so that a block of a few
// columns (the backward pass's right-hand sides) keeps every lane busy.  The
// same products, sums and partials (part[block * k + c], rows and waves
// summed in a fixed order) as k_spmm_wide.
template <bool VEC, int RED, int LPR>
__global__ __launch_bounds__(kThreads) void k_spmm_narrow(int64_t nrows, int k,
                                                          const int32_t* __restrict__ rp,
                                                          const int32_t* __restrict__ ci,
                                                          const double* __restrict__ av,
                                                          const double* __restrict__ x,
                                                          double* __restrict__ y,
                                                          double* __restrict__ part) {
  constexpr int CPL = 4;
  constexpr int RPW = kWave / LPR;
  constexpr int NWB = kThreads / kWave;
  constexpr bool SQ = RED != 0;
  __shared__ double red[SQ ? kThreads * CPL : 1];
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
  const int sub = lane / LPR;         // the lane's row within the wavefront's group
  const int cb = (lane % LPR) * CPL;  // the lane's first column
  const bool full = cb + CPL <= k;
  const int64_t nw = (int64_t)gridDim.x * NWB;
  double sq[CPL];
#pragma unroll
  for (int t = 0; t < CPL; ++t) sq[t] = 0.0;
  for (int64_t g = (int64_t)blockIdx.x * NWB + wid; g * RPW < nrows; g += nw) {
    const int64_t row = g * RPW + sub;
    if (row >= nrows || cb >= k) continue;
    const int beg = rp[row], end = rp[row + 1];
    double acc[CPL];
#pragma unroll
    for (int t = 0; t < CPL; ++t) acc[t] = 0.0;
    for (int p = beg; p < end; ++p) {
      const double a = av[p];
      const double* xr = x + (int64_t)ci[p] * k + cb;
      if (VEC && full) {
        const double2 u = *reinterpret_cast<const double2*>(xr);
        const double2 v = *reinterpret_cast<const double2*>(xr + 2);
        acc[0] = fma(a, u.x, acc[0]);
        acc[1] = fma(a, u.y, acc[1]);
        acc[2] = fma(a, v.x, acc[2]);
        acc[3] = fma(a, v.y, acc[3]);
      } else {
#pragma unroll
        for (int t = 0; t < CPL; ++t)
          if (cb + t < k) acc[t] = fma(a, xr[t], acc[t]);
      }
    }
    double* yr = y + row * k + cb;
    if (VEC && full) {
      *reinterpret_cast<double2*>(yr) = make_double2(acc[0], acc[1]);
      *reinterpret_cast<double2*>(yr + 2) = make_double2(acc[2], acc[3]);
    } else {
#pragma unroll
      for (int t = 0; t < CPL; ++t)
        if (cb + t < k) yr[t] = acc[t];
    }
    if constexpr (RED == 1) {
#pragma unroll
      for (int t = 0; t < CPL; ++t) sq[t] = fma(acc[t], acc[t], sq[t]);
    } else if constexpr (RED == 2) {
      const double* xo = x + row * k + cb;
#pragma unroll
      for (int t = 0; t < CPL; ++t)
        if (cb + t < k) sq[t] = fma(acc[t], xo[t], sq[t]);
    }
  }
  if constexpr (SQ) {
#pragma unroll
    for (int t = 0; t < CPL; ++t) red[threadIdx.x * CPL + t] = sq[t];
    __syncthreads();
    // column j = l * CPL + t: its lanes are l, l + LPR, ... of every wavefront
    const int j = threadIdx.x;
    if (j < k) {
      const int l = j / CPL, t = j % CPL;
      double s4[4] = {0.0, 0.0, 0.0, 0.0};
      for (int w = 0; w < NWB; ++w)
#pragma unroll 4
        for (int r = 0; r < RPW; ++r) s4[r & 3] += red[(w * kWave + r * LPR + l) * CPL + t];
      part[(int64_t)blockIdx.x * k + j] = (s4[0] + s4[1]) + (s4[2] + s4[3]);
    }
  }
}

// ---------------------------------------------------------------------------
// set-up kernels
// ---------------------------------------------------------------------------
__global__ void k_gather_vals(int64_t nnz, const int32_t* __restrict__ perm,
                              const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nnz) dst[i] = src[perm[i]];
}

// flag[0] = 1 if a[i] != b[i] for some i (any thread may set it; only 0 -> 1)
__global__ void k_values_differ(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                                int* flag) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && !(a[i] == b[i])) flag[0] = 1;
}

__global__ void k_to_f32(int64_t n, const double* __restrict__ src, float* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (float)src[i];
}

// per-row sums of |a| and a^2; a non-finite value sets flag[0]
__global__ void k_row_abs_sums(int64_t nrows, const int32_t* __restrict__ rp,
                               const double* __restrict__ av, double* __restrict__ rabs,
                               double* __restrict__ rsq, int* flag) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nrows) return;
  double s = 0.0, q = 0.0;
  bool bad = false;
  for (int p = rp[row]; p < rp[row + 1]; ++p) {
    const double a = av[p];
    bad |= !isfinite(a);
    s += fabs(a);
    q += a * a;
  }
  rabs[row] = s;
  if (rsq) rsq[row] = q;
  if (bad) atomicOr(flag, 1);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter (i, stream, 0, 0),
// key (seed low, seed high).  uniform53 builds a double in [0,1) from 53 random
// bits; the normal pair comes from the Box-Muller transform.
struct Philox {
  __device__ static void round(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint64_t p0 = (uint64_t)M0 * c[0], p1 = (uint64_t)M1 * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t r0 = hi1 ^ c[1] ^ k0, r1 = lo1, r2 = hi0 ^ c[3] ^ k1, r3 = lo0;
    c[0] = r0; c[1] = r1; c[2] = r2; c[3] = r3;
  }
  __device__ static void gen(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t (&out)[4]) {
    uint32_t c[4] = {c0, c1, 0u, 0u};
    uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
    for (int r = 0; r < 10; ++r) {
      round(c, k0, k1);
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
  }
  __device__ static double u53(uint32_t a, uint32_t b) {
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6)) * (1.0 / 9007199254740992.0);
  }
};

// D[i] = uniform53(philox(i, stream=0)) ; Omega[i + j*n] from stream j+1 via Box-Muller
__global__ void k_philox_uniform(int64_t n, uint64_t seed, uint32_t stream, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t r[4];
  Philox::gen(seed, (uint32_t)i, stream, r);
  out[i] = Philox::u53(r[0], r[1]);
}

__global__ void k_philox_normal(int64_t n, uint64_t seed, uint32_t stream, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t r[4];
  Philox::gen(seed, (uint32_t)i, stream, r);
  const double u1 = 1.0 - Philox::u53(r[0], r[1]);  // (0, 1]
  const double u2 = Philox::u53(r[2], r[3]);
  out[i] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

// row-major (rows x k) <-> column-major (ld) conversions
__global__ void k_colmajor_to_rows(int64_t rows, int k, const double* __restrict__ src, int64_t ld,
                                   double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * k) return;
  const int64_t r = i / k, c = i % k;
  dst[i] = src[r + c * ld];
}

__global__ void k_rows_to_colmajor(int64_t rows, int k, const double* __restrict__ src,
                                   double* __restrict__ dst, int64_t ld) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows * k) return;
  const int64_t c = i / rows, r = i % rows;
  dst[r + c * ld] = src[r * k + c];
}

static inline unsigned nblocks(int64_t work, int per) { return (unsigned)((work + per - 1) / per); }

// ---------------------------------------------------------------------------
// host-side launchers
// ---------------------------------------------------------------------------
// ---------------------------------------------------------------------------
// CSR streaming, used for the Lanczos step's SpMV pair.  The rows are cut at
// init into row blocks of at most stream_tile(D) nonzeros (a longer row is a
// block of its own).  A workgroup streams a row block's column indices and
// values with consecutive lanes on consecutive nonzeros (coalesced), gathers
// the operand rows, parks the D products per nonzero in LDS, and then one
// thread per row sums that row's segment in order.  The grid is persistent:
// workgroup b takes row blocks b, b + grid, ...
// STEP adds the epilogue of the fused second product (k_spmmT_step):
//   P = A^T Y + eps D X [- Xp Gamma_prev^T], with per-workgroup partials of
//   Xi = X^T P when XI is set.
// ---------------------------------------------------------------------------
template <typename VT, int D, bool STEP, bool PREV, bool XI>
__global__ __launch_bounds__(kThreads) void k_csr_stream(
    int nrb, const int32_t* __restrict__ rblk, const int32_t* __restrict__ rp,
    const int32_t* __restrict__ ci, const VT* __restrict__ av, const VT* __restrict__ xin,
    const VT* __restrict__ x, const double* __restrict__ dv, double eps,
    const VT* __restrict__ xp, const double* __restrict__ gprev, VT* __restrict__ out,
    double* __restrict__ part_xi) {
  constexpr int TILE = stream_tile(D);
  constexpr int NV = XI ? D * D : 1;
  __shared__ double prod[TILE * D];  // FP64 products also for FP32 operands
  __shared__ double gp[D * D];
  __shared__ double smem[(kThreads / kWave) * NV];
  const int t = threadIdx.x;
  const int lane = t % kWave, wid = t / kWave;
  if (PREV && t < D * D) gp[t] = gprev[t];  // read after the loop's first barrier
  double dots[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) dots[i] = 0.0;
  // XCD-aware order: workgroups are dispatched round-robin over the 8 XCDs, so
  // workgroup w runs on XCD w % 8.  Each XCD takes one contiguous eighth of the
  // row blocks; with rows in locality order its gathers then stay in its own
  // L2.  The grid is a multiple of 8.
  const int xcd = blockIdx.x % kXcds, slot = blockIdx.x / kXcds, per = gridDim.x / kXcds;
  const int lo = (int)((int64_t)nrb * xcd / kXcds), hi = (int)((int64_t)nrb * (xcd + 1) / kXcds);
  for (int b = lo + slot; b < hi; b += per) {
    const int r0 = rblk[b], r1 = rblk[b + 1];
    const int e0 = rp[r0];
    const int cnt = rp[r1] - e0;
    const bool tiled = cnt <= TILE;  // uniform over the workgroup
    if (tiled && (!STEP || sizeof(VT) == 4)) {
      // the matrix is read once per product: non-temporal loads keep it from
      // evicting the gathered operand rows out of L2.  A thread owns at most
      // IPT entries of the tile: all their index and value loads are issued
      // before the first gather, then all gathers, so each thread keeps IPT
      // independent index-then-gather chains in flight instead of one.  (The
      // fused FP64 product keeps the plain loop below: with its epilogue the
      // extra registers cost more than the loads in flight gain; in FP32 the
      // batched loads take 6% off the symmetric-form product.)
      constexpr int IPT = (TILE + kThreads - 1) / kThreads;
      int32_t cidx[IPT];
      VT aval[IPT];  // storage precision until the multiply (half the registers in FP32)
#pragma unroll
      for (int u = 0; u < IPT; ++u) {
        const int i = t + u * kThreads;
        if (i < cnt) {
          aval[u] = __builtin_nontemporal_load(av + e0 + i);
          cidx[u] = __builtin_nontemporal_load(ci + e0 + i);
        }
      }
#pragma unroll
      for (int u = 0; u < IPT; ++u) {
        const int i = t + u * kThreads;
        if (i < cnt) {
          const VT* xr = xin + (int64_t)cidx[u] * D;
#pragma unroll
          for (int j = 0; j < D; ++j) prod[i * D + j] = (double)aval[u] * (double)xr[j];
        }
      }
    } else if (tiled) {
      for (int i = t; i < cnt; i += kThreads) {
        const double a = __builtin_nontemporal_load(av + e0 + i);
        const VT* xr = xin + (int64_t)__builtin_nontemporal_load(ci + e0 + i) * D;
#pragma unroll
        for (int j = 0; j < D; ++j) prod[i * D + j] = a * (double)xr[j];
      }
    } else {
      double acc[D];
#pragma unroll
      for (int j = 0; j < D; ++j) acc[j] = 0.0;
      for (int i = t; i < cnt; i += kThreads) {
        const double a = av[e0 + i];
        const VT* xr = xin + (int64_t)ci[e0 + i] * D;
#pragma unroll
        for (int j = 0; j < D; ++j) acc[j] = fma(a, (double)xr[j], acc[j]);
      }
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const double v = wave_sum(acc[j]);
        if (lane == 0) prod[wid * D + j] = v;
      }
    }
    __syncthreads();
    for (int r = r0 + t; r < r1; r += kThreads) {
      double s[D];
#pragma unroll
      for (int j = 0; j < D; ++j) s[j] = 0.0;
      if (tiled) {
        const int pe = rp[r + 1] - e0;
        for (int p = rp[r] - e0; p < pe; ++p)
#pragma unroll
          for (int j = 0; j < D; ++j) s[j] += prod[p * D + j];
      } else {  // a single long row, r == r0, t == 0
#pragma unroll
        for (int w = 0; w < kThreads / kWave; ++w)
#pragma unroll
          for (int j = 0; j < D; ++j) s[j] += prod[w * D + j];
      }
      double xr[D];
      if constexpr (STEP) {
        const double sd = eps * dv[r];
#pragma unroll
        for (int j = 0; j < D; ++j) xr[j] = x[(int64_t)r * D + j];
#pragma unroll
        for (int j = 0; j < D; ++j) s[j] = fma(sd, xr[j], s[j]);
        if (PREV) {
          double pr[D];
#pragma unroll
          for (int j = 0; j < D; ++j) pr[j] = xp[(int64_t)r * D + j];
#pragma unroll
          for (int a = 0; a < D; ++a) {
            double u = s[a];
#pragma unroll
            for (int q = 0; q < D; ++q) u = fma(-pr[q], gp[a + q * D], u);
            s[a] = u;
          }
        }
      }
#pragma unroll
      for (int j = 0; j < D; ++j) {
        const VT o = VT(s[j]);
        out[(int64_t)r * D + j] = o;
        s[j] = (double)o;  // the Xi sums see the stored values
      }
      if constexpr (STEP && XI) {
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int q = 0; q < D; ++q) dots[a * D + q] += xr[a] * s[q];
      }
    }
    __syncthreads();  // prod is rewritten by the next row block
  }
  if constexpr (XI) {
    block_sum<NV>(dots, smem);
    if (t == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i) part_xi[(size_t)blockIdx.x * NV + i] = dots[i];
    }
  }
}

template <typename VT, int D, bool STEP, bool PREV, bool XI>
static int csr_stream(nsp_ctx* c, const Csr& a, const VT* xin, const VT* x, const VT* xp,
                      const double* gprev, VT* out, double* part_xi) {
  const VT* av = nullptr;
  if constexpr (sizeof(VT) == 8) av = a.val; else av = a.val32;
  if (a.nrb == 0) return 0;
  // a multiple of kXcds workgroups, about one row block each up to the cap
  const int grid = std::min(kStreamBlocks, (a.nrb + kXcds - 1) / kXcds * kXcds);
  // with many workgroups the Xi partials go behind the first kMaxD^2 slots and
  // one extra launch sums them, so the next kernel reads a single partial
  const bool split = XI && grid > kRedBlocks;
  double* pw = split ? part_xi + kMaxD * kMaxD : part_xi;
  k_csr_stream<VT, D, STEP, PREV, XI><<<grid, kThreads, 0, c->stream>>>(
      a.nrb, a.rblk, a.rowptr, a.colind, av, xin, x, c->Dv.as<double>(), c->prm.eps, xp, gprev, out,
      pw);
  NSP_HIP(hipGetLastError());
  if (split) {
    reduce_parts(c, grid, D * D, pw, part_xi);
    return 1;
  }
  return grid;
}

// Row blocks for the streaming kernels: consecutive rows while their nonzeros
// fit in ``tile`` (and at most 1024 rows); a row longer than ``tile`` alone.
static std::vector<int32_t> stream_blocks(const std::vector<int32_t>& rp, int64_t rows, int tile) {
  std::vector<int32_t> b{0};
  int64_t start = 0, acc = 0;
  for (int64_t r = 0; r < rows; ++r) {
    const int64_t len = (int64_t)rp[r + 1] - rp[r];
    if (r > start && (acc + len > tile || r - start >= 1024)) {
      b.push_back((int32_t)r);
      start = r;
      acc = 0;
    }
    acc += len;
    if (len > tile) {
      b.push_back((int32_t)(r + 1));
      start = r + 1;
      acc = 0;
    }
  }
  if (b.back() != rows) b.push_back((int32_t)rows);
  return b;
}

template <typename VT, int D>
static void spmm_d(nsp_ctx* c, const Csr& a, const VT* x, VT* y) {
  const VT* av = nullptr;
  if constexpr (sizeof(VT) == 8) av = a.val; else av = a.val32;
  if (a.rows == 0) return;
#define NSP_SPMM_CASE(L)                                                                       \
  case L:                                                                                      \
    k_spmm<VT, D, L><<<nblocks(a.rows * L, kThreads), kThreads, 0, c->stream>>>(              \
        a.rows, a.rowptr, a.colind, av, x, y);                                                 \
    break;
  switch (a.lpr) {
    NSP_SPMM_CASE(1) NSP_SPMM_CASE(2) NSP_SPMM_CASE(4) NSP_SPMM_CASE(8) NSP_SPMM_CASE(16)
    NSP_SPMM_CASE(32)
    default: throw Error(NSP_ERR_ARG, "unsupported lanes-per-row");
  }
#undef NSP_SPMM_CASE
  NSP_HIP(hipGetLastError());
}

template <typename VT>
void spmm_block(nsp_ctx* c, const Csr& a, int d, const VT* x, VT* y) {
  if (a.rblk && a.rblk_d == d) {
    switch (d) {
      case 1: csr_stream<VT, 1, false, false, false>(c, a, x, nullptr, nullptr, nullptr, y, nullptr); return;
      case 2: csr_stream<VT, 2, false, false, false>(c, a, x, nullptr, nullptr, nullptr, y, nullptr); return;
      case 4: csr_stream<VT, 4, false, false, false>(c, a, x, nullptr, nullptr, nullptr, y, nullptr); return;
      case 8: csr_stream<VT, 8, false, false, false>(c, a, x, nullptr, nullptr, nullptr, y, nullptr); return;
      default: break;
    }
  }
  switch (d) {
    case 1: spmm_d<VT, 1>(c, a, x, y); break;
    case 2: spmm_d<VT, 2>(c, a, x, y); break;
    case 4: spmm_d<VT, 4>(c, a, x, y); break;
    case 8: spmm_d<VT, 8>(c, a, x, y); break;
    default: throw Error(NSP_ERR_ARG, "block size must be 1, 2, 4 or 8");
  }
}
template void spmm_block<double>(nsp_ctx*, const Csr&, int, const double*, double*);
template void spmm_block<float>(nsp_ctx*, const Csr&, int, const float*, float*);

template <typename VT, int D, bool PREV, bool XI>
static int spmmT_step_d(nsp_ctx* c, const VT* y, const VT* x, const VT* xp, const double* gprev,
                        VT* out, double* part_xi) {
  const Csr& a = c->AT;
  const VT* av = nullptr;
  if constexpr (sizeof(VT) == 8) av = a.val; else av = a.val32;
  const int64_t groups = (a.rows + 0);
  unsigned grid = nblocks(groups * a.lpr, kThreads);
  // d = 1: one pass over the rows (the next kernel sums up to kStreamBlocks
  // scalar partials); wider blocks keep the grid (and their d x d partials) small
  if (XI) grid = std::min<unsigned>(grid, (unsigned)(D == 1 ? kStreamBlocks : kRedBlocks));
#define NSP_T_CASE(L)                                                                          \
  case L:                                                                                      \
    k_spmmT_step<VT, D, L, PREV, XI><<<grid, kThreads, 0, c->stream>>>(                        \
        a.rows, a.rowptr, a.colind, av, y, x, c->Dv.as<double>(), c->prm.eps, xp, gprev, out,  \
        part_xi);                                                                              \
    break;
  switch (a.lpr) {
    NSP_T_CASE(1) NSP_T_CASE(2) NSP_T_CASE(4) NSP_T_CASE(8) NSP_T_CASE(16) NSP_T_CASE(32)
    default: throw Error(NSP_ERR_ARG, "unsupported lanes-per-row");
  }
#undef NSP_T_CASE
  NSP_HIP(hipGetLastError());
  return (int)grid;
}

template <typename VT>
int spmmT_step(nsp_ctx* c, int d, const VT* y, const VT* x, const VT* xp, const double* gprev,
               VT* out, double* part_xi) {
  if (d == 8 && part_xi) {
    // block size 8: the product without its own Xi sums (their 64 per-thread
    // accumulators spill), then the Xi partials on the matrix cores
    spmmT_step<VT>(c, d, y, x, xp, gprev, out, nullptr);
    return xi8_parts<VT>(c, c->AT.rows, x, out, part_xi);
  }
  const bool prev = xp != nullptr, dots = part_xi != nullptr;
  const Csr& at = c->AT;
  if (at.rblk && at.rblk_d == d) {
#define NSP_STREAM(D)                                                                                     \
    if (prev && dots) return csr_stream<VT, D, true, true, true>(c, at, y, x, xp, gprev, out, part_xi);   \
    else if (prev) return csr_stream<VT, D, true, true, false>(c, at, y, x, xp, gprev, out, part_xi);     \
    else if (dots) return csr_stream<VT, D, true, false, true>(c, at, y, x, xp, gprev, out, part_xi);     \
    else return csr_stream<VT, D, true, false, false>(c, at, y, x, xp, gprev, out, part_xi);
    switch (d) {
      case 1: { NSP_STREAM(1) }
      case 2: { NSP_STREAM(2) }
      case 4: { NSP_STREAM(4) }
      case 8: { NSP_STREAM(8) }
      default: break;
    }
#undef NSP_STREAM
  }
#define NSP_DISPATCH(D)                                                                        \
  if (prev && dots) return spmmT_step_d<VT, D, true, true>(c, y, x, xp, gprev, out, part_xi);   \
  else if (prev) return spmmT_step_d<VT, D, true, false>(c, y, x, xp, gprev, out, part_xi);     \
  else if (dots) return spmmT_step_d<VT, D, false, true>(c, y, x, xp, gprev, out, part_xi);     \
  else return spmmT_step_d<VT, D, false, false>(c, y, x, xp, gprev, out, part_xi);
  switch (d) {
    case 1: { NSP_DISPATCH(1) break; }
    case 2: { NSP_DISPATCH(2) break; }
    case 4: { NSP_DISPATCH(4) break; }
    case 8: { NSP_DISPATCH(8) break; }
    default: throw Error(NSP_ERR_ARG, "block size must be 1, 2, 4 or 8");
  }
#undef NSP_DISPATCH
}
template int spmmT_step<double>(nsp_ctx*, int, const double*, const double*, const double*,
                                const double*, double*, double*);
template int spmmT_step<float>(nsp_ctx*, int, const float*, const float*, const float*,
                               const double*, float*, double*);

int spmm_wide(nsp_ctx* c, const Csr& a, int k, const double* x, double* y, double* part, bool dot) {
  if (a.rows == 0 || k == 0) return 0;
  static_assert(kThreads == 4 * kWave, "one 256-column panel per block");
  if (dot) NSP_REQUIRE(a.rows == a.cols, "the fused x . Ax sums need a square A");
  const bool vec = k % 2 == 0;
  const int red = part ? (dot ? 2 : 1) : 0;
  if (k <= 64) {
    // narrow block: LPR lanes of 4 columns per row, 64 / LPR rows per wavefront
    const int lpr = k <= 4 ? 1 : k <= 8 ? 2 : k <= 16 ? 4 : k <= 32 ? 8 : 16;
    const int64_t groups = (a.rows + kWave / lpr - 1) / (kWave / lpr);
    const int grid = (int)std::min<int64_t>(nblocks(groups, kThreads / kWave), kWideBlocks);
#define NSP_N(V, R, L) k_spmm_narrow<V, R, L><<<grid, kThreads, 0, c->stream>>>(a.rows, k, a.rowptr, a.colind, a.val, x, y, part)
#define NSP_NL(V, R) switch (lpr) { case 1: NSP_N(V, R, 1); break; case 2: NSP_N(V, R, 2); break; \
    case 4: NSP_N(V, R, 4); break; case 8: NSP_N(V, R, 8); break; default: NSP_N(V, R, 16); }
#define NSP_NV(R) if (vec) { NSP_NL(true, R) } else { NSP_NL(false, R) }
    if (red == 2) { NSP_NV(2); } else if (red == 1) { NSP_NV(1); } else { NSP_NV(0); }
#undef NSP_NV
#undef NSP_NL
#undef NSP_N
    NSP_HIP(hipGetLastError());
    return grid;
  }
  const int grid = (int)std::min<int64_t>(nblocks(a.rows, kThreads / kWave), kWideBlocks);
#define NSP_W(V, R) k_spmm_wide<V, R><<<grid, kThreads, 0, c->stream>>>(a.rows, k, a.rowptr, a.colind, a.val, x, y, part)
#define NSP_WV(R) if (vec) NSP_W(true, R); else NSP_W(false, R)
  if (red == 2) { NSP_WV(2); } else if (red == 1) { NSP_WV(1); } else { NSP_WV(0); }
#undef NSP_WV
#undef NSP_W
  NSP_HIP(hipGetLastError());
  return grid;
}

void sddmm(nsp_ctx* c, int k, const double* u, const double* v, double* grad) {
  const Csr& a = c->A;
  if (a.rows == 0) return;
  const int rows_per_block = kThreads / kWave;
  k_sddmm<<<nblocks(a.rows, rows_per_block), kThreads, 0, c->stream>>>(a.rows, k, a.rowptr,
                                                                        a.colind, u, v, grad);
  NSP_HIP(hipGetLastError());
}

void colmajor_to_rows(nsp_ctx* c, int64_t rows, int k, const double* src, int64_t ld, double* dst) {
  if (rows * k == 0) return;
  k_colmajor_to_rows<<<nblocks(rows * k, kThreads), kThreads, 0, c->stream>>>(rows, k, src, ld, dst);
  NSP_HIP(hipGetLastError());
}

void rows_to_colmajor(nsp_ctx* c, int64_t rows, int k, const double* src, double* dst, int64_t ld) {
  if (rows * k == 0) return;
  k_rows_to_colmajor<<<nblocks(rows * k, kThreads), kThreads, 0, c->stream>>>(rows, k, src, dst, ld);
  NSP_HIP(hipGetLastError());
}

// Lanes per row: the power of two nearest the mean row length, in [1, 32].
static int choose_lpr(int64_t rows, int64_t nnz) {
  const double mean = rows ? (double)nnz / (double)rows : 1.0;
  int l = 1;
  while (l < 32 && (double)(l * 2) <= mean * 1.41421356) l *= 2;
  return l;
}

void locality_order(int64_t m, int64_t n, const int64_t* rp, const int32_t* ci,
                    int32_t* row_order, int32_t* col_order) {
  const int64_t nnz = rp[m];
  // column -> rows lists (pattern of A^T) by a counting sort
  std::vector<int64_t> cp(n + 1, 0);
  std::vector<int32_t> cr(std::max<int64_t>(nnz, 1));
  for (int64_t p = 0; p < nnz; ++p) cp[ci[p] + 1]++;
  for (int64_t j = 0; j < n; ++j) cp[j + 1] += cp[j];
  {
    std::vector<int64_t> next(cp.begin(), cp.end() - 1);
    for (int64_t i = 0; i < m; ++i)
      for (int64_t p = rp[i]; p < rp[i + 1]; ++p) cr[next[ci[p]]++] = (int32_t)i;
  }
  std::vector<uint8_t> rseen(m, 0), cseen(n, 0);
  int64_t nr = 0, nc = 0;
  // col_order doubles as the queue of the search; each start column begins a
  // new connected piece once the previous piece is exhausted
  for (int64_t s = 0; s < n; ++s) {
    if (cseen[s]) continue;
    cseen[s] = 1;
    col_order[nc++] = (int32_t)s;
    for (int64_t h = nc - 1; h < nc; ++h) {
      const int32_t j = col_order[h];
      for (int64_t q = cp[j]; q < cp[j + 1]; ++q) {
        const int32_t i = cr[q];
        if (rseen[i]) continue;
        rseen[i] = 1;
        row_order[nr++] = i;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) {
          const int32_t j2 = ci[p];
          if (!cseen[j2]) {
            cseen[j2] = 1;
            col_order[nc++] = j2;
          }
        }
      }
    }
  }
  for (int64_t i = 0; i < m; ++i)  // rows without entries go last
    if (!rseen[i]) row_order[nr++] = (int32_t)i;
}

// The library's copy of A: rows and columns in the locality order (or the
// caller's order when reordering is off), columns sorted within a row, then
// the stored transpose by a counting sort by column.  Host work happens only
// here, once, at init; values are permuted on the device.
void prepare_matrix(nsp_ctx* c, const int64_t* rowptr64, const int32_t* colind, const double* vals) {
  const int64_t m = c->m, n = c->n, nnz = c->nnz;
  std::vector<int64_t> hrp(m + 1);
  std::vector<int32_t> hci(std::max<int64_t>(nnz, 1));
  NSP_HIP(hipMemcpy(hrp.data(), rowptr64, sizeof(int64_t) * (m + 1), hipMemcpyDeviceToHost));
  if (nnz) NSP_HIP(hipMemcpy(hci.data(), colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
  NSP_REQUIRE(hrp[0] == 0 && hrp[m] == nnz, "rowptr[0] must be 0 and rowptr[m] must equal nnz");
  for (int64_t i = 0; i < m; ++i) NSP_REQUIRE(hrp[i + 1] >= hrp[i], "rowptr must be non-decreasing");
  for (int64_t p = 0; p < nnz; ++p) NSP_REQUIRE(hci[p] >= 0 && hci[p] < n, "colind out of range");

  const bool re = c->prm.reorder != 0;
  const bool sym = c->prm.op == NSP_OP_SYM;
  std::vector<int32_t> rord(m), cord(n), cinv(n);
  if (re) {
    locality_order(m, n, hrp.data(), hci.data(), rord.data(), cord.data());
    if (sym) rord = cord;  // a symmetric permutation keeps A symmetric
  } else {
    std::iota(rord.begin(), rord.end(), 0);
    std::iota(cord.begin(), cord.end(), 0);
  }
  for (int64_t j = 0; j < n; ++j) cinv[cord[j]] = (int32_t)j;

  std::vector<int32_t> rp32(m + 1), ci2(std::max<int64_t>(nnz, 1)), pa(std::max<int64_t>(nnz, 1));
  std::vector<std::pair<int32_t, int32_t>> row;
  rp32[0] = 0;
  for (int64_t r = 0; r < m; ++r) {
    const int64_t i = rord[r];
    const int64_t b = hrp[i], e = hrp[i + 1];
    row.clear();
    for (int64_t p = b; p < e; ++p) row.emplace_back(cinv[hci[p]], (int32_t)p);
    if (re || sym) std::sort(row.begin(), row.end());
    const int64_t o = rp32[r];
    for (size_t t = 0; t < row.size(); ++t) {
      ci2[o + t] = row[t].first;
      pa[o + t] = row[t].second;
    }
    rp32[r + 1] = (int32_t)(o + (int64_t)row.size());
  }
  std::vector<int32_t> rpt(n + 1, 0), cit(std::max<int64_t>(nnz, 1)), pt(std::max<int64_t>(nnz, 1));
  for (int64_t p = 0; p < nnz; ++p) rpt[ci2[p] + 1]++;
  for (int64_t j = 0; j < n; ++j) rpt[j + 1] += rpt[j];
  {
    std::vector<int32_t> next(rpt.begin(), rpt.end() - 1);
    for (int64_t r = 0; r < m; ++r)
      for (int64_t p = rp32[r]; p < rp32[r + 1]; ++p) {
        const int32_t q = next[ci2[p]]++;
        cit[q] = (int32_t)r;
        pt[q] = (int32_t)p;
      }
  }
  const size_t nz = (size_t)std::max<int64_t>(nnz, 1);
  c->rowptr32.alloc(sizeof(int32_t) * (m + 1));
  c->colindA.alloc(sizeof(int32_t) * nz);
  c->permA.alloc(sizeof(int32_t) * nz);
  c->valsA.alloc(sizeof(double) * nz);
  c->colperm.alloc(sizeof(int32_t) * n);
  c->rowptrT.alloc(sizeof(int32_t) * (n + 1));
  c->colindT.alloc(sizeof(int32_t) * nz);
  c->permT.alloc(sizeof(int32_t) * nz);
  c->valsT.alloc(sizeof(double) * nz);
  NSP_HIP(hipMemcpy(c->rowptr32.p, rp32.data(), sizeof(int32_t) * (m + 1), hipMemcpyHostToDevice));
  NSP_HIP(hipMemcpy(c->colperm.p, cord.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
  NSP_HIP(hipMemcpy(c->rowptrT.p, rpt.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice));
  if (nnz) {
    NSP_HIP(hipMemcpy(c->colindA.p, ci2.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
    NSP_HIP(hipMemcpy(c->permA.p, pa.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
    NSP_HIP(hipMemcpy(c->colindT.p, cit.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
    NSP_HIP(hipMemcpy(c->permT.p, pt.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
    k_gather_vals<<<nblocks(nnz, kThreads), kThreads, 0, c->stream>>>(
        nnz, c->permA.as<int32_t>(), vals, c->valsA.as<double>());
    k_gather_vals<<<nblocks(nnz, kThreads), kThreads, 0, c->stream>>>(
        nnz, c->permT.as<int32_t>(), c->valsA.as<double>(), c->valsT.as<double>());
    NSP_HIP(hipGetLastError());
  }
  if (nnz >= kStreamMinNnz) {
    // nonzeros per row block: the LDS capacity, or less for smaller matrices so
    // that there are about 2048 row blocks to spread over the chip
    const int d = c->prm.d;
    int tile = 64;
    while (tile < stream_tile(d) && (int64_t)tile * 2048 < nnz) tile *= 2;
    const std::vector<int32_t> ba = stream_blocks(rp32, m, tile), bt = stream_blocks(rpt, n, tile);
    c->rblkA.alloc(sizeof(int32_t) * ba.size());
    c->rblkT.alloc(sizeof(int32_t) * bt.size());
    NSP_HIP(hipMemcpy(c->rblkA.p, ba.data(), sizeof(int32_t) * ba.size(), hipMemcpyHostToDevice));
    NSP_HIP(hipMemcpy(c->rblkT.p, bt.data(), sizeof(int32_t) * bt.size(), hipMemcpyHostToDevice));
    c->A.rblk = c->rblkA.as<int32_t>();
    c->A.nrb = (int)ba.size() - 1;
    c->A.rblk_d = d;
    c->AT.rblk = c->rblkT.as<int32_t>();
    c->AT.nrb = (int)bt.size() - 1;
    c->AT.rblk_d = d;
  }
  if (sym) {
    // the stored A must equal its stored transpose: same pattern here, same
    // values checked on the device below
    NSP_REQUIRE(rp32 == rpt && std::equal(ci2.begin(), ci2.begin() + nnz, cit.begin()),
                "op = NSP_OP_SYM needs a structurally symmetric A");
    check_symmetric_values(c);
  }
  c->sym = sym;
  c->reordered = re;
  c->A.rows = m; c->A.cols = n; c->A.nnz = nnz;
  c->A.rowptr = c->rowptr32.as<int32_t>();
  c->A.colind = c->colindA.as<int32_t>();
  c->A.val = c->valsA.as<double>();
  c->A.lpr = choose_lpr(m, nnz);
  c->AT.rows = n; c->AT.cols = m; c->AT.nnz = nnz;
  c->AT.rowptr = c->rowptrT.as<int32_t>();
  c->AT.colind = c->colindT.as<int32_t>();
  c->AT.val = c->valsT.as<double>();
  c->AT.lpr = choose_lpr(n, nnz);
  if (c->prm.prec == NSP_PREC_MIXED && nnz) {
    c->vals32.alloc(sizeof(float) * nnz);
    c->valsT32.alloc(sizeof(float) * nnz);
    c->A.val32 = c->vals32.as<float>();
    c->AT.val32 = c->valsT32.as<float>();
    copy_f32(c);
  }
  NSP_HIP(hipStreamSynchronize(c->stream));
}

// Stored A and A^T must hold equal mirrored values (symmetric form); the
// patterns were compared on the host in prepare_matrix.
void check_symmetric_values(nsp_ctx* c) {
  const int64_t nnz = c->nnz;
  if (!nnz) return;
  DBuf flag;
  flag.alloc(sizeof(int));
  NSP_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), c->stream));
  k_values_differ<<<nblocks(nnz, kThreads), kThreads, 0, c->stream>>>(
      nnz, c->valsA.as<double>(), c->valsT.as<double>(), flag.as<int>());
  NSP_HIP(hipGetLastError());
  int hflag = 0;
  NSP_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  NSP_HIP(hipStreamSynchronize(c->stream));
  NSP_REQUIRE(hflag == 0, "op = NSP_OP_SYM needs A(i,j) == A(j,i) for every stored entry");
}

// FP32 copies of the stored values (mixed precision)
void copy_f32(nsp_ctx* c) {
  const int64_t nnz = c->nnz;
  if (!nnz || !c->A.val32) return;
  k_to_f32<<<nblocks(nnz, kThreads), kThreads, 0, c->stream>>>(nnz, c->A.val, c->vals32.as<float>());
  k_to_f32<<<nblocks(nnz, kThreads), kThreads, 0, c->stream>>>(nnz, c->AT.val, c->valsT32.as<float>());
  NSP_HIP(hipGetLastError());
}

// New values for the same pattern (caller's CSR order): through the value
// permutations of prepare_matrix into the stored A and A^T, then the same
// checks, FP32 copies, norms and preconditioning as at init.
void refresh_values(nsp_ctx* c, const double* vals) {
  const int64_t nnz = c->nnz;
  if (nnz) {
    k_gather_vals<<<nblocks(nnz, kThreads), kThreads, 0, c->stream>>>(
        nnz, c->permA.as<int32_t>(), vals, c->valsA.as<double>());
    k_gather_vals<<<nblocks(nnz, kThreads), kThreads, 0, c->stream>>>(
        nnz, c->permT.as<int32_t>(), c->valsA.as<double>(), c->valsT.as<double>());
    NSP_HIP(hipGetLastError());
  }
  if (c->sym) check_symmetric_values(c);
  copy_f32(c);
  c->precond = false;
  c->precond_ic = false;
  c->ic.norm_bound = 0.0;
  matrix_norms(c);
  precondition(c);
  if (c->precond) matrix_norms(c);
  NSP_HIP(hipStreamSynchronize(c->stream));
}

__global__ void k_rows_copy(int64_t n, int ncols, const int32_t* __restrict__ idx, bool scatter,
                            const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                            int64_t ldd) {
  const int64_t total = n * ncols;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = t % n, j = t / n;
    const int64_t k = idx ? idx[i] : i;
    if (scatter) dst[k + j * ldd] = src[i + j * lds];
    else dst[i + j * ldd] = src[k + j * lds];
  }
}

void gather_rows(nsp_ctx* c, int64_t n, int ncols, const int32_t* idx, const double* src,
                 int64_t lds, double* dst, int64_t ldd) {
  if (n <= 0 || ncols <= 0) return;
  const int g = (int)std::min<int64_t>(nblocks(n * ncols, kThreads), 4096);
  k_rows_copy<<<g, kThreads, 0, c->stream>>>(n, ncols, idx, false, src, lds, dst, ldd);
  NSP_HIP(hipGetLastError());
}

void scatter_rows(nsp_ctx* c, int64_t n, int ncols, const int32_t* idx, const double* src,
                  int64_t lds, double* dst, int64_t ldd) {
  if (n <= 0 || ncols <= 0) return;
  const int g = (int)std::min<int64_t>(nblocks(n * ncols, kThreads), 4096);
  k_rows_copy<<<g, kThreads, 0, c->stream>>>(n, ncols, idx, true, src, lds, dst, ldd);
  NSP_HIP(hipGetLastError());
}

__global__ void k_scatter_vals(int64_t nnz, const int32_t* __restrict__ perm,
                               const double* __restrict__ src, double* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nnz) dst[perm[i]] = src[i];
}

void scatter_vals(nsp_ctx* c, const double* src, double* dst) {
  if (c->nnz == 0) return;
  k_scatter_vals<<<nblocks(c->nnz, kThreads), kThreads, 0, c->stream>>>(
      c->nnz, c->permA.as<int32_t>(), src, dst);
  NSP_HIP(hipGetLastError());
}

// D and Omega are given (or drawn) in the caller's order of the unknowns and
// stored in the library's order.
void init_random(nsp_ctx* c, const double* D, const double* Omega) {
  const int64_t n = c->n;
  const int d = c->prm.d;
  const int32_t* cp = c->colperm.as<int32_t>();
  c->Dv.alloc(sizeof(double) * n);
  c->omega.alloc(sizeof(double) * n * d);
  DBuf draw;
  if (!D || !Omega) draw.alloc(sizeof(double) * n * d);
  if (D) {
    gather_rows(c, n, 1, cp, D, n, c->Dv.as<double>(), n);
  } else {
    k_philox_uniform<<<nblocks(n, kThreads), kThreads, 0, c->stream>>>(n, c->prm.seed, 0u,
                                                                        draw.as<double>());
    NSP_HIP(hipGetLastError());
    gather_rows(c, n, 1, cp, draw.as<double>(), n, c->Dv.as<double>(), n);
  }
  if (Omega) {
    gather_rows(c, n, d, cp, Omega, n, c->omega.as<double>(), n);
  } else {
    for (int j = 0; j < d; ++j)
      k_philox_normal<<<nblocks(n, kThreads), kThreads, 0, c->stream>>>(
          n, c->prm.seed, (uint32_t)(j + 1), draw.as<double>() + (int64_t)j * n);
    NSP_HIP(hipGetLastError());
    gather_rows(c, n, d, cp, draw.as<double>(), n, c->omega.as<double>(), n);
  }
  NSP_HIP(hipGetLastError());
  std::vector<double> hd(n);
  NSP_HIP(hipMemcpyAsync(hd.data(), c->Dv.p, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  NSP_HIP(hipStreamSynchronize(c->stream));
  double mx = 0.0;
  for (double v : hd) {
    NSP_REQUIRE(std::isfinite(v) && v >= 0.0, "D must be finite and non-negative");
    mx = std::max(mx, v);
  }
  c->maxD = mx;
}

// ||A||_F, ||A||_1 ||A||_inf; also rejects non-finite values
double matrix_norms(nsp_ctx* c) {
  const int64_t m = c->m, n = c->n;
  DBuf rabs, rsq, cabs, flag;
  rabs.alloc(sizeof(double) * m);
  rsq.alloc(sizeof(double) * m);
  cabs.alloc(sizeof(double) * n);
  flag.alloc(sizeof(int));
  NSP_HIP(hipMemsetAsync(flag.p, 0, sizeof(int), c->stream));
  k_row_abs_sums<<<nblocks(m, kThreads), kThreads, 0, c->stream>>>(m, c->A.rowptr, c->A.val,
                                                                    rabs.as<double>(), rsq.as<double>(),
                                                                    flag.as<int>());
  k_row_abs_sums<<<nblocks(n, kThreads), kThreads, 0, c->stream>>>(n, c->AT.rowptr, c->AT.val,
                                                                    cabs.as<double>(), nullptr,
                                                                    flag.as<int>());
  NSP_HIP(hipGetLastError());
  std::vector<double> hr(m), hq(m), hc(n);
  int hflag = 0;
  NSP_HIP(hipMemcpyAsync(hr.data(), rabs.p, sizeof(double) * m, hipMemcpyDeviceToHost, c->stream));
  NSP_HIP(hipMemcpyAsync(hq.data(), rsq.p, sizeof(double) * m, hipMemcpyDeviceToHost, c->stream));
  NSP_HIP(hipMemcpyAsync(hc.data(), cabs.p, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  NSP_HIP(hipMemcpyAsync(&hflag, flag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  NSP_HIP(hipStreamSynchronize(c->stream));
  if (hflag) throw Error(NSP_ERR_NONFINITE, "A contains a non-finite value");
  double fro = 0.0, ninf = 0.0, n1 = 0.0;
  for (int64_t i = 0; i < m; ++i) { fro += hq[i]; ninf = std::max(ninf, hr[i]); }
  for (int64_t j = 0; j < n; ++j) n1 = std::max(n1, hc[j]);
  c->normA_fro = std::sqrt(fro);
  c->normA1_inf = n1 * ninf;
  c->normA_inf = ninf;
  return c->normA_fro;
}

// ---------------------------------------------------------------------------
// Outer preconditioning with a diagonal P_R = diag(p) (Sec. 4.4): the Cholesky
// factor of M = A^T A (normal form) or M = A (symmetric form) with every
// off-diagonal entry dropped, p_j = sqrt(M_jj), and p_j = 1 where M_jj is not
// positive.  Row j of the stored A^T is column j of A.
// ---------------------------------------------------------------------------
__global__ void k_jacobi_diag(int64_t n, const int32_t* __restrict__ rp,
                              const int32_t* __restrict__ ci, const double* __restrict__ val,
                              bool sym, double* __restrict__ p) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int32_t q = rp[j]; q < rp[j + 1]; ++q) {
    if (sym) {
      if (ci[q] == j) s += val[q];
    } else {
      s = fma(val[q], val[q], s);
    }
  }
  p[j] = s > 0.0 ? sqrt(s) : 1.0;
}

// val(i, j) /= p[j] (cols) and /= p[i] (rows) over a CSR
__global__ void k_scale_vals(int64_t rows, const int32_t* __restrict__ rp,
                             const int32_t* __restrict__ ci, const double* __restrict__ p,
                             bool by_row, bool by_col, double* __restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  const double pr = by_row ? p[i] : 1.0;
  for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
    double v = val[q] / pr;
    if (by_col) v /= p[ci[q]];
    val[q] = v;
  }
}

void precondition(nsp_ctx* c) {
  c->normA_fro_orig = c->normA_fro;
  if (c->prm.precond == NSP_PRECOND_NONE) return;
  if (c->prm.precond == NSP_PRECOND_IC) {
    ic_setup(c);
    return;
  }
  const int64_t m = c->m, n = c->n, nnz = c->nnz;
  c->pdiag.alloc(sizeof(double) * n);
  double* p = c->pdiag.as<double>();
  k_jacobi_diag<<<nblocks(n, kThreads), kThreads, 0, c->stream>>>(n, c->AT.rowptr, c->AT.colind,
                                                                   c->AT.val, c->sym, p);
  NSP_HIP(hipGetLastError());
  if (nnz) {
    // A P^{-T}: columns of A, rows of A^T; P^{-1} A P^{-T}: both sides
    k_scale_vals<<<nblocks(m, kThreads), kThreads, 0, c->stream>>>(m, c->A.rowptr, c->A.colind, p,
                                                                    c->sym, true, c->valsA.as<double>());
    k_scale_vals<<<nblocks(n, kThreads), kThreads, 0, c->stream>>>(n, c->AT.rowptr, c->AT.colind, p,
                                                                    true, c->sym, c->valsT.as<double>());
    NSP_HIP(hipGetLastError());
    copy_f32(c);
  }
  c->precond = true;
  NSP_HIP(hipStreamSynchronize(c->stream));
}

// Y = B X for column-major FP64 X, Y (apply_op).  Columns go through the
// row-interleaved path in chunks of at most 8.
void apply_b_chunks(nsp_ctx* c, const double* X, int64_t ldx, double* Y, int64_t ldy, int ncols,
                    int wmax, double* xc, double* xr, double* yr, double* zr) {
  const int64_t n = c->n;
  const int32_t* cp = c->colperm.as<int32_t>();
  for (int j0 = 0; j0 < ncols;) {
    const int left = std::min(ncols - j0, wmax);
    const int w = left >= 8 ? 8 : left >= 4 ? 4 : left >= 2 ? 2 : 1;
    gather_rows(c, n, w, cp, X + (int64_t)j0 * ldx, ldx, xc, n);
    colmajor_to_rows(c, n, w, xc, n, xr);
    if (c->precond_ic) {
      // B_R X = L^{-1} (A^T A or A) L^{-T} X + eps D X
      NSP_HIP(hipMemcpyAsync(zr, xr, sizeof(double) * n * w, hipMemcpyDeviceToDevice, c->stream));
      ic_solve_lt<double>(c, w, zr);
      double* res = zr;
      if (!c->sym) {
        spmm_block<double>(c, c->A, w, zr, yr);
        spmm_block<double>(c, c->AT, w, yr, zr);
      } else {
        spmm_block<double>(c, c->A, w, zr, yr);
        res = yr;
      }
      ic_solve_l<double>(c, w, res);
      add_eps_dx(c, w, xr, res);
      rows_to_colmajor(c, n, w, res, xc, n);
      scatter_rows(c, n, w, cp, xc, n, Y + (int64_t)j0 * ldy, ldy);
      j0 += w;
      continue;
    }
    // B X: A^T (A X) + eps D X, or A X + eps D X for the symmetric form (the
    // stored A^T is A itself then)
    const double* yin = xr;
    if (!c->sym) {
      spmm_block<double>(c, c->A, w, xr, yr);
      yin = yr;
    }
    spmmT_step<double>(c, w, yin, xr, nullptr, nullptr, zr, nullptr);
    rows_to_colmajor(c, n, w, zr, xc, n);
    scatter_rows(c, n, w, cp, xc, n, Y + (int64_t)j0 * ldy, ldy);
    j0 += w;
  }
  NSP_HIP(hipStreamSynchronize(c->stream));
}

void apply_b_colmajor(nsp_ctx* c, const double* X, int64_t ldx, double* Y, int64_t ldy, int ncols) {
  const int64_t m = c->m, n = c->n;
  DBuf xc, xr, yr, zr;
  xc.alloc(sizeof(double) * n * kMaxD);
  xr.alloc(sizeof(double) * n * kMaxD);
  yr.alloc(sizeof(double) * m * kMaxD);
  zr.alloc(sizeof(double) * n * kMaxD);
  apply_b_chunks(c, X, ldx, Y, ldy, ncols, kMaxD, xc.as<double>(), xr.as<double>(), yr.as<double>(),
                 zr.as<double>());
}

}  // namespace nsp
