// Device helpers: wavefront / block reductions and fixed-order sums of
// per-block partials written by an earlier kernel.
#pragma once

#include <hip/hip_runtime.h>

namespace nsp {

constexpr int kWave = 64;

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

template <typename T, int W>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  return v;
}

// Sums of X(:, i) P(:, j) over the rows of two row-interleaved n x 8 blocks
// on the matrix cores (v_mfma_f64_16x16x4f64), for the 8 x 8 Gram-type
// matrices of block size 8.  A wave takes 8 consecutive rows at a time, lane l
// holding row g8_row(l) and column l % 8 of them (the 64 values are read in
// one coalesced pass).  Lane l gives A(l % 16, l / 16) and B(l / 16, l % 16),
// so with X's value as A and P's as B the product's diagonal 8 x 8 blocks are
// the sums over rows 0..3 (D(i, j)) and rows 4..7 (D(8 + i, 8 + j)); the
// off-diagonal blocks mix rows and are dropped.  Register v of lane l holds
// D(l / 16 + 4 v, l % 16) (layout checked on the device).
typedef double g8_acc __attribute__((ext_vector_type(4)));
__device__ __forceinline__ int g8_row(int lane) { return 4 * ((lane >> 3) & 1) + (lane >> 4); }
__device__ __forceinline__ int g8_off(int lane) { return g8_row(lane) * 8 + (lane & 7); }
__device__ __forceinline__ g8_acc g8_step(double xv, double pv, g8_acc acc) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(xv, pv, acc, 0, 0, 0);
}
// out[i * 8 + j] = the block's sum: the two diagonal blocks of every wave, the
// waves in order.  tile: shared, (blockDim.x / 64) * 256 doubles.  Every thread
// of the block calls it.
__device__ __forceinline__ void g8_finish(const g8_acc& acc, double* tile, double* out) {
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
  for (int v = 0; v < 4; ++v) tile[wid * 256 + (lane / 16 + 4 * v) * 16 + lane % 16] = acc[v];
  __syncthreads();
  if (threadIdx.x < 64) {
    const int i = threadIdx.x / 8, j = threadIdx.x % 8;
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += tile[w * 256 + i * 16 + j] + tile[w * 256 + (8 + i) * 16 + 8 + j];
    out[threadIdx.x] = s;
  }
}

// Sum NV per-thread values over the block; the result is valid in thread 0.
// smem must hold (blockDim.x / 64) * NV doubles.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* smem) {
  const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) smem[wid * NV + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += smem[w * NV + i];
      v[i] = s;
    }
  }
  __syncthreads();
}

// Fixed-order sum of per-block partials, done cooperatively by one block:
// res[v] = sum_b part[b * NV + v] for v < NV.  Every thread of the block must
// call it; res (shared, NV doubles) is valid in all threads afterwards.  smem
// must hold blockDim.x doubles.  The partials come from an earlier kernel on
// the same stream, so no fence or atomic is involved.
template <int NV>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int nparts,
                                                double* res, double* smem) {
  static_assert(NV <= 256, "at most 256 values");
  const int t = threadIdx.x;
  const int groups = (int)blockDim.x / NV > 0 ? (int)blockDim.x / NV : 1;
  double s = 0.0;
  if (t < groups * NV) {
    const int v = t % NV, g = t / NV;
    // eight independent partial sums keep eight loads in flight per thread
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int b = g;
    for (; b + 7 * groups < nparts; b += 8 * groups) {
#pragma unroll
      for (int u = 0; u < 8; ++u) acc[u] += part[(size_t)(b + u * groups) * NV + v];
    }
    for (int u = 0; b < nparts; b += groups, ++u) acc[u & 7] += part[(size_t)b * NV + v];
    s = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
  }
  smem[t] = s;
  __syncthreads();
  if ((groups & (groups - 1)) == 0) {
    // groups a power of two (block sizes and NV are): a fixed-order tree in LDS
    for (int h = groups / 2; h > 0; h >>= 1) {
      if (t < h * NV) smem[t] += smem[t + h * NV];
      __syncthreads();
    }
    if (t < NV) res[t] = smem[t];
  } else if (t < NV) {
    double r = 0.0;
    for (int g = 0; g < groups; ++g) r += smem[g * NV + t];
    res[t] = r;
  }
  __syncthreads();
}

}  // namespace nsp
