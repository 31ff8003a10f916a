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
