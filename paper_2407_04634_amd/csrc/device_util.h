// Device helpers: wavefront / block reductions and the "last block finishes"
// grid reduction used by kernels that end in a small reduced result.
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

// Grid reduction epilogue.  Every block calls this with its block sums in
// thread 0 (after block_sum).  The block that arrives last sums the partials
// of all blocks in block order (deterministic) into ``out`` (NV doubles),
// resets the counter, and returns true in all its threads; the other blocks
// return false.  Partials are written with device-scope release semantics and
// read after an acquire, so the last block sees every block's partial even
// when blocks ran on different XCDs.
template <int NV>
__device__ bool grid_sum_last(const double (&v)[NV], double* partials, unsigned* counter,
                              double* out, double* smem) {
  static_assert(NV <= 256, "grid_sum_last handles at most 256 values");
  __shared__ int am_last;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) partials[(size_t)blockIdx.x * NV + i] = v[i];
    __threadfence();
    unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    am_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!am_last) return false;
  __threadfence();
  // thread t sums value (t % NV) over blocks b = t / NV, t / NV + G, ... (G = groups)
  const int groups = blockDim.x / NV > 0 ? blockDim.x / NV : 1;
  const int t = threadIdx.x;
  double s = 0.0;
  if (t < groups * NV) {
    const int i = t % NV, g = t / NV;
    for (unsigned b = g; b < gridDim.x; b += groups)
      s += partials[(size_t)b * NV + i];
  }
  smem[t] = s;
  __syncthreads();
  if (t < NV) {
    double r = 0.0;
    for (int g = 0; g < groups; ++g) r += smem[g * NV + t];
    out[t] = r;
  }
  if (t == 0) __hip_atomic_store(counter, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  return true;
}

}  // namespace nsp
