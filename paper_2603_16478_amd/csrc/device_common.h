// Device helpers shared by the HIP kernels of the adjoint library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace adj {

constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Sum over groups of `width` consecutive lanes (width a power of two <= 64).
template <int width>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = width / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}

// Block-wide sum for blockDim.x <= 1024; result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* lds /* >= 16 */) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (kWave - 1), wid = threadIdx.x / kWave;
  if (lane == 0) lds[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + kWave - 1) / kWave;
    for (int i = 0; i < nw; ++i) r += lds[i];
  }
  __syncthreads();
  return r;
}

// "Last block done" handshake: every block has written its partial results;
// returns true in exactly one block (the last to arrive), after an acquire
// fence, so it may read all partials.  Resets the counter for the next use.
__device__ __forceinline__ bool last_block(unsigned* counter, bool* flag_lds) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned prev = atomicAdd(counter, 1u);
    *flag_lds = (prev == gridDim.x - 1);
  }
  __syncthreads();
  bool last = *flag_lds;
  if (last) {
    __threadfence();
    if (threadIdx.x == 0) *counter = 0u;
  }
  return last;
}

// res[i] = sum_b P[b * ld + i] for i < cnt (cnt <= 256), fixed order; all
// 256 threads of the block take part; tmp: 256 doubles of LDS.
__device__ __forceinline__ void sum_partials(const double* __restrict__ P, int nb, int ld, int cnt,
                                             double* __restrict__ res, double* __restrict__ tmp) {
  int G = 1;
  while (2 * G * cnt <= 256) G *= 2;  // threads per entry (power of two)
  const int t = threadIdx.x, i = t / G, g = t % G;
  double a = 0.0;
  if (i < cnt)
    for (int b = g; b < nb; b += G) a += P[(size_t)b * ld + i];
  tmp[t] = a;
  __syncthreads();
  for (int h = G / 2; h > 0; h >>= 1) {
    if (g < h && i < cnt) tmp[t] += tmp[t + h];
    __syncthreads();
  }
  if (g == 0 && i < cnt) res[i] = tmp[t];
  __syncthreads();
}

}  // namespace adj
