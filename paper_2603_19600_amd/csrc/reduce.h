// Deterministic FP64 reductions: wave64 shuffle sums, a workgroup sum per
// block into a fixed-size partial array, and a single-workgroup final sum in
// a fixed order, so results do not depend on scheduling.
#pragma once

#include "common.h"

namespace fx {

constexpr int kRedBlocks = 1024;   // partial sums per reduction

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sums v[j] over the workgroup (kBlock threads); thread 0 writes out_slot[j * stride].
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *out_slot, int64_t stride) {
  __shared__ double red[NV][kBlock / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const double w = wave_sum(v[j]);
    if (lane == 0) red[j][wid] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      double t = 0.0;
      for (int w = 0; w < kBlock / 64; ++w) t += red[j][w];
      out_slot[j * stride] = t;
    }
  }
}

// Single workgroup of kBlock threads: out[j] = sum of partial[j * count + 0 .. count-1].
template <int NV>
__device__ __forceinline__ void final_sum(const double *__restrict__ partial, double (&out)[NV],
                                          int count = kRedBlocks) {
  __shared__ double red[NV][kBlock];
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    double t = 0.0;
    for (int i = threadIdx.x; i < count; i += kBlock) t += partial[(int64_t)j * count + i];
    red[j][threadIdx.x] = t;
  }
  __syncthreads();
  for (int w = kBlock / 2; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
#pragma unroll
      for (int j = 0; j < NV; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < NV; ++j) out[j] = red[j][0];
}

}  // namespace fx
