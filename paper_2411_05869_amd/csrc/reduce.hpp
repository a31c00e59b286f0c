// Deterministic reductions of float64 values over a grid of 256-thread blocks.
//
// A block first adds its threads' values with a fixed shuffle tree and writes
// one partial per block.  The partials are then added in a fixed order (thread
// t takes partials t, t + 256, ... and a fixed tree combines the threads), so
// every result is bitwise reproducible whatever the scheduling.  The final pass
// runs in a later kernel: either a one-block kernel, or redundantly in every
// block of the kernel that consumes the result (for a few hundred partials
// this costs less than a launch).
#pragma once

#include "device.hpp"

namespace gps {

constexpr int kRedThreads = 256;

// Block sum of v[0..NV) into out[blockIdx.x * NV + i].
template <int NV>
__device__ __forceinline__ void block_sum_store(double (&v)[NV], double* __restrict__ out) {
  __shared__ double sh[NV][kRedThreads / kWave];
  const int w = threadIdx.x / kWave;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double x = v[i];
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) x += __shfl_xor(x, off, kWave);
    if (lane_id() == 0) sh[i][w] = x;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double s = 0;
#pragma unroll
    for (int j = 0; j < kRedThreads / kWave; ++j) s += sh[threadIdx.x][j];
    out[blockIdx.x * NV + threadIdx.x] = s;
  }
}

// Sums part[b * NV + i] over b in a fixed order (partials written by an earlier
// launch); the result is returned to every thread of the block.
// A thread loads four of its strided partials at once and adds them in the
// order of a plain strided loop.
template <int NV>
__device__ __forceinline__ void reduce_partials(const double* __restrict__ part, int nb, double* __restrict__ res) {
  constexpr int kBatch = 4;
  __shared__ double sh[NV][kRedThreads];
  double s[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) s[i] = 0;
  for (int b0 = threadIdx.x; b0 < nb; b0 += kBatch * kRedThreads) {
    double v[kBatch][NV];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int b = b0 + u * kRedThreads;
#pragma unroll
      for (int i = 0; i < NV; ++i) v[u][i] = b < nb ? part[b * NV + i] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
      if (b0 + u * kRedThreads < nb)
#pragma unroll
        for (int i = 0; i < NV; ++i) s[i] += v[u][i];
  }
#pragma unroll
  for (int i = 0; i < NV; ++i) sh[i][threadIdx.x] = s[i];
  __syncthreads();
  for (int st = kRedThreads / 2; st > 0; st >>= 1) {
    if (threadIdx.x < st)
#pragma unroll
      for (int i = 0; i < NV; ++i) sh[i][threadIdx.x] += sh[i][threadIdx.x + st];
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < NV; ++i) res[i] = sh[i][0];
  __syncthreads();
}

}  // namespace gps
