// Device helpers shared by the kernel sources: fixed-order block reductions and the
// block-to-XCD remap.
//
// Wave size is 64.  Every reduction is a fixed tree: per-thread FP64 sums, a wave
// butterfly (__shfl_xor), a fixed-order sum of the waves of a block into one partial
// per block, then a fixed-order strided sum of the partials in a later kernel, so
// results are bitwise reproducible run to run.
#pragma once
#include <hip/hip_runtime.h>

#include <stdint.h>

namespace rmh {

// ------------------------------------------------------------------------------------------
// reductions

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// Sum over the block (any multiple of 64 threads up to 1024); result valid in thread 0.
template <int NQ>
__device__ __forceinline__ void block_sum(double (&v)[NQ], double (*lds)[16]) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double w = wave_sum(v[q]);
    if (lane == 0) lds[q][wid] = w;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      double s = 0.0;
      for (int i = 0; i < nw; ++i) s += lds[q][i];
      v[q] = s;
    }
  }
  __syncthreads();  // lds may be reused by the caller right away
}

// Strided fixed-order sum of n values by a whole block; result in thread 0.
// Fixed-order sum of p[0, n): four independent loads in flight per thread, then the block tree.
__device__ __forceinline__ double block_sum_array(const double* p, int32_t n, double (*lds)[16]) {
  const int32_t B = blockDim.x;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int32_t i = threadIdx.x;
  for (; i + 3 * B < n; i += 4 * B) {
    a0 += p[i];
    a1 += p[i + B];
    a2 += p[i + 2 * B];
    a3 += p[i + 3 * B];
  }
  for (; i < n; i += B) a0 += p[i];
  double v[1] = {(a0 + a1) + (a2 + a3)};
  block_sum<1>(v, lds);
  return v[0];
}

__device__ __forceinline__ int32_t remap_block(int32_t b, int32_t G, int32_t xcd) {
  // Consecutive hardware block ids go round-robin over the 8 XCDs; give each XCD a
  // contiguous range of the lattice so neighbouring sites share its L2.
  if (xcd && (G & 7) == 0) return (b & 7) * (G >> 3) + (b >> 3);
  return b;
}

}  // namespace rmh
