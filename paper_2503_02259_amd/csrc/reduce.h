// Deterministic column reductions over n×k row-major blocks (k ≤ 64).
//
// A grid of G blocks covers the rows in fixed chunks; each block writes its
// 64 per-column partial sums, and the last block to finish (ticket counter)
// adds the G partials in block order.  The result does not depend on
// scheduling, so repeated runs and runs inside a batch are bitwise equal.
#pragma once

#include "common.h"

namespace higp {

constexpr int kRedThreads = 256;  // 4 row lanes × 64 columns
constexpr int kRedMaxBlocks = 1024;

struct RedGrid {
  int blocks;
  int64_t chunk;  // rows per block (multiple of 4)
};

inline RedGrid red_grid(int64_t n) {
  int64_t g = (n + 127) / 128;
  if (g > kRedMaxBlocks) g = kRedMaxBlocks;
  if (g < 1) g = 1;
  int64_t chunk = (n + g - 1) / g;
  chunk = (chunk + 3) / 4 * 4;
  g = (n + chunk - 1) / chunk;
  if (g < 1) g = 1;
  return RedGrid{(int)g, chunk};
}

// Block-level: reduce `v` (this thread's partial for column tid&63) over the
// 4 row lanes; writes work[blockIdx.x*64 + c].  Then the last block sums all
// partials in order and calls fin(c, total) for c < k (threads 0..k-1).
// Must be called by all threads of the block.  `sh` is 256 doubles of LDS.
// Returns true (in every thread) only in the block that ran fin; the caller
// must not use __syncthreads() afterwards in the other blocks.
template <typename Fin>
__device__ __forceinline__ bool block_colsum_finish(double v, int k, double* work,
                                                    unsigned* counter, double* sh, Fin fin) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  if (tid < 64) {
    const double s = ((sh[tid] + sh[tid + 64]) + sh[tid + 128]) + sh[tid + 192];
    work[(int64_t)blockIdx.x * 64 + tid] = s;
  }
  __threadfence();
  __syncthreads();
  __shared__ unsigned ticket;
  if (tid == 0) ticket = atomicAdd(counter, 1u);
  __syncthreads();
  if (ticket != gridDim.x - 1) return false;
  __threadfence();
  if (tid < k) {
    double s = 0.0;
    for (unsigned b = 0; b < gridDim.x; ++b)
      s += __hip_atomic_load(&work[(int64_t)b * 64 + tid], __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    fin(tid, s);
  }
  if (tid == 0) *counter = 0u;
  __syncthreads();
  return true;
}

template <typename T>
__device__ __forceinline__ double ld(const T* p, int64_t i) {
  return (double)p[i];
}

}  // namespace higp
