// Deterministic column reductions over n×k row-major blocks (k ≤ 64).
//
// A grid of G blocks covers the rows in fixed chunks.  Inside a block the 256
// threads form cw = 2^⌈log₂k⌉ column lanes × 256/cw row lanes (so a single
// column still uses every thread); the row lanes of a wavefront are summed by
// a fixed butterfly of lane shuffles, the four wavefronts' sums are added in
// order through LDS, each block writes its per-column partial sums, and the
// last block to finish (ticket counter) adds the G partials in block order.  The result depends
// only on n and k, not on scheduling, so repeated runs and runs inside a
// batch are bitwise equal.
#pragma once

#include "common.h"

namespace higp {

constexpr int kRedThreads = 256;  // 4 row lanes × 64 columns
// At most 256 blocks: the last block adds G partials per column and every
// block takes a ticket, so the tail grows with G.  At n = 1e5, k = 33 the
// PCG update took 150 µs with up to 1024 blocks and 74 µs with 256 (128:
// 137 µs, too few loads in flight).
constexpr int kRedMaxBlocks = 256;
constexpr int kRowBatch = 4;       // rows whose loads a thread keeps in flight

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

// Thread → (column lane c, first row r0, row stride) for k ≤ 64 columns.
struct ColLanes {
  int c, r0, step, lg;
};

__device__ __forceinline__ ColLanes col_lanes(int k) {
  const int lg = k <= 1 ? 0 : 32 - __clz(k - 1);  // cw = 2^lg ≥ k
  ColLanes L;
  L.lg = lg;
  L.c = (int)threadIdx.x & ((1 << lg) - 1);
  L.r0 = (int)threadIdx.x >> lg;
  L.step = kRedThreads >> lg;
  return L;
}

// Block-level: sum `v` (this thread's partial for its column lane) over the
// row lanes; on return sh[c] (c < cw) holds column c's block sum.  Within a
// wavefront the lanes of one column differ in lane bits lg..5, summed by an
// XOR butterfly (fixed order); then the four wavefronts' sums are added in
// wavefront order.  Must be called by all threads.  `sh` is 256 doubles of
// LDS.
__device__ __forceinline__ void block_colsum(double v, int k, double* sh) {
  const ColLanes L = col_lanes(k);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  for (int m = 32; m >= (1 << L.lg); m >>= 1) v += __shfl_xor(v, m);
  __syncthreads();  // sh may still be read by a previous call
  if (lane < (1 << L.lg)) sh[wave * 64 + lane] = v;
  __syncthreads();
  if (tid < (1 << L.lg)) sh[tid] = ((sh[tid] + sh[64 + tid]) + sh[128 + tid]) + sh[192 + tid];
  __syncthreads();
}

// Block sums as above, written to work[blockIdx.x*64 + c]; then the last
// block sums all partials in a fixed order and calls fin(c, total) for c < k
// (threads 0..k-1).  Must be called by all threads of the block.  Returns
// true (in every thread) only in the block that ran fin; the caller must not
// use __syncthreads() afterwards in the other blocks.
template <typename Fin>
__device__ __forceinline__ bool block_colsum_finish(double v, int k, double* work,
                                                    unsigned* counter, double* sh, Fin fin) {
  const int tid = threadIdx.x;
  block_colsum(v, k, sh);
  if (tid < k) work[(int64_t)blockIdx.x * 64 + tid] = sh[tid];
  __threadfence();
  __syncthreads();
  __shared__ unsigned ticket;
  if (tid == 0) ticket = atomicAdd(counter, 1u);
  __syncthreads();
  if (ticket != gridDim.x - 1) return false;
  __threadfence();
  // Row lane r of column c adds the partials of blocks r, r + step, … in
  // order; the lanes are then combined by the fixed tree.  Eight partials are
  // loaded at a time (independent L2 round trips in flight) and added in the
  // same order.
  const ColLanes L = col_lanes(k);
  double s = 0.0;
  if (L.c < k) {
    auto part = [&](unsigned b) {
      return __hip_atomic_load(&work[(int64_t)b * 64 + L.c], __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
    };
    unsigned b = L.r0;
    for (; b + 7 * L.step < gridDim.x; b += 8 * L.step) {
      double w[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) w[u] = part(b + u * L.step);
#pragma unroll
      for (int u = 0; u < 8; ++u) s += w[u];
    }
    for (; b < gridDim.x; b += L.step) s += part(b);
  }
  block_colsum(s, k, sh);
  if (tid < k) fin(tid, sh[tid]);
  if (tid == 0) *counter = 0u;
  __syncthreads();
  return true;
}

template <typename T>
__device__ __forceinline__ double ld(const T* p, int64_t i) {
  return (double)p[i];
}

}  // namespace higp
