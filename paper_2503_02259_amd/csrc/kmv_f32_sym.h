// The symmetric-tiled FP32 MatVec unit (one pair of 1024-point blocks) and
// its finishing sum, shared by the single-problem launcher
// (kmatvec_f32_sym.hip) and the batched serving launcher
// (kmatvec_f32_batch.hip); see kmatvec_f32_sym.hip for the design.
#pragma once

#include "kmv_f32_tile.h"

namespace higp {
namespace {

constexpr int64_t kSymMinPoints = 32768;  // below: too few block pairs to fill the chip
constexpr int kSymTile = 128;
constexpr int kSymSub = 8;                     // tiles per super block
constexpr int kSymSuper = kSymTile * kSymSub;  // points per super block
constexpr int kMicro = 8;                      // micro tile edge

struct SymArgs {
  const float* Xp;  // prepared points, 4·NQ floats each; rows ≥ n are read as far sentinels
  const float* V;   // n×k; rows ≥ n are read as 0
  float* prow;      // [item][1024][k] row sums (Y_A part)
  float* pcol;      // [item][1024][k] column sums (Y_B part, A < B)
  int64_t n;        // points
  int ns;           // super blocks, ⌈n/1024⌉
};

// Whether a square FP32 MatVec of n points in d dimensions with k vectors
// takes the symmetric form: one or two vectors, d ≤ max_d (8 for one vector,
// 4 for two; the batched launch serves one vector), enough block pairs to
// fill the chip, and per-pair slots of at most 2 GiB (they grow as n²/1024).
inline bool sym_eligible(int64_t n, int d, int k, int flags, int max_d) {
  if (k > 2 || d > max_d || n < kSymMinPoints || (flags & HIGP_FLAG_NO_SYMMETRIC) != 0)
    return false;
  const int64_t ns = (n + kSymSuper - 1) / kSymSuper;
  const int64_t slot_bytes = ns * (ns + 1) / 2 * kSymSuper * k * 4;
  return 2 * slot_bytes <= (int64_t(1) << 31);
}

// Items enumerate the pairs (A, B), A ≤ B, row by row: row A holds ns − A.
__device__ __forceinline__ void item_pair(int idx, int ns, int& A, int& B) {
  int a = 0, start = 0;
  while (idx >= start + (ns - a)) {
    start += ns - a;
    ++a;
  }
  A = a;
  B = a + (idx - start);
}

__host__ __device__ __forceinline__ int64_t item_index(int A, int B, int ns) {
  return (int64_t)A * ns - (int64_t)A * (A - 1) / 2 + (B - A);
}

// float4s per staged point: one for d ≤ 4, two for d ≤ 8.
template <int D>
constexpr int sym_nq() {
  return D > 4 ? 2 : 1;
}

// Both super blocks (points and vectors) are staged in LDS once per pair.
// Thread (tr, tc) of the 16×16 grid takes rows ii·16 + tr and columns
// jj·16 + tc (ii, jj < 8) of each 128×128 tile, so that the 16-byte point
// reads of a wave hit consecutive LDS addresses.
// The partial-sum buffer is double-buffered for one vector; for two, a
// single buffer (and one more barrier per tile) keeps the LDS of a
// workgroup under 80 KB, so that two fit on a CU.
template <int K>
constexpr int part_bufs() {
  return K == 1 ? 2 : 1;
}

template <int K, int NQ>
struct SymLds {
  float4 x[2][kSymSuper * NQ];                  // [0]: rows (A), [1]: columns (B)
  float v[2][kSymSuper * K];
  float part[part_bufs<K>()][16][kSymTile * K];  // per-group partial sums
  float colacc[kSymSuper * K];                  // column sums of the pair (B side)
};

template <int K, int NQ>
__device__ __forceinline__ void stage_block(const SymArgs& a, int64_t p0, float4* x, float* v) {
  for (int e = threadIdx.x; e < kSymSuper * NQ; e += 256)
    x[e] = p0 + e / NQ < a.n ? *reinterpret_cast<const float4*>(a.Xp + (p0 * NQ + e) * 4)
                             : make_float4(kFar, kFar, kFar, kFar);
  for (int e = threadIdx.x; e < kSymSuper * K; e += 256)
    v[e] = p0 * K + e < a.n * K ? a.V[p0 * K + e] : 0.0f;
}

// One block pair (A, B) with slots `item`; called by all 256 threads.
template <int KERN, int D, int K, bool DIAG>
__device__ __forceinline__ void sym_pair(const SymArgs& a, int A, int B, int64_t item,
                                         SymLds<K, sym_nq<D>()>& L) {
  constexpr int NQ = sym_nq<D>();
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  const int rs = DIAG ? 1 : 0;  // row side: the column block itself on the diagonal
  for (int e = tid; e < kSymSuper * K; e += 256) L.colacc[e] = 0.0f;
  if (!DIAG) stage_block<K, NQ>(a, (int64_t)A * kSymSuper, L.x[0], L.v[0]);
  stage_block<K, NQ>(a, (int64_t)B * kSymSuper, L.x[1], L.v[1]);
  __syncthreads();
  float* prow = a.prow + (size_t)item * kSymSuper * K;
  float* pcol = a.pcol + (size_t)item * kSymSuper * K;
  int buf = 0;
  for (int rt = 0; rt < kSymSub; ++rt) {
    float xi[kMicro][D], vi[kMicro][K], ar[kMicro][K];
#pragma unroll
    for (int ii = 0; ii < kMicro; ++ii) {
      const int r = rt * kSymTile + ii * 16 + tr;
#pragma unroll
      for (int h = 0; h < NQ; ++h) {
        const float4 q = L.x[rs][r * NQ + h];
        if (4 * h < D) xi[ii][4 * h] = q.x;
        if (4 * h + 1 < D) xi[ii][4 * h + 1] = q.y;
        if (4 * h + 2 < D) xi[ii][4 * h + 2] = q.z;
        if (4 * h + 3 < D) xi[ii][4 * h + 3] = q.w;
      }
#pragma unroll
      for (int c = 0; c < K; ++c) {
        vi[ii][c] = L.v[rs][r * K + c];
        ar[ii][c] = 0.0f;
      }
    }
    for (int ct = 0; ct < kSymSub; ++ct) {
      float xj[kMicro][D], vj[kMicro][K], ac[kMicro][K];
#pragma unroll
      for (int jj = 0; jj < kMicro; ++jj) {
        const int q0 = ct * kSymTile + jj * 16 + tc;
#pragma unroll
        for (int h = 0; h < NQ; ++h) {
          const float4 q = L.x[1][q0 * NQ + h];
          if (4 * h < D) xj[jj][4 * h] = q.x;
          if (4 * h + 1 < D) xj[jj][4 * h + 1] = q.y;
          if (4 * h + 2 < D) xj[jj][4 * h + 2] = q.z;
          if (4 * h + 3 < D) xj[jj][4 * h + 3] = q.w;
        }
#pragma unroll
        for (int c = 0; c < K; ++c) {
          vj[jj][c] = L.v[1][q0 * K + c];
          ac[jj][c] = 0.0f;
        }
      }
#pragma unroll
      for (int ii = 0; ii < kMicro; ++ii) {
#pragma unroll
        for (int jj = 0; jj < kMicro; ++jj) {
          float r2 = 0.0f;
#pragma unroll
          for (int c = 0; c < D; ++c) {
            const float df = xi[ii][c] - xj[jj][c];
            r2 = fmaf(df, df, r2);
          }
          float kv, kg;
          kval_f32<KERN, false>(r2, kv, kg);
#pragma unroll
          for (int c = 0; c < K; ++c) {
            ar[ii][c] = fmaf(kv, vj[jj][c], ar[ii][c]);
            if constexpr (!DIAG) ac[jj][c] = fmaf(kv, vi[ii][c], ac[jj][c]);
          }
        }
      }
      if constexpr (!DIAG) {
        // Column sums of this tile: the 16 row groups' partials, in order.
#pragma unroll
        for (int jj = 0; jj < kMicro; ++jj)
#pragma unroll
          for (int c = 0; c < K; ++c) L.part[buf][tr][(jj * 16 + tc) * K + c] = ac[jj][c];
        __syncthreads();
        for (int e = tid; e < kSymTile * K; e += 256) {
          float s = 0.0f;
#pragma unroll
          for (int g = 0; g < 16; ++g) s += L.part[buf][g][e];
          L.colacc[ct * kSymTile * K + e] += s;
        }
        if constexpr (part_bufs<K>() == 2)
          buf ^= 1;
        else
          __syncthreads();
      }
    }
    // Row sums of this row tile: the 16 column groups' partials, in order.
#pragma unroll
    for (int ii = 0; ii < kMicro; ++ii)
#pragma unroll
      for (int c = 0; c < K; ++c) L.part[buf][tc][(ii * 16 + tr) * K + c] = ar[ii][c];
    __syncthreads();
    for (int e = tid; e < kSymTile * K; e += 256) {
      float s = 0.0f;
#pragma unroll
      for (int g = 0; g < 16; ++g) s += L.part[buf][g][e];
      prow[rt * kSymTile * K + e] = s;
    }
    if constexpr (part_bufs<K>() == 2)
      buf ^= 1;
    else
      __syncthreads();
  }
  if constexpr (!DIAG) {
    __syncthreads();
    for (int e = tid; e < kSymSuper * K; e += 256) pcol[e] = L.colacc[e];
  }
}

// Y[i] = f²·(Σ_{A<S} colsum(A, S)[i] + Σ_{B≥S} rowsum(S, B)[i]) + s·V[i], S the
// super block of row i, added in that order in FP64.
template <int K>
__global__ void kmv_f32_sym_finish(int64_t n, int ns, const float* __restrict__ prow,
                                   const float* __restrict__ pcol, const float* __restrict__ V,
                                   float* __restrict__ Y, double f2, double s) {
  const int64_t count = n * K;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / K;
    const int S = (int)(i / kSymSuper);
    const int64_t off = (i % kSymSuper) * K + (e % K);
    double acc = 0.0;
    for (int A = 0; A < S; ++A) acc += pcol[item_index(A, S, ns) * kSymSuper * K + off];
    for (int B = S; B < ns; ++B) acc += prow[item_index(S, B, ns) * kSymSuper * K + off];
    Y[e] = (float)(f2 * acc + s * (double)V[e]);
  }
}

}  // namespace
}  // namespace higp
