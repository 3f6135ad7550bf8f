// Shared building blocks of the FP32 on-the-fly MatVec: point preparation,
// the tile unit (one row tile × one J chunk) and the epilogue.  Included by
// the single-problem launcher and the batched (serving) launcher; see
// kmatvec_f32.hip for the design.
#pragma once

#include "bufload.h"
#include "kvalue.h"

namespace higp {
namespace {


constexpr int kWaves = 4;
constexpr int kBJ = 128;       // J points per LDS tile
constexpr float kFar = 1e18f;  // squared distance ~1e36: exp2 underflows to exactly 0

// Padded storage width of a point with D coordinates: 4, 8, or D rounded up
// to a multiple of 4 (16-byte loads).
__host__ __device__ constexpr int pad_dim(int d) {
  return d <= 4 ? 4 : (d <= 8 ? 8 : (d + 3) / 4 * 4);
}

// Compile-time dimension of the kernel instance serving d coordinates.
inline int dim_code(int d) {
  return d <= 2 ? 2 : d == 3 ? 3 : d == 4 ? 4 : d <= 8 ? 8 : d <= 16 ? 16 : d <= 20 ? 20 : 32;
}

// a1: x̃ = x·xs padded to P floats; rows n..npad−1 are far-away sentinels.
__global__ void prep_points_f32(int64_t n, int64_t npad, int d, int P, const float* __restrict__ X,
                                float xs, float* __restrict__ Xp) {
  const int64_t count = npad * P;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / P;
    const int c = (int)(e % P);
    Xp[e] = i >= n ? kFar : (c < d ? X[i * d + c] * xs : 0.0f);
  }
}

// dst[0..count_pad) = src[0..count) followed by zeros.
__global__ void copy_pad_f32(int64_t count, int64_t count_pad, const float* __restrict__ src,
                             float* __restrict__ dst) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count_pad;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = e < count ? src[e] : 0.0f;
}

struct Args {
  const float* Xp;  // npad×P prepared points of the J (column) side
  const float* Xq;  // prepared points of the row side (Xp for a square MatVec)
  const float* V;   // n×k (16-byte aligned, readable up to nk_pad elements)
  float* part;      // partials [S][m][k]: Σ k·v over each J chunk
  float* part2;     // same layout: Σ k_l·v (GRAD)
  int64_t m;        // rows (query points; n for a square MatVec)
  int64_t nk_pad;
  int jt_count;     // J tiles
  int jt_chunk;     // J tiles per chunk
  int nsplit;       // S
  int k;
};

// One work unit: row tile `rt` × J chunk `split` of one MatVec, partial sums
// written to part[split].  Called by every thread of a 256-thread workgroup.
template <int KERN, int D, int NB, int NV, int RB, bool GRAD, bool EXACT>
__device__ __forceinline__ void kmv_f32_unit(const Args& a, int64_t rt, int split, float* smem) {
  constexpr int P = pad_dim(D);
  constexpr int BM = 32 * RB * kWaves;
  constexpr int NBa = NB > 0 ? NB : 1;
  constexpr int NVa = NV > 0 ? NV : 1;
  constexpr int G2 = GRAD ? 2 : 1;  // contractions: k·v and (GRAD) k_l·v
  constexpr int KMAX = NB * 32 + NV;  // largest k served; EXACT: k == KMAX
  const int k = EXACT ? KMAX : a.k;   // V row stride in LDS (compile-time when EXACT)
  const int vtile = kBJ * k;
  float* Xs = smem;                 // [2][kBJ][P]
  float* Vs = smem + 2 * kBJ * P;   // [2][kBJ·k]

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int half = lane >> 5;
  const int l32 = lane & 31;

  const int jt_beg = split * a.jt_chunk;
  const int jt_end = jt_beg + a.jt_chunk < a.jt_count ? jt_beg + a.jt_chunk : a.jt_count;

  float xi[RB][P];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int64_t i = rt * BM + wave * 32 * RB + rb * 32 + l32;
#pragma unroll
    for (int c = 0; c < P; ++c) xi[rb][c] = i < a.m ? a.Xq[i * P + c] : 0.0f;
  }

  f32x16 acc[G2][RB][NBa];
  double tot[G2][RB][NBa][16];
  float accv[G2][RB][NVa];
  double totv[G2][RB][NVa];
#pragma unroll
  for (int g = 0; g < G2; ++g)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        acc[g][rb][b] = f32x16{0};
#pragma unroll
        for (int r = 0; r < 16; ++r) tot[g][rb][b][r] = 0.0;
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        accv[g][rb][v] = 0.0f;
        totv[g][rb][v] = 0.0;
      }
    }

  // Global → LDS copy of J tile `jt` into buffer `buf`: every wave issues its
  // share of 16-byte chunks, 64 consecutive chunks (1 KB) per instruction.
  constexpr int XC = kBJ * P / 4;  // chunks of the X tile
  const int vchunks = vtile / 4;   // chunks of the V tile
  auto gload = [&](int64_t jt, int buf) {
    char* xs = reinterpret_cast<char*>(Xs + buf * kBJ * P);
    char* vs = reinterpret_cast<char*>(Vs + buf * vtile);
    const int64_t j0 = jt * kBJ;
    const __amdgpu_buffer_rsrc_t rx = make_rsrc(a.Xp + j0 * P, (int64_t)kBJ * P * 4);
    for (int m = wave * 64; m < XC; m += 256)
      if (m + lane < XC)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (lds_void_t*)(xs + 16 * m), 16,
                                                 16 * (m + lane), 0, 0, 0);
    const __amdgpu_buffer_rsrc_t rv = make_rsrc(a.V + j0 * k, (a.nk_pad - j0 * k) * 4);
    for (int m = wave * 64; m < vchunks; m += 256)
      if (m + lane < vchunks)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rv, (lds_void_t*)(vs + 16 * m), 16,
                                                 16 * (m + lane), 0, 0, 0);
  };

  // Partial sums of this chunk → part[split] (FP64 totals, rounded once).
  auto flush = [&]() {
    const int64_t nk = a.m * k;
    float* q1 = a.part + (int64_t)split * nk + rt * BM * k;
    float* q2 = GRAD ? a.part2 + (int64_t)split * nk + rt * BM * k : nullptr;
    const int64_t rows_left = a.m - rt * BM;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int lrow0 = wave * 32 * RB + rb * 32;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int col = b * 32 + l32;
        if (col < k) {
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int lrow = lrow0 + 8 * (r >> 2) + 4 * half + (r & 3);
            if (lrow < rows_left) {
              q1[lrow * k + col] = (float)tot[0][rb][b][r];
              if constexpr (GRAD) q2[lrow * k + col] = (float)tot[G2 - 1][rb][b][r];
            }
          }
        }
#pragma unroll
        for (int g = 0; g < G2; ++g)
#pragma unroll
          for (int r = 0; r < 16; ++r) tot[g][rb][b][r] = 0.0;
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        // lanes l and l+32 hold the two halves of row l%32
#pragma unroll
        for (int g = 0; g < G2; ++g) totv[g][rb][v] += __shfl_xor(totv[g][rb][v], 32);
        if (half == 0 && lrow0 + l32 < rows_left) {
          q1[(lrow0 + l32) * k + NB * 32 + v] = (float)totv[0][rb][v];
          if constexpr (GRAD) q2[(lrow0 + l32) * k + NB * 32 + v] = (float)totv[G2 - 1][rb][v];
        }
#pragma unroll
        for (int g = 0; g < G2; ++g) totv[g][rb][v] = 0.0;
      }
    }
  };

  int cur = 0;
  if (jt_beg < jt_end) gload(jt_beg, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  for (int jt = jt_beg; jt < jt_end; ++jt) {
    if (jt + 1 < jt_end) gload(jt + 1, cur ^ 1);

    const float* xs = Xs + cur * kBJ * P + half * P;
    const float* vb_base = Vs + cur * vtile + half * k + l32;
    const float* vv_base = Vs + cur * vtile + half * k + NB * 32;
#pragma unroll 4
    for (int st = 0; st < kBJ / 2; ++st) {
      const float* xj = xs + st * 2 * P;
      float kv[RB], kg[RB];
      f32x4 xv[P / 4];  // x_j, shared by the RB rows
#pragma unroll
      for (int q = 0; q < P / 4; ++q) xv[q] = *reinterpret_cast<const f32x4*>(xj + 4 * q);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        float r2 = 0.0f;
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const float df = xi[rb][c] - xv[c >> 2][c & 3];
          r2 = fmaf(df, df, r2);
        }
        kval_f32<KERN, GRAD>(r2, kv[rb], kg[rb]);
      }
      const int vo = st * 2 * k;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const float vb = vb_base[vo + b * 32];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          acc[0][rb][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(kv[rb], vb, acc[0][rb][b], 0, 0, 0);
          if constexpr (GRAD)
            acc[G2 - 1][rb][b] =
                __builtin_amdgcn_mfma_f32_32x32x2f32(kg[rb], vb, acc[G2 - 1][rb][b], 0, 0, 0);
        }
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const float vv = vv_base[vo + v];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          accv[0][rb][v] = fmaf(kv[rb], vv, accv[0][rb][v]);
          if constexpr (GRAD) accv[G2 - 1][rb][v] = fmaf(kg[rb], vv, accv[G2 - 1][rb][v]);
        }
      }
    }
    // Tile sums → FP64 running totals.
#pragma unroll
    for (int g = 0; g < G2; ++g)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
        for (int b = 0; b < NB; ++b) {
#pragma unroll
          for (int r = 0; r < 16; ++r) tot[g][rb][b][r] += (double)acc[g][rb][b][r];
          acc[g][rb][b] = f32x16{0};
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          totv[g][rb][v] += (double)accv[g][rb][v];
          accv[g][rb][v] = 0.0f;
        }
      }

    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    cur ^= 1;
  }
  flush();
}

// The 16-column form for k ≤ 16 (+ NV ≤ 1 VALU column): v_mfma_f32_16x16x4f32
// does half the MACs of the 32×32×2 form per kernel value, so a MatVec of 16
// or 17 vectors (16 Lanczos probes; y and 16 probes) needs half the MFMA time.
// A wave's row block is 16 rows; per step (4 J points) each lane forms
// K[i0 + lane%16][j0 + lane/16] for each of its RB row blocks as the A
// operand, against V[j0 + lane/16][lane%16] from LDS as the B operand; the
// accumulator holds row 4·(lane/16) + r, column lane%16 in register r.  The
// VALU column is added per lane and the 4 lanes of a row are summed at the
// end.  Accumulation as in the 32-column form: FP32 within a J tile, FP64
// running totals across tiles.
template <int KERN, int D, int NV, int RB, bool GRAD, bool EXACT>
__device__ __forceinline__ void kmv_f32_unit16(const Args& a, int64_t rt, int split,
                                               float* smem) {
  constexpr int P = pad_dim(D);
  constexpr int BM = 16 * RB * kWaves;
  constexpr int NVa = NV > 0 ? NV : 1;
  constexpr int G2 = GRAD ? 2 : 1;
  constexpr int KMAX = 16 + NV;
  const int k = EXACT ? KMAX : a.k;
  const int vtile = kBJ * k;
  float* Xs = smem;                // [2][kBJ][P]
  float* Vs = smem + 2 * kBJ * P;  // [2][kBJ·k]

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int q = lane >> 4;
  const int l16 = lane & 15;

  const int jt_beg = split * a.jt_chunk;
  const int jt_end = jt_beg + a.jt_chunk < a.jt_count ? jt_beg + a.jt_chunk : a.jt_count;

  float xi[RB][P];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    const int64_t i = rt * BM + wave * 16 * RB + rb * 16 + l16;
#pragma unroll
    for (int c = 0; c < P; ++c) xi[rb][c] = i < a.m ? a.Xq[i * P + c] : 0.0f;
  }

  f32x4 acc[G2][RB];
  double tot[G2][RB][4];
  float accv[G2][RB][NVa];
  double totv[G2][RB][NVa];
#pragma unroll
  for (int g = 0; g < G2; ++g)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      acc[g][rb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int r = 0; r < 4; ++r) tot[g][rb][r] = 0.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        accv[g][rb][v] = 0.0f;
        totv[g][rb][v] = 0.0;
      }
    }

  constexpr int XC = kBJ * P / 4;
  const int vchunks = vtile / 4;
  auto gload = [&](int64_t jt, int buf) {
    char* xs = reinterpret_cast<char*>(Xs + buf * kBJ * P);
    char* vs = reinterpret_cast<char*>(Vs + buf * vtile);
    const int64_t j0 = jt * kBJ;
    const __amdgpu_buffer_rsrc_t rx = make_rsrc(a.Xp + j0 * P, (int64_t)kBJ * P * 4);
    for (int m = wave * 64; m < XC; m += 256)
      if (m + lane < XC)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (lds_void_t*)(xs + 16 * m), 16,
                                                 16 * (m + lane), 0, 0, 0);
    const __amdgpu_buffer_rsrc_t rv = make_rsrc(a.V + j0 * k, (a.nk_pad - j0 * k) * 4);
    for (int m = wave * 64; m < vchunks; m += 256)
      if (m + lane < vchunks)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rv, (lds_void_t*)(vs + 16 * m), 16,
                                                 16 * (m + lane), 0, 0, 0);
  };

  auto flush = [&]() {
    const int64_t nk = a.m * k;
    float* q1 = a.part + (int64_t)split * nk + rt * BM * k;
    float* q2 = GRAD ? a.part2 + (int64_t)split * nk + rt * BM * k : nullptr;
    const int64_t rows_left = a.m - rt * BM;
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
      const int lrow0 = wave * 16 * RB + rb * 16;
      if (l16 < k) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int lrow = lrow0 + 4 * q + r;
          if (lrow < rows_left) {
            q1[lrow * k + l16] = (float)tot[0][rb][r];
            if constexpr (GRAD) q2[lrow * k + l16] = (float)tot[G2 - 1][rb][r];
          }
        }
      }
#pragma unroll
      for (int g = 0; g < G2; ++g)
#pragma unroll
        for (int r = 0; r < 4; ++r) tot[g][rb][r] = 0.0;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        // lanes l16 + 16q hold the J points ≡ q (mod 4) of row l16
#pragma unroll
        for (int g = 0; g < G2; ++g) {
          totv[g][rb][v] += __shfl_xor(totv[g][rb][v], 16);
          totv[g][rb][v] += __shfl_xor(totv[g][rb][v], 32);
        }
        if (q == 0 && lrow0 + l16 < rows_left) {
          q1[(lrow0 + l16) * k + 16 + v] = (float)totv[0][rb][v];
          if constexpr (GRAD) q2[(lrow0 + l16) * k + 16 + v] = (float)totv[G2 - 1][rb][v];
        }
#pragma unroll
        for (int g = 0; g < G2; ++g) totv[g][rb][v] = 0.0;
      }
    }
  };

  int cur = 0;
  if (jt_beg < jt_end) gload(jt_beg, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  for (int jt = jt_beg; jt < jt_end; ++jt) {
    if (jt + 1 < jt_end) gload(jt + 1, cur ^ 1);

    const float* xs = Xs + cur * kBJ * P + q * P;
    const float* vb_base = Vs + cur * vtile + q * k + l16;
    const float* vv_base = Vs + cur * vtile + q * k + 16;
    const bool col_ok = EXACT || l16 < k;  // B columns beyond k are zero
#pragma unroll 2
    for (int st = 0; st < kBJ / 4; ++st) {
      const float* xj = xs + st * 4 * P;
      float kv[RB], kg[RB];
      f32x4 xv[P / 4];
#pragma unroll
      for (int c4 = 0; c4 < P / 4; ++c4) xv[c4] = *reinterpret_cast<const f32x4*>(xj + 4 * c4);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        float r2 = 0.0f;
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const float df = xi[rb][c] - xv[c >> 2][c & 3];
          r2 = fmaf(df, df, r2);
        }
        kval_f32<KERN, GRAD>(r2, kv[rb], kg[rb]);
      }
      const int vo = st * 4 * k;
      const float vb = col_ok ? vb_base[vo] : 0.0f;
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        acc[0][rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv[rb], vb, acc[0][rb], 0, 0, 0);
        if constexpr (GRAD)
          acc[G2 - 1][rb] =
              __builtin_amdgcn_mfma_f32_16x16x4f32(kg[rb], vb, acc[G2 - 1][rb], 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const float vv = vv_base[vo + v];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          accv[0][rb][v] = fmaf(kv[rb], vv, accv[0][rb][v]);
          if constexpr (GRAD) accv[G2 - 1][rb][v] = fmaf(kg[rb], vv, accv[G2 - 1][rb][v]);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < G2; ++g)
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) tot[g][rb][r] += (double)acc[g][rb][r];
        acc[g][rb] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          totv[g][rb][v] += (double)accv[g][rb][v];
          accv[g][rb][v] = 0.0f;
        }
      }

    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    cur ^= 1;
  }
  flush();
}

// out = f²·Σ_s P1[s] + s·V (chunks added in order, in FP64; V null: no
// s·V term, as for a rectangular MatVec), and the derivative outputs.
__global__ void kmv_f32_epilogue(const float* __restrict__ P1, const float* __restrict__ P2,
                                 const float* __restrict__ V, float* o1, float* o2, float* o3,
                                 int64_t count, int nsplit, double f2, double s, double cl,
                                 double cf) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s1 = 0.0, s2 = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) {
      s1 += (double)P1[sp * count + e];
      if (P2) s2 += (double)P2[sp * count + e];
    }
    if (o1) o1[e] = (float)(f2 * s1 + (V ? s * (double)V[e] : 0.0));
    if (o2) o2[e] = (float)(cl * s2);
    if (o3) o3[e] = (float)(cf * s1);
  }
}

}  // namespace
}  // namespace higp
