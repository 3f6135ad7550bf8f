// FP32 on-the-fly kernel MatVec (and derivative MatVec) with
// v_mfma_f32_32x32x2f32 on gfx950.
//
// HiGP forms small kernel-matrix blocks, multiplies them into the vectors
// immediately and discards them ("Statement of Need", MatVec paragraph).
// Here every kernel value is formed in a register, directly in the MFMA
// A-operand slot, and multiplied by the matrix core with a V tile held in
// LDS; K is never stored.
//
// Work decomposition (split-J, XCD-aware).  Workgroup b owns row tile
// b / S (BM rows) and J chunk b mod S (a contiguous run of 128-point J
// tiles).  Workgroups are dealt to the 8 XCDs round-robin, so with S a
// multiple of 8 every XCD streams only its own S/8 chunks of X and V, which
// stay in that XCD's L2.  J tiles are copied global → LDS directly
// (buffer_load … lds, double-buffered, no staging registers).  Each
// workgroup writes the raw partial sums of its chunk; an epilogue kernel adds
// the S partials of every output in chunk order (deterministic, no atomics)
// and applies f², s and the derivative factors.
//
// Per wave: RB blocks of 32 rows.  At MFMA step j0 lane l supplies
// K[i0 + l%32][j0 + l/32] for each row block; the RB products share the x_j
// and V reads.  NB blocks of 32 columns go through the matrix core; NV ≤ 2
// trailing columns are accumulated on the VALU (k = 33 is 32 MFMA columns
// plus one VALU column rather than padding to 64).  Accumulator layout
// (32×32): lane l, register r holds row 8(r/4) + 4(l/32) + r%4, column l%32.
//
// Accumulation is FP32 within one J tile (64 MFMA steps); tile sums are added
// into FP64 running totals, so a long FP32 accumulation over n terms does
// not build up rounding error.
//
// Points come from a prepared copy Xp (step a1): x̃ padded to P = 4 or 8
// floats with zeros, and padded to whole J tiles with far-away sentinel
// points (all coordinates kFar) whose kernel value is exactly 0, so no tile
// needs masking in the inner loop.  V is read as a contiguous block of 128·k
// floats per tile (row stride k in LDS); reads past its end return 0.
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "kvalue.h"

namespace higp {
namespace {

constexpr int kWaves = 4;
constexpr int kBJ = 128;       // J points per LDS tile
constexpr float kFar = 1e18f;  // squared distance ~1e36: exp2 underflows to exactly 0

typedef __attribute__((address_space(3))) void lds_void_t;

// a1: x̃ = x·xs padded to P floats; rows n..npad−1 are far-away sentinels.
template <int P>
__global__ void prep_points_f32(int64_t n, int64_t npad, int d, const float* __restrict__ X,
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

// Buffer resource over `bytes` bytes at `base` (reads past the end return 0).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int64_t bytes) {
  const int nrec = bytes > 0x7fffffff ? 0x7fffffff : (int)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, nrec, 0x00020000);
}

struct Args {
  const float* Xp;  // npad×P prepared points
  const float* V;   // n×k (16-byte aligned, readable up to nk_pad elements)
  float* part;      // partials [S][n][k]: Σ k·v over each J chunk
  float* part2;     // same layout: Σ k_l·v (GRAD)
  int64_t n;
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
  constexpr int P = D <= 4 ? 4 : 8;
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
    for (int c = 0; c < P; ++c) xi[rb][c] = i < a.n ? a.Xp[i * P + c] : 0.0f;
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
    const int64_t nk = a.n * k;
    float* q1 = a.part + (int64_t)split * nk + rt * BM * k;
    float* q2 = GRAD ? a.part2 + (int64_t)split * nk + rt * BM * k : nullptr;
    const int64_t rows_left = a.n - rt * BM;
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
#pragma unroll 2
    for (int st = 0; st < kBJ / 2; ++st) {
      const float* xj = xs + st * 2 * P;
      float kv[RB], kg[RB];
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) {
        float r2 = 0.0f;
        const f32x4 xa = *reinterpret_cast<const f32x4*>(xj);
        if constexpr (P == 4) {
#pragma unroll
          for (int c = 0; c < D; ++c) {
            const float df = xi[rb][c] - xa[c];
            r2 = fmaf(df, df, r2);
          }
        } else {
          const f32x4 xb = *reinterpret_cast<const f32x4*>(xj + 4);
#pragma unroll
          for (int c = 0; c < D; ++c) {
            const float df = xi[rb][c] - (c < 4 ? xa[c & 3] : xb[c & 3]);
            r2 = fmaf(df, df, r2);
          }
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

template <int KERN, int D, int NB, int NV, int RB, bool GRAD, bool EXACT>
__global__ __launch_bounds__(256) void kmv_f32(Args a) {
  extern __shared__ __attribute__((aligned(16))) float smem[];
  kmv_f32_unit<KERN, D, NB, NV, RB, GRAD, EXACT>(a, blockIdx.x / a.nsplit, blockIdx.x % a.nsplit,
                                                  smem);
}

// ---------------------------------------------------------------------------
// Batched MatVec of many independent problems (continuous-batching serving):
// one persistent launch; each workgroup repeatedly takes the next work unit
// (problem, row tile, J chunk) from a global counter.  A problem's split count
// depends only on its own n, so its partial sums — and its result — are the
// same whatever else is in the batch.

struct BatchJob {
  Args a;
  int64_t first_unit;  // units of earlier jobs of the same launch (prefix sum)
  int kernel;          // HIGP_GAUSSIAN / HIGP_MATERN32
  int dcode;           // 2, 3, 4 or 8 (padded point dimension)
};

// Column kinds of a batched launch: 0 = k ≤ 32 through one 32-column MFMA
// block; 1 / 2 = k = 1 / 2 on the VALU only (a CG-only round).  The VALU
// kinds take four 32-row blocks per wave (more independent work per LDS read
// of a point) and reserve LDS only for the columns they carry, so more
// workgroups fit on a CU.
template <int KIND> struct KindCols;
template <> struct KindCols<0> { static constexpr int NB = 1, NV = 0, RB = 2, KMAX = 32; };
template <> struct KindCols<1> { static constexpr int NB = 0, NV = 1, RB = 4, KMAX = 1; };
template <> struct KindCols<2> { static constexpr int NB = 0, NV = 2, RB = 4, KMAX = 2; };

template <int KIND>
constexpr int64_t kind_rows() {  // rows per work unit
  return 32LL * KindCols<KIND>::RB * kWaves;
}

template <int KIND>
constexpr size_t kind_lds() {  // X tile (8 floats a point) + V tile, double-buffered
  return (size_t)2 * kBJ * (8 + KindCols<KIND>::KMAX) * 4;
}

template <int KERN, int KIND>
__device__ __forceinline__ void batch_unit(const Args& a, int dcode, int64_t rt, int split,
                                           float* smem) {
  constexpr int NB = KindCols<KIND>::NB, NV = KindCols<KIND>::NV, RB = KindCols<KIND>::RB;
  constexpr bool EX = KIND != 0;  // k = 1 and k = 2 are exact
  if (dcode == 2) kmv_f32_unit<KERN, 2, NB, NV, RB, false, EX>(a, rt, split, smem);
  else if (dcode == 3) kmv_f32_unit<KERN, 3, NB, NV, RB, false, EX>(a, rt, split, smem);
  else if (dcode == 4) kmv_f32_unit<KERN, 4, NB, NV, RB, false, EX>(a, rt, split, smem);
  else kmv_f32_unit<KERN, 8, NB, NV, RB, false, EX>(a, rt, split, smem);
}

template <int KIND>
__global__ __launch_bounds__(256) void kmv_f32_batch(const BatchJob* __restrict__ jobs, int njobs,
                                                     int64_t total, unsigned long long* counter) {
  extern __shared__ __attribute__((aligned(16))) float smem[];
  __shared__ long long unit_sh;
  for (;;) {
    if (threadIdx.x == 0) unit_sh = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const int64_t u = unit_sh;
    __syncthreads();
    if (u >= total) break;
    int lo = 0, hi = njobs - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) / 2;
      if (jobs[mid].first_unit <= u) lo = mid;
      else hi = mid - 1;
    }
    const Args a = jobs[lo].a;
    const int64_t local = u - jobs[lo].first_unit;
    const int64_t rt = local / a.nsplit;
    const int split = (int)(local % a.nsplit);
    if (jobs[lo].kernel == HIGP_GAUSSIAN)
      batch_unit<HIGP_GAUSSIAN, KIND>(a, jobs[lo].dcode, rt, split, smem);
    else
      batch_unit<HIGP_MATERN32, KIND>(a, jobs[lo].dcode, rt, split, smem);
    __syncthreads();
  }
}

// out = f²·Σ_s P1[s] + s·V (chunks added in order, in FP64), and the
// derivative outputs.
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
    if (o1) o1[e] = (float)(f2 * s1 + s * (double)V[e]);
    if (o2) o2[e] = (float)(cl * s2);
    if (o3) o3[e] = (float)(cf * s1);
  }
}

using Fn = void (*)(Args);

template <int KERN, int D, int NB, int NV, bool GRAD, bool EXACT>
Fn inst(int* rb) {
  constexpr int RB = (NB == 2 || GRAD) ? 1 : 2;
  *rb = RB;
  return kmv_f32<KERN, D, NB, NV, RB, GRAD, EXACT>;
}

// Column blocking: NB blocks of 32 MFMA columns and NV ≤ 2 VALU columns.
// EXACT instances (k = 1, 2, 32, 33, 34, 64) know the V row stride at
// compile time.
template <int KERN, int D, bool GRAD>
Fn pick_cols(int k, int* rb) {
  if (k == 1) return inst<KERN, D, 0, 1, GRAD, true>(rb);
  if (k == 2) return inst<KERN, D, 0, 2, GRAD, true>(rb);
  if (k == 32) return inst<KERN, D, 1, 0, GRAD, true>(rb);
  if (k < 32) return inst<KERN, D, 1, 0, GRAD, false>(rb);
  if (k == 33) return inst<KERN, D, 1, 1, GRAD, true>(rb);
  if (k == 34) return inst<KERN, D, 1, 2, GRAD, true>(rb);
  if (k == 64) return inst<KERN, D, 2, 0, GRAD, true>(rb);
  return inst<KERN, D, 2, 0, GRAD, false>(rb);
}

template <int KERN, bool GRAD>
Fn pick_d(int d, int k, int* rb) {
  if (d <= 2) return pick_cols<KERN, 2, GRAD>(k, rb);
  if (d == 3) return pick_cols<KERN, 3, GRAD>(k, rb);
  if (d == 4) return pick_cols<KERN, 4, GRAD>(k, rb);
  return pick_cols<KERN, 8, GRAD>(k, rb);
}

// Split count override for tuning experiments (HIGP_F32_SPLITS; 0 = automatic).
int g_split_override = [] {
  const char* e = getenv("HIGP_F32_SPLITS");
  return e ? atoi(e) : 0;
}();

// Resident workgroups per CU for (kernel, LDS bytes), cached per device.
int blocks_per_cu(Fn fn, size_t lds) {
  static std::mutex mu;
  static std::unordered_map<uint64_t, int> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const uint64_t key = reinterpret_cast<uint64_t>(fn) ^ ((uint64_t)lds << 40) ^ ((uint64_t)dev << 60);
  std::lock_guard<std::mutex> g(mu);
  auto itc = cache.find(key);
  if (itc != cache.end()) return itc->second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(fn), 256,
                                                   lds) != hipSuccess ||
      nb < 1)
    nb = 1;
  cache[key] = nb;
  return nb;
}

}  // namespace

int launch_kmatvec_f32(const Problem& p, int k, const void* Vin, MatvecOut out, hipStream_t st,
                       int num_cus) {
  const bool grad = out.dl != nullptr || out.df != nullptr;
  int rb = 1;
  Fn fn;
  if (p.kernel == HIGP_GAUSSIAN)
    fn = grad ? pick_d<HIGP_GAUSSIAN, true>(p.d, k, &rb) : pick_d<HIGP_GAUSSIAN, false>(p.d, k, &rb);
  else
    fn = grad ? pick_d<HIGP_MATERN32, true>(p.d, k, &rb) : pick_d<HIGP_MATERN32, false>(p.d, k, &rb);
  const float xs = (float)coord_scale(p.kernel, HIGP_FP32, p.l);
  const double cl = p.f * p.f * dl_factor(p.kernel, HIGP_FP32, p.l);

  const int bm = 32 * rb * kWaves;
  const int P = p.d <= 4 ? 4 : 8;
  const int64_t nk = p.n * k;
  const int64_t jt_count = (p.n + kBJ - 1) / kBJ;
  const int64_t npad = jt_count * kBJ;
  const int64_t rt_count = (p.n + bm - 1) / bm;
  const size_t lds = (size_t)2 * kBJ * P * 4 + (size_t)2 * kBJ * k * 4;
  if (lds > 65536 &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return set_error(HIGP_ERR_HIP, "cannot reserve %zu bytes of LDS", lds);
  // Split count S: a multiple of 8 (one set of J chunks per XCD) when the
  // grid is large enough, growing until there are several rounds of
  // workgroups per CU (so the last, partial round costs little) while every
  // chunk keeps at least two J tiles.
  const int64_t slots = (int64_t)num_cus * blocks_per_cu(fn, lds);
  int S = 1;
  while (S < 64 && rt_count * S < 8 * slots && jt_count >= 4LL * S) S *= 2;
  if (g_split_override > 0) S = g_split_override;
  const int jt_chunk = (int)((jt_count + S - 1) / S);
  const int64_t grid = rt_count * S;
  if (grid > 0x7fffffffLL) return set_error(HIGP_ERR_INVALID_ARG, "n too large");

  // Scratch: prepared points (whole J tiles); a zero-padded copy of V unless
  // V is 16-byte aligned and n·k is a multiple of 4 (tiles move 16-byte
  // chunks); the partial slots.
  const bool direct_v = (reinterpret_cast<uintptr_t>(Vin) & 15) == 0 && nk % 4 == 0;
  const int64_t nk_pad = (nk + 3) / 4 * 4;
  const size_t xp_bytes = ((size_t)npad * P * 4 + 255) / 256 * 256;
  const size_t v_bytes = direct_v ? 0 : ((size_t)nk_pad * 4 + 255) / 256 * 256;
  const size_t part_bytes = ((size_t)S * nk * 4 + 255) / 256 * 256;
  void* scratch = nullptr;
  HIGP_TRY(scratch_alloc(&scratch, xp_bytes + v_bytes + part_bytes * (grad ? 2 : 1), st));
  char* base = static_cast<char*>(scratch);
  float* Xp = reinterpret_cast<float*>(base);
  const float* V = static_cast<const float*>(Vin);
  int rc = HIGP_OK;
  if (!direct_v) {
    float* Vc = reinterpret_cast<float*>(base + xp_bytes);
    const unsigned cb = (unsigned)std::min<int64_t>((nk_pad + 255) / 256, 4096);
    hipLaunchKernelGGL(copy_pad_f32, dim3(cb), dim3(256), 0, st, nk, nk_pad,
                       static_cast<const float*>(Vin), Vc);
    V = Vc;
  }
  {
    const unsigned pb = (unsigned)std::min<int64_t>((npad * P + 255) / 256, 4096);
    if (P == 4)
      hipLaunchKernelGGL(prep_points_f32<4>, dim3(pb), dim3(256), 0, st, p.n, npad, p.d,
                         static_cast<const float*>(p.X), xs, Xp);
    else
      hipLaunchKernelGGL(prep_points_f32<8>, dim3(pb), dim3(256), 0, st, p.n, npad, p.d,
                         static_cast<const float*>(p.X), xs, Xp);
  }
  Args a{};
  a.Xp = Xp;
  a.V = V;
  a.part = reinterpret_cast<float*>(base + xp_bytes + v_bytes);
  a.part2 = grad ? reinterpret_cast<float*>(base + xp_bytes + v_bytes + part_bytes) : nullptr;
  a.n = p.n;
  a.nk_pad = direct_v ? nk : nk_pad;
  a.jt_count = (int)jt_count;
  a.jt_chunk = jt_chunk;
  a.nsplit = S;
  a.k = k;
  hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(256), lds, st, a);
  const unsigned eb = (unsigned)std::min<int64_t>((nk + 255) / 256, 8LL * num_cus);
  hipLaunchKernelGGL(kmv_f32_epilogue, dim3(eb), dim3(256), 0, st, (const float*)a.part,
                     (const float*)a.part2, V, static_cast<float*>(out.kv),
                     static_cast<float*>(out.dl), static_cast<float*>(out.df), nk, S, p.f * p.f,
                     p.s, cl, 2.0 * p.f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) rc = set_error(HIGP_ERR_HIP, "FP32 MatVec launch failed: %s", hipGetErrorString(e));
  scratch_free(scratch, st);
  return rc;
}

}  // namespace higp

namespace higp {

// Split count of one problem in a batched launch: a function of n only, so a
// problem's partial sums do not depend on the rest of the batch.
int batch_splits(int64_t n) {
  const int64_t jt = (n + kBJ - 1) / kBJ;
  int S = 1;
  while (S < 16 && jt >= 8LL * S) S *= 2;
  return S;
}

size_t prepared_points_bytes(int64_t n, int d) {
  const int64_t npad = (n + kBJ - 1) / kBJ * kBJ;
  return (size_t)npad * (d <= 4 ? 4 : 8) * 4;
}

int prepare_points_f32(const Problem& p, float* Xp, hipStream_t st) {
  const int P = p.d <= 4 ? 4 : 8;
  const int64_t npad = (p.n + kBJ - 1) / kBJ * kBJ;
  const float xs = (float)coord_scale(p.kernel, HIGP_FP32, p.l);
  const unsigned pb = (unsigned)std::min<int64_t>((npad * P + 255) / 256, 4096);
  if (P == 4)
    hipLaunchKernelGGL(prep_points_f32<4>, dim3(pb), dim3(256), 0, st, p.n, npad, p.d,
                       static_cast<const float*>(p.X), xs, Xp);
  else
    hipLaunchKernelGGL(prep_points_f32<8>, dim3(pb), dim3(256), 0, st, p.n, npad, p.d,
                       static_cast<const float*>(p.X), xs, Xp);
  return hipGetLastError() == hipSuccess ? HIGP_OK : set_error(HIGP_ERR_HIP, "prep launch failed");
}

namespace {

template <int KIND>
int launch_batch_kind(const std::vector<BatchJob>& hj, const std::vector<const BatchMatvec*>& src,
                      int64_t total, size_t part_elems, hipStream_t st, int num_cus) {
  const int count = (int)hj.size();
  if (count == 0) return HIGP_OK;
  const size_t jobs_bytes = ((size_t)count * sizeof(BatchJob) + 255) / 256 * 256;
  void* mem = nullptr;
  HIGP_TRY(scratch_alloc(&mem, jobs_bytes + 256 + part_elems * 4, st));
  char* base = static_cast<char*>(mem);
  BatchJob* djobs = reinterpret_cast<BatchJob*>(base);
  unsigned long long* counter = reinterpret_cast<unsigned long long*>(base + jobs_bytes);
  float* part = reinterpret_cast<float*>(base + jobs_bytes + 256);
  std::vector<BatchJob> j2 = hj;
  size_t off = 0;
  for (int i = 0; i < count; ++i) {
    j2[i].a.part = part + off;
    off += (size_t)j2[i].a.nsplit * src[i]->n * src[i]->k;
  }
  int rc = HIGP_OK;
  if (hipMemcpyAsync(djobs, j2.data(), count * sizeof(BatchJob), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemsetAsync(counter, 0, 8, st) != hipSuccess)
    rc = set_error(HIGP_ERR_HIP, "batch setup failed");
  const size_t lds = kind_lds<KIND>();
  static int bpc = 0;
  if (bpc == 0) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void*>(kmv_f32_batch<KIND>), 256, lds) != hipSuccess ||
        nb < 1)
      nb = 1;
    bpc = nb;
  }
  if (rc == HIGP_OK) {
    const int64_t grid = std::min<int64_t>(total, (int64_t)num_cus * bpc);
    hipLaunchKernelGGL(kmv_f32_batch<KIND>, dim3((unsigned)grid), dim3(256), lds, st,
                       (const BatchJob*)djobs, count, total, counter);
    for (int i = 0; i < count; ++i) {
      const int64_t nk = src[i]->n * src[i]->k;
      const unsigned eb = (unsigned)std::min<int64_t>((nk + 255) / 256, 2LL * num_cus);
      hipLaunchKernelGGL(kmv_f32_epilogue, dim3(eb), dim3(256), 0, st, (const float*)j2[i].a.part,
                         (const float*)nullptr, src[i]->V, src[i]->Y, (float*)nullptr,
                         (float*)nullptr, nk, j2[i].a.nsplit, src[i]->f * src[i]->f, src[i]->s,
                         0.0, 0.0);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
      rc = set_error(HIGP_ERR_HIP, "batched MatVec launch failed: %s", hipGetErrorString(e));
  }
  scratch_free(mem, st);
  return rc;
}

}  // namespace

int launch_kmatvec_f32_batch(const BatchMatvec* jobs, int count, hipStream_t st, int num_cus) {
  if (count <= 0) return HIGP_OK;
  std::vector<BatchJob> hj[3];
  std::vector<const BatchMatvec*> src[3];
  int64_t total[3] = {0, 0, 0};
  size_t part_elems[3] = {0, 0, 0};
  for (int i = 0; i < count; ++i) {
    const BatchMatvec& J = jobs[i];
    if (J.k < 1 || J.k > 32)
      return set_error(HIGP_ERR_UNSUPPORTED, "batched MatVec supports 1 <= k <= 32");
    const int kind = J.k == 1 ? 1 : (J.k == 2 ? 2 : 0);
    const int S = batch_splits(J.n);
    const int64_t jt = (J.n + kBJ - 1) / kBJ;
    const int64_t bm = kind == 0 ? kind_rows<0>() : kind_rows<1>();
    const int64_t rt = (J.n + bm - 1) / bm;
    BatchJob b{};
    b.a.Xp = J.Xp;
    b.a.V = J.V;
    b.a.n = J.n;
    b.a.nk_pad = (J.n * J.k + 3) / 4 * 4;
    b.a.jt_count = (int)jt;
    b.a.jt_chunk = (int)((jt + S - 1) / S);
    b.a.nsplit = S;
    b.a.k = J.k;
    b.first_unit = total[kind];
    b.kernel = J.kernel;
    b.dcode = J.d <= 2 ? 2 : (J.d == 3 ? 3 : (J.d == 4 ? 4 : 8));
    total[kind] += rt * S;
    part_elems[kind] += (size_t)S * J.n * J.k;
    hj[kind].push_back(b);
    src[kind].push_back(&J);
  }
  HIGP_TRY(launch_batch_kind<0>(hj[0], src[0], total[0], part_elems[0], st, num_cus));
  HIGP_TRY(launch_batch_kind<1>(hj[1], src[1], total[1], part_elems[1], st, num_cus));
  HIGP_TRY(launch_batch_kind<2>(hj[2], src[2], total[2], part_elems[2], st, num_cus));
  return HIGP_OK;
}

}  // namespace higp
