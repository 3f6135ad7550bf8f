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
// Points come from a prepared copy Xp (step a1): x̃ padded to P = 4, 8, 16,
// 20 or 32 floats with zeros, and padded to whole J tiles with far-away sentinel
// points (all coordinates kFar) whose kernel value is exactly 0, so no tile
// needs masking in the inner loop.  V is read as a contiguous block of 128·k
// floats per tile (row stride k in LDS); reads past its end return 0.
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <unordered_map>

#include "kmv_f32_tile.h"

namespace higp {
namespace {

template <int KERN, int D, int NB, int NV, int RB, bool GRAD, bool EXACT>
__global__ __launch_bounds__(256) void kmv_f32(Args a) {
  extern __shared__ __attribute__((aligned(16))) float smem[];
  kmv_f32_unit<KERN, D, NB, NV, RB, GRAD, EXACT>(a, blockIdx.x / a.nsplit, blockIdx.x % a.nsplit,
                                                  smem);
}

template <int KERN, int D, int NV, int RB, bool GRAD, bool EXACT>
__global__ __launch_bounds__(256) void kmv_f32_16(Args a) {
  extern __shared__ __attribute__((aligned(16))) float smem[];
  kmv_f32_unit16<KERN, D, NV, RB, GRAD, EXACT>(a, blockIdx.x / a.nsplit, blockIdx.x % a.nsplit,
                                               smem);
}

using Fn = void (*)(Args);

// Instances; *bm receives the rows per workgroup.
template <int KERN, int D, int NB, int NV, bool GRAD, bool EXACT>
Fn inst(int* bm) {
  constexpr int RB = (NB == 2 || GRAD) ? 1 : 2;
  *bm = 32 * RB * kWaves;
  return kmv_f32<KERN, D, NB, NV, RB, GRAD, EXACT>;
}

template <int KERN, int D, int NV, bool GRAD, bool EXACT>
Fn inst16(int* bm) {
  constexpr int RB = (GRAD || D > 8) ? 2 : 4;
  *bm = 16 * RB * kWaves;
  return kmv_f32_16<KERN, D, NV, RB, GRAD, EXACT>;
}

// Column blocking: k ≤ 2 on the VALU; 3 ≤ k ≤ 17 one 16-column MFMA block
// (plus one VALU column for k = 17); otherwise NB blocks of 32 MFMA columns
// and NV ≤ 2 VALU columns.  EXACT instances (k = 1, 2, 16, 17, 32, 33, 34,
// 64) know the V row stride at compile time.
template <int KERN, int D, bool GRAD>
Fn pick_cols(int k, int* bm) {
  if (k == 1) return inst<KERN, D, 0, 1, GRAD, true>(bm);
  if (k == 2) return inst<KERN, D, 0, 2, GRAD, true>(bm);
  if (k == 16) return inst16<KERN, D, 0, GRAD, true>(bm);
  if (k < 16) return inst16<KERN, D, 0, GRAD, false>(bm);
  if (k == 17) return inst16<KERN, D, 1, GRAD, true>(bm);
  if (k == 32) return inst<KERN, D, 1, 0, GRAD, true>(bm);
  if (k < 32) return inst<KERN, D, 1, 0, GRAD, false>(bm);
  if (k == 33) return inst<KERN, D, 1, 1, GRAD, true>(bm);
  if (k == 34) return inst<KERN, D, 1, 2, GRAD, true>(bm);
  if (k == 64) return inst<KERN, D, 2, 0, GRAD, true>(bm);
  return inst<KERN, D, 2, 0, GRAD, false>(bm);
}

template <int KERN, bool GRAD>
Fn pick_d(int d, int k, int* bm) {
  switch (dim_code(d)) {
    case 2: return pick_cols<KERN, 2, GRAD>(k, bm);
    case 3: return pick_cols<KERN, 3, GRAD>(k, bm);
    case 4: return pick_cols<KERN, 4, GRAD>(k, bm);
    case 8: return pick_cols<KERN, 8, GRAD>(k, bm);
    case 16: return pick_cols<KERN, 16, GRAD>(k, bm);
    case 20: return pick_cols<KERN, 20, GRAD>(k, bm);
    default: return pick_cols<KERN, 32, GRAD>(k, bm);
  }
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

// Y = K̂V (Xq null; m = n) or the rectangular Y = f²·k(Xq, X)·V with m rows.
static int run_f32(const Problem& p, int64_t m, const float* Xq, int k, const void* Vin,
                   MatvecOut out, hipStream_t st, int num_cus) {
  const bool grad = out.dl != nullptr || out.df != nullptr;
  const bool cross = Xq != nullptr;
  const int64_t rows = cross ? m : p.n;
  int bm = 0;
  Fn fn;
  if (p.kernel == HIGP_GAUSSIAN)
    fn = grad ? pick_d<HIGP_GAUSSIAN, true>(p.d, k, &bm) : pick_d<HIGP_GAUSSIAN, false>(p.d, k, &bm);
  else
    fn = grad ? pick_d<HIGP_MATERN32, true>(p.d, k, &bm) : pick_d<HIGP_MATERN32, false>(p.d, k, &bm);
  const float xs = (float)coord_scale(p.kernel, HIGP_FP32, p.l);
  const double cl = p.f * p.f * dl_factor(p.kernel, HIGP_FP32, p.l);

  const int P = pad_dim(dim_code(p.d));
  const int64_t nk = p.n * k;   // V elements
  const int64_t mk = rows * k;  // Y elements
  const int64_t jt_count = (p.n + kBJ - 1) / kBJ;
  const int64_t npad = jt_count * kBJ;
  const int64_t mpad = cross ? (m + kBJ - 1) / kBJ * kBJ : 0;
  const int64_t rt_count = (rows + bm - 1) / bm;
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

  // Scratch: prepared points (whole J tiles) and, for a rectangular MatVec,
  // prepared row points; a zero-padded copy of V unless V is 16-byte aligned
  // and n·k is a multiple of 4 (tiles move 16-byte chunks); the partial slots.
  const bool direct_v = (reinterpret_cast<uintptr_t>(Vin) & 15) == 0 && nk % 4 == 0;
  const int64_t nk_pad = (nk + 3) / 4 * 4;
  const size_t xp_bytes = ((size_t)npad * P * 4 + 255) / 256 * 256;
  const size_t v_bytes = direct_v ? 0 : ((size_t)nk_pad * 4 + 255) / 256 * 256;
  const size_t part_bytes = ((size_t)S * mk * 4 + 255) / 256 * 256;
  const size_t xq_bytes = ((size_t)mpad * P * 4 + 255) / 256 * 256;
  void* scratch = nullptr;
  HIGP_TRY(scratch_alloc(&scratch, xp_bytes + v_bytes + part_bytes * (grad ? 2 : 1) + xq_bytes,
                         st));
  char* base = static_cast<char*>(scratch);
  float* Xp = reinterpret_cast<float*>(base);
  float* Xqp = cross ? reinterpret_cast<float*>(base + xp_bytes + v_bytes +
                                                part_bytes * (grad ? 2 : 1))
                     : Xp;
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
    hipLaunchKernelGGL(prep_points_f32, dim3(pb), dim3(256), 0, st, p.n, npad, p.d, P,
                       static_cast<const float*>(p.X), xs, Xp);
    if (cross) {
      const unsigned qb = (unsigned)std::min<int64_t>((mpad * P + 255) / 256, 4096);
      hipLaunchKernelGGL(prep_points_f32, dim3(qb), dim3(256), 0, st, m, mpad, p.d, P, Xq, xs,
                         Xqp);
    }
  }
  Args a{};
  a.Xp = Xp;
  a.Xq = Xqp;
  a.V = V;
  a.part = reinterpret_cast<float*>(base + xp_bytes + v_bytes);
  a.part2 = grad ? reinterpret_cast<float*>(base + xp_bytes + v_bytes + part_bytes) : nullptr;
  a.m = rows;
  a.nk_pad = direct_v ? nk : nk_pad;
  a.jt_count = (int)jt_count;
  a.jt_chunk = jt_chunk;
  a.nsplit = S;
  a.k = k;
  hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(256), lds, st, a);
  const unsigned eb = (unsigned)std::min<int64_t>((mk + 255) / 256, 8LL * num_cus);
  hipLaunchKernelGGL(kmv_f32_epilogue, dim3(eb), dim3(256), 0, st, (const float*)a.part,
                     (const float*)a.part2, cross ? (const float*)nullptr : V,
                     static_cast<float*>(out.kv), static_cast<float*>(out.dl),
                     static_cast<float*>(out.df), mk, S, p.f * p.f, cross ? 0.0 : p.s, cl,
                     2.0 * p.f);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) rc = set_error(HIGP_ERR_HIP, "FP32 MatVec launch failed: %s", hipGetErrorString(e));
  scratch_free(scratch, st);
  return rc;
}

int launch_kmatvec_f32(const Problem& p, int k, const void* V, MatvecOut out, hipStream_t st,
                       int num_cus) {
  if (out.kv && !out.dl && !out.df && kmatvec_f32_sym_applies(p, k))
    return launch_kmatvec_f32_sym(p, k, V, out.kv, st);
  return run_f32(p, p.n, nullptr, k, V, out, st, num_cus);
}

int launch_kmatvec_f32_cross(const Problem& p, int64_t m, const void* Xq, int k, const void* V,
                             void* Y, hipStream_t st, int num_cus) {
  MatvecOut out;
  out.kv = Y;
  return run_f32(p, m, static_cast<const float*>(Xq), k, V, out, st, num_cus);
}

}  // namespace higp
