// BF16 precision forms of the on-the-fly kernel MatVec on gfx950: distances in
// FP32, the kernel tile and V rounded to bfloat16 (round to nearest even) and
// multiplied by v_mfma_f32_32x32x16_bf16 with FP32 accumulation.
//
// Split form (SPLIT = true): K and V are each carried as a pair hi + lo of
// bfloat16 values, hi = RNE(x), lo = RNE(x − hi), which holds 16 significant
// bits; the product takes the three leading terms K_hi·V_hi + K_hi·V_lo +
// K_lo·V_hi (three MFMAs instead of one), leaving a relative error of order
// 2⁻¹⁶ instead of 2⁻⁸.  The single form makes K̂ indefinite once the bfloat16
// rounding noise of a tight cluster of m points (norm ≈ 2⁻⁸·√m) exceeds s;
// the split form pushes that limit out by a factor of 2⁸.
//
// Squared distances come from the matrix core too.  With augmented vectors
//   a_i = (x̃_i, ‖x̃_i‖², 1),   b_j = (−2·x̃_j, 1, ‖x̃_j‖²)      (length d + 2)
// a_i·b_j = ‖x̃_i − x̃_j‖², so a 32(j)×32(i) distance block is (d+2)/2 FP32
// 32×32×2 MFMAs and needs no VALU at all; at d = 8 this replaces 16 VALU
// operations per pair.  The expansion loses ~u·‖x̃‖² absolutely, so the points
// are first centred on their mean (the kernel depends on differences only),
// which for points filling a box shrinks ‖x̃‖² about fourfold; what remains is
// below the bfloat16 rounding of the single form and of the order of the
// split form's 2⁻¹⁶.
//
// The distance accumulator leaves lane l holding column i = l%32 and the 16
// rows j = 8(r/4) + 4(l/32) + r%4 (r = 0..15).  The contraction needs lane l
// to supply K[i][·] for its own row i = l%32 — which it already has — for 8 J
// indices per 32×32×16 MFMA.  The sum over j does not care about order, so the
// two MFMAs of a 32-point block take registers r = 0..7 and r = 8..15 as their
// K operand, and V is laid out once per MatVec (bf16, zero-padded columns) in
// exactly that permuted row order, 16 bytes per lane per MFMA.
//
// Structure otherwise follows the FP32 kernel: 128-point J tiles copied
// global → LDS directly and double-buffered, XCD-aware split-J with
// deterministic partial sums, FP32 accumulation inside a tile and FP64 running
// totals across tiles.
#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <unordered_map>

#include "bufload.h"
#include "kvalue.h"
#include "reduce.h"

namespace higp {
namespace {

constexpr int kWaves = 4;
constexpr int kBJ = 128;       // J points per tile
constexpr float kFarSq = 1e30f;  // squared norm of a sentinel point: exp2 → 0

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Column means of X (n×d) → ctr[0..d), summed in FP64 in a fixed order.
__global__ __launch_bounds__(kRedThreads) void point_mean(int64_t n, int d, int64_t chunk,
                                                          const float* __restrict__ X,
                                                          float* __restrict__ ctr, double* work,
                                                          unsigned* counter) {
  __shared__ double sh[kRedThreads];
  const ColLanes L = col_lanes(d);
  const int c = L.c;
  const int r0 = L.r0;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  double acc = 0.0;
  if (c < d)
    for (int64_t i = beg + r0; i < end; i += L.step) acc += (double)X[i * d + c];
  (void)block_colsum_finish(acc, d, work, counter, sh,
                            [&](int col, double tot) { ctr[col] = (float)(tot / (double)n); });
}

// a1 for the BF16 forms.  XA[i][0..DA): a_i; XB tile jt: [DA][kBJ] (SoA) of b_j,
// with sentinel points beyond n.  x̃ = (x − ctr)·xs.
template <int DA>
__global__ void prep_points_bf16(int64_t n, int64_t npad, int d, const float* __restrict__ X,
                                 const float* __restrict__ ctr, float xs, float* __restrict__ XA,
                                 float* __restrict__ XB) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npad;
       i += (int64_t)gridDim.x * blockDim.x) {
    float x[DA];
    float nrm = 0.0f;
#pragma unroll
    for (int c = 0; c < DA; ++c) {
      x[c] = (i < n && c < d) ? (X[i * d + c] - ctr[c]) * xs : 0.0f;
      nrm = fmaf(x[c], x[c], nrm);
    }
    const int64_t jt = i / kBJ, jj = i % kBJ;
    float* b = XB + jt * DA * kBJ + jj;
#pragma unroll
    for (int c = 0; c < DA; ++c) {
      float bv;
      if (c < d) bv = -2.0f * x[c];
      else if (c == d) bv = 1.0f;
      else if (c == d + 1) bv = i < n ? nrm : kFarSq;
      else bv = 0.0f;
      b[c * kBJ] = bv;
    }
    if (i < n) {
#pragma unroll
      for (int c = 0; c < DA; ++c) {
        float av;
        if (c < d) av = x[c];
        else if (c == d) av = nrm;
        else if (c == d + 1) av = 1.0f;
        else av = 0.0f;
        XA[i * DA + c] = av;
      }
    }
  }
}

// V (n×k, float) → bf16 in the contraction's operand order.  Within J tile jt
// and 32-point block jb, MFMA q ∈ {0,1}, column block b, half h and column c,
// 8 consecutive bf16 hold rows j = jb·32 + 16q + 8(e/4) + 4h + e%4, e = 0..7.
// Layout: [jt][jb][q][b][h][c][e]; rows ≥ n and columns ≥ k are 0.  With VL
// non-null the lo parts RNE(v − hi) go there in the same layout.
__global__ void prep_v_bf16(int64_t n, int k, int nb, int64_t npad, const float* __restrict__ V,
                            __bf16* __restrict__ VB, __bf16* __restrict__ VL) {
  const int64_t total = npad * nb * 32;  // one thread per (row, padded column)
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = t / (nb * 32);
    const int col = (int)(t % (nb * 32));
    const int b = col / 32, c = col % 32;
    const int64_t jt = j / kBJ;
    const int jl = (int)(j % kBJ);
    const int jb = jl / 32, jr = jl % 32;
    const int q = jr / 16, w = jr % 16;        // w = 8(e/4) + 4h + e%4
    const int h = (w / 4) % 2;
    const int e = (w / 8) * 4 + w % 4;
    const float v = (j < n && col < k) ? V[j * k + col] : 0.0f;
    const int64_t o = ((((((jt * 4 + jb) * 2 + q) * nb + b) * 2 + h) * 32 + c) * 8) + e;
    const __bf16 hi = (__bf16)v;
    VB[o] = hi;
    if (VL) VL[o] = (__bf16)(v - (float)hi);
  }
}

struct Args {
  const float* XA;  // n×DA
  const float* XB;  // [jt][DA][kBJ]
  const __bf16* VB; // [jt][4][2][NB][2][32][8]
  const __bf16* VL; // lo parts, same layout (split form only)
  float* part;      // partials [S][n][k]
  int64_t n;
  int jt_count, jt_chunk, nsplit, k;
};

template <int KERN, int DA, int NB, bool SPLIT>
__global__ __launch_bounds__(256) void kmv_bf16(Args a) {
  constexpr int BM = 32 * kWaves;
  constexpr int XT = DA * kBJ;            // floats per X tile
  constexpr int VT = kBJ * NB * 32;       // bf16 per V tile (per part)
  constexpr int VP = SPLIT ? 2 : 1;       // V parts: hi (and lo)
  extern __shared__ __attribute__((aligned(16))) float smem[];
  float* Xs = smem;                                        // [2][DA][kBJ]
  __bf16* Vs = reinterpret_cast<__bf16*>(smem + 2 * XT);   // [2][VP][VT]

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int half = lane >> 5;
  const int l32 = lane & 31;
  const int split = blockIdx.x % a.nsplit;
  const int64_t rt = blockIdx.x / a.nsplit;
  const int jt_beg = split * a.jt_chunk;
  const int jt_end = jt_beg + a.jt_chunk < a.jt_count ? jt_beg + a.jt_chunk : a.jt_count;
  const int k = a.k;

  // B operand of the distance MFMAs: a_i[2t + half] for this lane's row i.
  const int64_t irow = rt * BM + wave * 32 + l32;
  float ai[DA / 2];
#pragma unroll
  for (int t = 0; t < DA / 2; ++t) ai[t] = irow < a.n ? a.XA[irow * DA + 2 * t + half] : 0.0f;

  f32x16 acc[NB];
  double tot[NB][16];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    acc[b] = f32x16{0};
#pragma unroll
    for (int r = 0; r < 16; ++r) tot[b][r] = 0.0;
  }

  auto gload = [&](int jt, int buf) {
    char* xs = reinterpret_cast<char*>(Xs + buf * XT);
    char* vs = reinterpret_cast<char*>(Vs + buf * VP * VT);
    const __amdgpu_buffer_rsrc_t rx = make_rsrc(a.XB + (int64_t)jt * XT, (int64_t)XT * 4);
    for (int m = wave * 64; m < XT / 4; m += 256)
      if (m + lane < XT / 4)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (lds_void_t*)(xs + 16 * m), 16,
                                                 16 * (m + lane), 0, 0, 0);
#pragma unroll
    for (int part = 0; part < VP; ++part) {
      const __bf16* src = part == 0 ? a.VB : a.VL;
      char* dst = vs + part * VT * 2;
      const __amdgpu_buffer_rsrc_t rv = make_rsrc(src + (int64_t)jt * VT, (int64_t)VT * 2);
      for (int m = wave * 64; m < VT / 8; m += 256)
        if (m + lane < VT / 8)
          __builtin_amdgcn_raw_ptr_buffer_load_lds(rv, (lds_void_t*)(dst + 16 * m), 16,
                                                   16 * (m + lane), 0, 0, 0);
    }
  };

  int cur = 0;
  if (jt_beg < jt_end) gload(jt_beg, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  for (int jt = jt_beg; jt < jt_end; ++jt) {
    if (jt + 1 < jt_end) gload(jt + 1, cur ^ 1);
    const float* xs = Xs + cur * XT;
    const bf16x8* vs = reinterpret_cast<const bf16x8*>(Vs + cur * VP * VT);
    const bf16x8* vl = vs + VT / 8;  // lo parts (split form)
#pragma unroll 1
    for (int jb = 0; jb < kBJ / 32; ++jb) {
      // distances r̃²(i = l%32, j = jb·32 + 8(r/4) + 4·half + r%4)
      f32x16 dist = f32x16{0};
#pragma unroll
      for (int t = 0; t < DA / 2; ++t) {
        const float bj = xs[(2 * t + half) * kBJ + jb * 32 + l32];
        dist = __builtin_amdgcn_mfma_f32_32x32x2f32(bj, ai[t], dist, 0, 0, 0);
      }
      bf16x8 kb[2], kl[2];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        float kv, kg;
        const float r2 = KERN == HIGP_MATERN32 ? fmaxf(dist[r], 0.0f) : dist[r];
        kval_f32<KERN, false>(r2, kv, kg);
        const __bf16 h = (__bf16)kv;
        kb[r >> 3][r & 7] = h;
        if (SPLIT) kl[r >> 3][r & 7] = (__bf16)(kv - (float)h);
      }
#pragma unroll
      for (int q = 0; q < 2; ++q)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int o = (((jb * 2 + q) * NB + b) * 2 + half) * 32 + l32;
          const bf16x8 vb = vs[o];
          acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kb[q], vb, acc[b], 0, 0, 0);
          if (SPLIT) {
            acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kb[q], vl[o], acc[b], 0, 0, 0);
            acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kl[q], vb, acc[b], 0, 0, 0);
          }
        }
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int r = 0; r < 16; ++r) tot[b][r] += (double)acc[b][r];
      acc[b] = f32x16{0};
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    cur ^= 1;
  }

  // Partials of this chunk (rows i = 8(r/4) + 4·half + r%4 of the wave).
  const int64_t nk = a.n * k;
  float* q1 = a.part + (int64_t)split * nk;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int col = b * 32 + l32;
    if (col >= k) continue;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t row = rt * BM + wave * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
      if (row < a.n) q1[row * k + col] = (float)tot[b][r];
    }
  }
}

__global__ void kmv_bf16_epilogue(const float* __restrict__ P1, const float* __restrict__ V,
                                  float* __restrict__ Y, int64_t count, int nsplit, double f2,
                                  double s) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s1 = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) s1 += (double)P1[sp * count + e];
    Y[e] = (float)(f2 * s1 + s * (double)V[e]);
  }
}

using Fn = void (*)(Args);

template <int KERN, int DA, bool SPLIT>
Fn pick_nb(int nb) {
  return nb == 1 ? kmv_bf16<KERN, DA, 1, SPLIT> : kmv_bf16<KERN, DA, 2, SPLIT>;
}

template <int KERN, bool SPLIT>
Fn pick_da(int da, int nb) {
  if (da == 4) return pick_nb<KERN, 4, SPLIT>(nb);
  if (da == 6) return pick_nb<KERN, 6, SPLIT>(nb);
  if (da == 8) return pick_nb<KERN, 8, SPLIT>(nb);
  return pick_nb<KERN, 10, SPLIT>(nb);
}

template <int KERN>
Fn pick(int da, int nb, bool split) {
  return split ? pick_da<KERN, true>(da, nb) : pick_da<KERN, false>(da, nb);
}

int blocks_per_cu(Fn fn, size_t lds) {
  static std::mutex mu;
  static std::unordered_map<uint64_t, int> cache;
  int dev = 0;
  (void)hipGetDevice(&dev);
  const uint64_t key = reinterpret_cast<uint64_t>(fn) ^ ((uint64_t)lds << 40) ^ ((uint64_t)dev << 60);
  std::lock_guard<std::mutex> g(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(fn), 256,
                                                   lds) != hipSuccess ||
      nb < 1)
    nb = 1;
  cache[key] = nb;
  return nb;
}

}  // namespace

int launch_kmatvec_bf16(const Problem& p, int k, const void* Vin, MatvecOut out, hipStream_t st,
                        int num_cus, bool split) {
  if (out.dl || out.df)
    return set_error(HIGP_ERR_UNSUPPORTED, "derivative MatVecs are not provided in the BF16 forms");
  if (p.d > 8) return set_error(HIGP_ERR_UNSUPPORTED, "the BF16 forms take d <= 8");
  const int da = ((p.d + 2) + 1) / 2 * 2;  // augmented length, even
  const int nb = k <= 32 ? 1 : 2;
  Fn fn = p.kernel == HIGP_GAUSSIAN ? pick<HIGP_GAUSSIAN>(da, nb, split)
                                    : pick<HIGP_MATERN32>(da, nb, split);
  const float xs = (float)coord_scale(p.kernel, HIGP_FP32, p.l);
  const int bm = 32 * kWaves;
  const int64_t nk = p.n * k;
  const int64_t jt_count = (p.n + kBJ - 1) / kBJ;
  const int64_t npad = jt_count * kBJ;
  const int64_t rt_count = (p.n + bm - 1) / bm;
  const size_t xt = (size_t)da * kBJ * 4, vt = (size_t)kBJ * nb * 32 * 2 * (split ? 2 : 1);
  const size_t lds = 2 * (xt + vt);
  if (lds > 65536 &&
      hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return set_error(HIGP_ERR_HIP, "cannot reserve %zu bytes of LDS", lds);
  const int64_t slots = (int64_t)num_cus * blocks_per_cu(fn, lds);
  int S = 1;
  while (S < 64 && rt_count * S < 8 * slots && jt_count >= 4LL * S) S *= 2;
  const int jt_chunk = (int)((jt_count + S - 1) / S);
  const int64_t grid = rt_count * S;
  if (grid > 0x7fffffffLL) return set_error(HIGP_ERR_INVALID_ARG, "n too large");

  const size_t xa_bytes = ((size_t)p.n * da * 4 + 255) / 256 * 256;
  const size_t xb_bytes = ((size_t)npad * da * 4 + 255) / 256 * 256;
  const size_t vb_bytes = ((size_t)npad * nb * 32 * 2 + 255) / 256 * 256;  // per part
  const size_t part_bytes = ((size_t)S * nk * 4 + 255) / 256 * 256;
  const RedGrid rg = red_grid(p.n);
  const size_t ctr_bytes = 256 + 256 + ((size_t)rg.blocks * 64 * 8 + 255) / 256 * 256;
  void* scratch = nullptr;
  const size_t vparts = split ? 2 : 1;
  HIGP_TRY(scratch_alloc(&scratch, xa_bytes + xb_bytes + vparts * vb_bytes + part_bytes + ctr_bytes,
                         st));
  char* base = static_cast<char*>(scratch);
  float* XA = reinterpret_cast<float*>(base);
  float* XB = reinterpret_cast<float*>(base + xa_bytes);
  __bf16* VB = reinterpret_cast<__bf16*>(base + xa_bytes + xb_bytes);
  __bf16* VL = split ? reinterpret_cast<__bf16*>(base + xa_bytes + xb_bytes + vb_bytes) : nullptr;
  float* part = reinterpret_cast<float*>(base + xa_bytes + xb_bytes + vparts * vb_bytes);
  char* cbase = base + xa_bytes + xb_bytes + vparts * vb_bytes + part_bytes;
  float* ctr = reinterpret_cast<float*>(cbase);
  unsigned* counter = reinterpret_cast<unsigned*>(cbase + 256);
  double* work = reinterpret_cast<double*>(cbase + 512);
  const float* X = static_cast<const float*>(p.X);
  const float* V = static_cast<const float*>(Vin);
  if (hipMemsetAsync(counter, 0, 4, st) != hipSuccess) {
    scratch_free(scratch, st);
    return set_error(HIGP_ERR_HIP, "hipMemsetAsync failed");
  }
  hipLaunchKernelGGL(point_mean, dim3(rg.blocks), dim3(kRedThreads), 0, st, p.n, p.d, rg.chunk, X,
                     ctr, work, counter);
  const unsigned pb = (unsigned)std::min<int64_t>((npad + 255) / 256, 4096);
  switch (da) {
    case 4: hipLaunchKernelGGL(prep_points_bf16<4>, dim3(pb), dim3(256), 0, st, p.n, npad, p.d, X, (const float*)ctr, xs, XA, XB); break;
    case 6: hipLaunchKernelGGL(prep_points_bf16<6>, dim3(pb), dim3(256), 0, st, p.n, npad, p.d, X, (const float*)ctr, xs, XA, XB); break;
    case 8: hipLaunchKernelGGL(prep_points_bf16<8>, dim3(pb), dim3(256), 0, st, p.n, npad, p.d, X, (const float*)ctr, xs, XA, XB); break;
    default: hipLaunchKernelGGL(prep_points_bf16<10>, dim3(pb), dim3(256), 0, st, p.n, npad, p.d, X, (const float*)ctr, xs, XA, XB); break;
  }
  const unsigned vbk = (unsigned)std::min<int64_t>((npad * nb * 32 + 255) / 256, 4096);
  hipLaunchKernelGGL(prep_v_bf16, dim3(vbk), dim3(256), 0, st, p.n, k, nb, npad, V, VB, VL);
  Args a{};
  a.XA = XA;
  a.XB = XB;
  a.VB = VB;
  a.VL = VL;
  a.part = part;
  a.n = p.n;
  a.jt_count = (int)jt_count;
  a.jt_chunk = jt_chunk;
  a.nsplit = S;
  a.k = k;
  hipLaunchKernelGGL(fn, dim3((unsigned)grid), dim3(256), lds, st, a);
  const unsigned eb = (unsigned)std::min<int64_t>((nk + 255) / 256, 8LL * num_cus);
  hipLaunchKernelGGL(kmv_bf16_epilogue, dim3(eb), dim3(256), 0, st, (const float*)part, V,
                     static_cast<float*>(out.kv), nk, S, p.f * p.f, p.s);
  int rc = HIGP_OK;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) rc = set_error(HIGP_ERR_HIP, "BF16 MatVec launch failed: %s", hipGetErrorString(e));
  scratch_free(scratch, st);
  return rc;
}

}  // namespace higp
