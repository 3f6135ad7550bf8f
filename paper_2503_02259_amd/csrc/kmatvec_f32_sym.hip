// Symmetric-tiled on-the-fly MatVec for one or two vectors (FP32, VALU).
//
// K̂ is symmetric, so one kernel value k(x_i, x_j) serves output row i (with
// v_j) and output row j (with v_i).  The points are grouped in super blocks
// of 1024 (8 tiles of 128); a workgroup takes one pair (A, B), A ≤ B, of
// super blocks:
//   A < B: every kernel value of the 1024×1024 block is evaluated once and
//          used twice, Y_A += K_AB·V_B and Y_B += K_ABᵀ·V_A;
//   A = B: the block is evaluated in full and used for Y_A only.
// So about n²/2 kernel values are evaluated instead of n².  With one or two
// vectors the contraction is 1–2 FMAs per kernel value on the VALU and the
// distance and exponential dominate, so this nearly halves the work.  (With
// 32 or more vectors the contraction runs on MFMA, whose operand layout puts
// the contracted index on lane/32; using a K tile for Kᵀ would need a
// cross-lane transpose, so the wide path stays unsymmetric.)
//
// Work inside a pair: both blocks are staged in LDS (a point as one float4
// for d ≤ 4, two for d ≤ 8; the latter is taken for one vector only, where it
// measured 1.12–1.20× the full-block form); 256 threads form a
// 16×16 grid of 8×8 micro tiles over each 128×128 tile; row sums stay in
// registers across the 8 column tiles, column sums of each column tile are
// added over the 16 row groups through LDS in a fixed order.  Each pair writes its row and column sums to slots
// of its own; a second kernel adds, for every row, the slots of its super
// block in a fixed order in FP64 and applies f² and s — deterministic, no
// atomics.
#include <algorithm>

#include "kmv_f32_sym.h"

namespace higp {
namespace {

template <int KERN, int D, int K>
__global__ __launch_bounds__(256) void kmv_f32_sym(SymArgs a) {
  __shared__ SymLds<K, sym_nq<D>()> L;
  int A, B;
  item_pair(blockIdx.x, a.ns, A, B);
  if (A == B)
    sym_pair<KERN, D, K, true>(a, A, B, blockIdx.x, L);
  else
    sym_pair<KERN, D, K, false>(a, A, B, blockIdx.x, L);
}

typedef void (*SymFn)(SymArgs);

template <int KERN, int D>
SymFn pick_sym_k(int k) {
  return k == 1 ? kmv_f32_sym<KERN, D, 1> : kmv_f32_sym<KERN, D, 2>;
}

template <int KERN>
SymFn pick_sym(int d, int k) {
  switch (dim_code(d)) {
    case 2: return pick_sym_k<KERN, 2>(k);
    case 3: return pick_sym_k<KERN, 3>(k);
    case 4: return pick_sym_k<KERN, 4>(k);
    case 8: return pick_sym_k<KERN, 8>(k);
    default: return nullptr;  // d > 8: not eligible
  }
}

}  // namespace

// The slots of the block pairs grow as n²/1024 (2·4·k bytes per pair and
// point of a block); above 2 GiB of slots the full-block form is used.
bool kmatvec_f32_sym_applies(const Problem& p, int k) {
  // d = 5..8 stages two float4s per point and fits one workgroup per CU:
  // 1.12× the full-block form for one vector (n = 1e5), no gain for two.
  return sym_eligible(p.n, p.d, k, p.flags, k == 1 ? 8 : 4);
}

int launch_kmatvec_f32_sym(const Problem& p, int k, const void* Vin, void* Y, hipStream_t st) {
  const int ns = (int)((p.n + kSymSuper - 1) / kSymSuper);
  const int64_t items = (int64_t)ns * (ns + 1) / 2;
  if (items > 0x7fffffffLL) return set_error(HIGP_ERR_INVALID_ARG, "n too large");
  const SymFn fn = p.kernel == HIGP_GAUSSIAN ? pick_sym<HIGP_GAUSSIAN>(p.d, k)
                                             : pick_sym<HIGP_MATERN32>(p.d, k);
  if (fn == nullptr) return set_error(HIGP_ERR_INVALID_ARG, "symmetric form needs d <= 8");
  const int P = p.d <= 4 ? 4 : 8;  // floats per prepared point
  const size_t xp_bytes = ((size_t)p.n * P * 4 + 255) / 256 * 256;
  const size_t slot_bytes = (size_t)items * kSymSuper * k * 4;
  void* scratch = nullptr;
  HIGP_TRY(scratch_alloc(&scratch, xp_bytes + 2 * slot_bytes, st));
  char* base = static_cast<char*>(scratch);
  SymArgs a{};
  a.Xp = reinterpret_cast<float*>(base);
  a.V = static_cast<const float*>(Vin);
  a.prow = reinterpret_cast<float*>(base + xp_bytes);
  a.pcol = reinterpret_cast<float*>(base + xp_bytes + slot_bytes);
  a.n = p.n;
  a.ns = ns;
  const float xs = (float)coord_scale(p.kernel, HIGP_FP32, p.l);
  hipLaunchKernelGGL(prep_points_f32, dim3((unsigned)std::min<int64_t>((p.n * P + 255) / 256, 4096)),
                     dim3(256), 0, st, p.n, p.n, p.d, P, static_cast<const float*>(p.X), xs,
                     const_cast<float*>(a.Xp));
  hipLaunchKernelGGL(fn, dim3((unsigned)items), dim3(256), 0, st, a);
  const unsigned fb = (unsigned)std::min<int64_t>((p.n * k + 255) / 256, 4096);
  if (k == 1)
    hipLaunchKernelGGL(kmv_f32_sym_finish<1>, dim3(fb), dim3(256), 0, st, p.n, ns,
                       (const float*)a.prow, (const float*)a.pcol, static_cast<const float*>(Vin),
                       static_cast<float*>(Y), p.f * p.f, p.s);
  else
    hipLaunchKernelGGL(kmv_f32_sym_finish<2>, dim3(fb), dim3(256), 0, st, p.n, ns,
                       (const float*)a.prow, (const float*)a.pcol, static_cast<const float*>(Vin),
                       static_cast<float*>(Y), p.f * p.f, p.s);
  int rc = HIGP_OK;
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    rc = set_error(HIGP_ERR_HIP, "symmetric FP32 MatVec launch failed: %s", hipGetErrorString(e));
  scratch_free(scratch, st);
  return rc;
}

}  // namespace higp
