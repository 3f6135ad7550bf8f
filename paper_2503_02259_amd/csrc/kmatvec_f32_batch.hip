// Batched FP32 on-the-fly MatVec of many independent problems (continuous-
// batching serving), built on the tile unit of the single-problem MatVec and
// (for large single-column problems) on the symmetric block-pair unit.
#include <algorithm>
#include <atomic>
#include <vector>

#include "kmv_f32_sym.h"

namespace higp {
namespace {

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

// Column kinds of a batched launch: 0 = 18 ≤ k ≤ 32 through one 32-column
// MFMA block; 1 / 2 = k = 1 / 2 on the VALU only (a CG-only round); 4 / 5 =
// 3 ≤ k ≤ 16 / k = 17 through one 16-column MFMA block (+ one VALU column),
// the Lanczos rounds of a request with 16 probes.  (Kind 3, the symmetric
// block pairs, has its own kernel below.)  The VALU kinds take four 32-row
// blocks per wave (more independent work per LDS read of a point) and
// reserve LDS only for the columns they carry, so more workgroups fit on a
// CU.
template <int KIND> struct KindCols;
template <> struct KindCols<0> {
  static constexpr int NB = 1, NV = 0, RB = 2, KMAX = 32;
  static constexpr bool W16 = false, EXACT = false;
};
template <> struct KindCols<1> {
  static constexpr int NB = 0, NV = 1, RB = 4, KMAX = 1;
  static constexpr bool W16 = false, EXACT = true;
};
template <> struct KindCols<2> {
  static constexpr int NB = 0, NV = 2, RB = 4, KMAX = 2;
  static constexpr bool W16 = false, EXACT = true;
};
template <> struct KindCols<4> {
  static constexpr int NB = 0, NV = 0, RB = 4, KMAX = 16;
  static constexpr bool W16 = true, EXACT = false;
};
template <> struct KindCols<5> {
  static constexpr int NB = 0, NV = 1, RB = 4, KMAX = 17;
  static constexpr bool W16 = true, EXACT = true;
};

template <int KIND>
constexpr int64_t kind_rows() {  // rows per work unit
  return (KindCols<KIND>::W16 ? 16LL : 32LL) * KindCols<KIND>::RB * kWaves;
}

template <int KIND>
constexpr size_t kind_lds() {  // X tile (8 floats a point) + V tile, double-buffered
  return (size_t)2 * kBJ * (8 + KindCols<KIND>::KMAX) * 4;
}

template <int KERN, int KIND, int D>
__device__ __forceinline__ void batch_unit_d(const Args& a, int64_t rt, int split, float* smem) {
  constexpr int NB = KindCols<KIND>::NB, NV = KindCols<KIND>::NV, RB = KindCols<KIND>::RB;
  constexpr bool EX = KindCols<KIND>::EXACT;
  if constexpr (KindCols<KIND>::W16)
    kmv_f32_unit16<KERN, D, NV, RB, false, EX>(a, rt, split, smem);
  else
    kmv_f32_unit<KERN, D, NB, NV, RB, false, EX>(a, rt, split, smem);
}

template <int KERN, int KIND>
__device__ __forceinline__ void batch_unit(const Args& a, int dcode, int64_t rt, int split,
                                           float* smem) {
  if (dcode == 2) batch_unit_d<KERN, KIND, 2>(a, rt, split, smem);
  else if (dcode == 3) batch_unit_d<KERN, KIND, 3>(a, rt, split, smem);
  else if (dcode == 4) batch_unit_d<KERN, KIND, 4>(a, rt, split, smem);
  else batch_unit_d<KERN, KIND, 8>(a, rt, split, smem);
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

// Kind 3: single-column problems large enough for the symmetric form; a
// work unit is one block pair (A ≤ B) of one problem (kmv_f32_sym.h).  A
// problem's pairs and their slots depend only on its own n, so its result
// does not depend on the rest of the batch either.
struct SymJob {
  SymArgs a;
  int64_t first_unit;  // units of earlier jobs of the same launch
  int kernel;
  int dcode;           // 2, 3 or 4 (one float4 per point), 8 (two)
};

// NQ = 1: problems with d ≤ 4; NQ = 2: d = 5..8 (a launch of their own,
// since the staged points take twice the LDS).
template <int KERN, bool DIAG, int NQ>
__device__ __forceinline__ void sym_unit(const SymArgs& a, int dcode, int A, int B, int64_t item,
                                         SymLds<1, NQ>& L) {
  if constexpr (NQ == 2) {
    sym_pair<KERN, 8, 1, DIAG>(a, A, B, item, L);
  } else {
    if (dcode == 2) sym_pair<KERN, 2, 1, DIAG>(a, A, B, item, L);
    else if (dcode == 3) sym_pair<KERN, 3, 1, DIAG>(a, A, B, item, L);
    else sym_pair<KERN, 4, 1, DIAG>(a, A, B, item, L);
  }
}

template <int NQ>
__global__ __launch_bounds__(256) void kmv_f32_batch_sym(const SymJob* __restrict__ jobs,
                                                         int njobs, int64_t total,
                                                         unsigned long long* counter) {
  __shared__ SymLds<1, NQ> L;
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
    const SymArgs a = jobs[lo].a;
    const int dcode = jobs[lo].dcode;
    const int64_t item = u - jobs[lo].first_unit;
    int A, B;
    item_pair((int)item, a.ns, A, B);
    if (jobs[lo].kernel == HIGP_GAUSSIAN) {
      if (A == B) sym_unit<HIGP_GAUSSIAN, true, NQ>(a, dcode, A, B, item, L);
      else sym_unit<HIGP_GAUSSIAN, false, NQ>(a, dcode, A, B, item, L);
    } else {
      if (A == B) sym_unit<HIGP_MATERN32, true, NQ>(a, dcode, A, B, item, L);
      else sym_unit<HIGP_MATERN32, false, NQ>(a, dcode, A, B, item, L);
    }
    __syncthreads();
  }
}

}  // namespace


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
  return (size_t)npad * pad_dim(dim_code(d)) * 4;
}

int prepare_points_f32(const Problem& p, float* Xp, hipStream_t st) {
  const int P = pad_dim(dim_code(p.d));
  const int64_t npad = (p.n + kBJ - 1) / kBJ * kBJ;
  const float xs = (float)coord_scale(p.kernel, HIGP_FP32, p.l);
  const unsigned pb = (unsigned)std::min<int64_t>((npad * P + 255) / 256, 4096);
  hipLaunchKernelGGL(prep_points_f32, dim3(pb), dim3(256), 0, st, p.n, npad, p.d, P,
                     static_cast<const float*>(p.X), xs, Xp);
  return hipGetLastError() == hipSuccess ? HIGP_OK : set_error(HIGP_ERR_HIP, "prep launch failed");
}

namespace {

// Resident 256-thread workgroups per CU of a persistent kernel: a property of
// the kernel and the architecture, so it is computed once per process (the
// cache is atomic: launches may come from several host threads).
int resident_blocks(const void* fn, size_t lds, std::atomic<int>& cache) {
  const int v = cache.load(std::memory_order_relaxed);
  if (v > 0) return v;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 256, lds) != hipSuccess || nb < 1)
    nb = 1;
  cache.store(nb, std::memory_order_relaxed);
  return nb;
}

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
  static std::atomic<int> cache{0};
  const int bpc = resident_blocks(reinterpret_cast<const void*>(kmv_f32_batch<KIND>), lds, cache);
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

template <int NQ>
int launch_batch_sym(const std::vector<const BatchMatvec*>& src, hipStream_t st, int num_cus) {
  const int count = (int)src.size();
  if (count == 0) return HIGP_OK;
  std::vector<SymJob> hj(count);
  std::vector<size_t> slot_off(count);
  int64_t total = 0;
  size_t slots = 0;  // floats per slot array (rows and columns each)
  for (int i = 0; i < count; ++i) {
    const BatchMatvec& J = *src[i];
    const int ns = (int)((J.n + kSymSuper - 1) / kSymSuper);
    const int64_t items = (int64_t)ns * (ns + 1) / 2;
    SymJob b{};
    b.a.Xp = J.Xp;
    b.a.V = J.V;
    b.a.n = J.n;
    b.a.ns = ns;
    b.first_unit = total;
    b.kernel = J.kernel;
    b.dcode = J.d <= 2 ? 2 : (J.d == 3 ? 3 : (J.d == 4 ? 4 : 8));
    hj[i] = b;
    slot_off[i] = slots;
    total += items;
    slots += (size_t)items * kSymSuper;
  }
  const size_t jobs_bytes = ((size_t)count * sizeof(SymJob) + 255) / 256 * 256;
  void* mem = nullptr;
  HIGP_TRY(scratch_alloc(&mem, jobs_bytes + 256 + 2 * slots * 4, st));
  char* base = static_cast<char*>(mem);
  SymJob* djobs = reinterpret_cast<SymJob*>(base);
  unsigned long long* counter = reinterpret_cast<unsigned long long*>(base + jobs_bytes);
  float* prow = reinterpret_cast<float*>(base + jobs_bytes + 256);
  float* pcol = prow + slots;
  for (int i = 0; i < count; ++i) {
    hj[i].a.prow = prow + slot_off[i];
    hj[i].a.pcol = pcol + slot_off[i];
  }
  int rc = HIGP_OK;
  if (hipMemcpyAsync(djobs, hj.data(), count * sizeof(SymJob), hipMemcpyHostToDevice, st) !=
          hipSuccess ||
      hipMemsetAsync(counter, 0, 8, st) != hipSuccess)
    rc = set_error(HIGP_ERR_HIP, "batch setup failed");
  static std::atomic<int> cache{0};
  const int bpc = resident_blocks(reinterpret_cast<const void*>(kmv_f32_batch_sym<NQ>), 0, cache);
  if (rc == HIGP_OK) {
    const int64_t grid = std::min<int64_t>(total, (int64_t)num_cus * bpc);
    hipLaunchKernelGGL(kmv_f32_batch_sym<NQ>, dim3((unsigned)grid), dim3(256), 0, st,
                       (const SymJob*)djobs, count, total, counter);
    for (int i = 0; i < count; ++i) {
      const BatchMatvec& J = *src[i];
      const unsigned fb = (unsigned)std::min<int64_t>((J.n + 255) / 256, 2LL * num_cus);
      hipLaunchKernelGGL(kmv_f32_sym_finish<1>, dim3(fb), dim3(256), 0, st, J.n, hj[i].a.ns,
                         (const float*)hj[i].a.prow, (const float*)hj[i].a.pcol, J.V, J.Y,
                         J.f * J.f, J.s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
      rc = set_error(HIGP_ERR_HIP, "batched symmetric MatVec launch failed: %s",
                     hipGetErrorString(e));
  }
  scratch_free(mem, st);
  return rc;
}

}  // namespace

int launch_kmatvec_f32_batch(const BatchMatvec* jobs, int count, hipStream_t st, int num_cus) {
  if (count <= 0) return HIGP_OK;
  constexpr int kKinds = 6;  // kind 3 (symmetric) is collected separately
  std::vector<BatchJob> hj[kKinds];
  std::vector<const BatchMatvec*> src[kKinds];
  std::vector<const BatchMatvec*> sym[2];  // d ≤ 4, d = 5..8
  int64_t total[kKinds] = {0, 0, 0, 0, 0, 0};
  size_t part_elems[kKinds] = {0, 0, 0, 0, 0, 0};
  const int64_t rows_of[kKinds] = {kind_rows<0>(), kind_rows<1>(), kind_rows<2>(), 0,
                                   kind_rows<4>(), kind_rows<5>()};
  for (int i = 0; i < count; ++i) {
    const BatchMatvec& J = jobs[i];
    if (J.k < 1 || J.k > 32)
      return set_error(HIGP_ERR_UNSUPPORTED, "batched MatVec supports 1 <= k <= 32");
    if (J.k == 1 && sym_eligible(J.n, J.d, 1, J.flags, 8)) {
      sym[J.d <= 4 ? 0 : 1].push_back(&J);
      continue;
    }
    const int kind = J.k == 1 ? 1 : J.k == 2 ? 2 : J.k <= 16 ? 4 : J.k == 17 ? 5 : 0;
    const int S = batch_splits(J.n);
    const int64_t jt = (J.n + kBJ - 1) / kBJ;
    const int64_t bm = rows_of[kind];
    const int64_t rt = (J.n + bm - 1) / bm;
    BatchJob b{};
    b.a.Xp = J.Xp;
    b.a.Xq = J.Xp;
    b.a.V = J.V;
    b.a.m = J.n;
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
  HIGP_TRY(launch_batch_kind<4>(hj[4], src[4], total[4], part_elems[4], st, num_cus));
  HIGP_TRY(launch_batch_kind<5>(hj[5], src[5], total[5], part_elems[5], st, num_cus));
  HIGP_TRY(launch_batch_sym<1>(sym[0], st, num_cus));
  HIGP_TRY(launch_batch_sym<2>(sym[1], st, num_cus));
  return HIGP_OK;
}

}  // namespace higp
