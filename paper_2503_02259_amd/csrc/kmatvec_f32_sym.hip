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
// Work inside a pair: both blocks are staged in LDS; 256 threads form a
// 16×16 grid of 8×8 micro tiles over each 128×128 tile; row sums stay in
// registers across the 8 column tiles, column sums of each column tile are
// added over the 16 row groups through LDS in a fixed order.  Each pair writes its row and column sums to slots
// of its own; a second kernel adds, for every row, the slots of its super
// block in a fixed order in FP64 and applies f² and s — deterministic, no
// atomics.
#include <algorithm>

#include "kmv_f32_tile.h"

namespace higp {
namespace {

constexpr int64_t kSymMinPoints = 32768;  // below: too few block pairs to fill the chip
constexpr int kSymTile = 128;
constexpr int kSymSub = 8;                     // tiles per super block
constexpr int kSymSuper = kSymTile * kSymSub;  // points per super block
constexpr int kMicro = 8;                      // micro tile edge

struct SymArgs {
  const float* Xp;  // ns·1024 × 4 prepared points (sentinels beyond n)
  const float* V;   // ns·1024 × k, zero beyond n
  float* prow;      // [item][1024][k] row sums (Y_A part)
  float* pcol;      // [item][1024][k] column sums (Y_B part, A < B)
  int ns;           // super blocks
};

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

template <int K>
struct SymLds {
  float4 x[2][kSymSuper];                       // [0]: rows (A), [1]: columns (B)
  float v[2][kSymSuper * K];
  float part[part_bufs<K>()][16][kSymTile * K];  // per-group partial sums
  float colacc[kSymSuper * K];                  // column sums of the pair (B side)
};

template <int K>
__device__ __forceinline__ void stage_block(const SymArgs& a, int64_t p0, float4* x, float* v) {
  for (int e = threadIdx.x; e < kSymSuper; e += 256)
    x[e] = *reinterpret_cast<const float4*>(a.Xp + (p0 + e) * 4);
  for (int e = threadIdx.x; e < kSymSuper * K; e += 256) v[e] = a.V[p0 * K + e];
}

template <int KERN, int D, int K, bool DIAG>
__device__ __forceinline__ void sym_pair(const SymArgs& a, int A, int B, SymLds<K>& L) {
  const int tid = threadIdx.x, tr = tid >> 4, tc = tid & 15;
  const int rs = DIAG ? 1 : 0;  // row side: the column block itself on the diagonal
  for (int e = tid; e < kSymSuper * K; e += 256) L.colacc[e] = 0.0f;
  if (!DIAG) stage_block<K>(a, (int64_t)A * kSymSuper, L.x[0], L.v[0]);
  stage_block<K>(a, (int64_t)B * kSymSuper, L.x[1], L.v[1]);
  __syncthreads();
  float* prow = a.prow + (size_t)blockIdx.x * kSymSuper * K;
  float* pcol = a.pcol + (size_t)blockIdx.x * kSymSuper * K;
  int buf = 0;
  for (int rt = 0; rt < kSymSub; ++rt) {
    float xi[kMicro][D], vi[kMicro][K], ar[kMicro][K];
#pragma unroll
    for (int ii = 0; ii < kMicro; ++ii) {
      const int r = rt * kSymTile + ii * 16 + tr;
      const float4 q = L.x[rs][r];
      xi[ii][0] = q.x;
      if (D > 1) xi[ii][1] = q.y;
      if (D > 2) xi[ii][2] = q.z;
      if (D > 3) xi[ii][3] = q.w;
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
        const float4 q = L.x[1][q0];
        xj[jj][0] = q.x;
        if (D > 1) xj[jj][1] = q.y;
        if (D > 2) xj[jj][2] = q.z;
        if (D > 3) xj[jj][3] = q.w;
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

template <int KERN, int D, int K>
__global__ __launch_bounds__(256) void kmv_f32_sym(SymArgs a) {
  __shared__ SymLds<K> L;
  int A, B;
  item_pair(blockIdx.x, a.ns, A, B);
  if (A == B)
    sym_pair<KERN, D, K, true>(a, A, B, L);
  else
    sym_pair<KERN, D, K, false>(a, A, B, L);
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
    default: return pick_sym_k<KERN, 4>(k);
  }
}

}  // namespace

// The slots of the block pairs grow as n²/1024 (2·4·k bytes per pair and
// point of a block); above 2 GiB of slots the full-block form is used.
bool kmatvec_f32_sym_applies(const Problem& p, int k) {
  if (k > 2 || p.d > 4 || p.n < kSymMinPoints || (p.flags & HIGP_FLAG_NO_SYMMETRIC) != 0)
    return false;
  const int64_t ns = (p.n + kSymSuper - 1) / kSymSuper;
  const int64_t slot_bytes = ns * (ns + 1) / 2 * kSymSuper * k * 4;
  return 2 * slot_bytes <= (int64_t(1) << 31);
}

int launch_kmatvec_f32_sym(const Problem& p, int k, const void* Vin, void* Y, hipStream_t st) {
  const int ns = (int)((p.n + kSymSuper - 1) / kSymSuper);
  const int64_t npad = (int64_t)ns * kSymSuper;
  const int64_t items = (int64_t)ns * (ns + 1) / 2;
  if (items > 0x7fffffffLL) return set_error(HIGP_ERR_INVALID_ARG, "n too large");
  const size_t xp_bytes = ((size_t)npad * 4 * 4 + 255) / 256 * 256;
  const size_t v_bytes = ((size_t)npad * k * 4 + 255) / 256 * 256;
  const size_t slot_bytes = (size_t)items * kSymSuper * k * 4;
  void* scratch = nullptr;
  HIGP_TRY(scratch_alloc(&scratch, xp_bytes + v_bytes + 2 * slot_bytes, st));
  char* base = static_cast<char*>(scratch);
  SymArgs a{};
  a.Xp = reinterpret_cast<float*>(base);
  a.V = reinterpret_cast<float*>(base + xp_bytes);
  a.prow = reinterpret_cast<float*>(base + xp_bytes + v_bytes);
  a.pcol = reinterpret_cast<float*>(base + xp_bytes + v_bytes + slot_bytes);
  a.ns = ns;
  const float xs = (float)coord_scale(p.kernel, HIGP_FP32, p.l);
  hipLaunchKernelGGL(prep_points_f32, dim3((unsigned)std::min<int64_t>((npad * 4 + 255) / 256, 4096)),
                     dim3(256), 0, st, p.n, npad, p.d, 4, static_cast<const float*>(p.X), xs,
                     const_cast<float*>(a.Xp));
  hipLaunchKernelGGL(copy_pad_f32, dim3((unsigned)std::min<int64_t>((npad * k + 255) / 256, 4096)),
                     dim3(256), 0, st, p.n * k, npad * k, static_cast<const float*>(Vin),
                     const_cast<float*>(a.V));
  const SymFn fn = p.kernel == HIGP_GAUSSIAN ? pick_sym<HIGP_GAUSSIAN>(p.d, k)
                                             : pick_sym<HIGP_MATERN32>(p.d, k);
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
