// FP64 on-the-fly kernel MatVec (and derivative MatVec) with
// v_mfma_f64_16x16x4f64 on gfx950.
//
// The plain-method form: distances, kernel values (software exp), products
// and sums all in double.  Each workgroup owns a row tile I of 64 rows and a
// chunk of the J range (split-J, so that small n still fills the GPU); J
// tiles of X and V are staged through LDS; each lane forms one kernel value
// per MFMA step in the A-operand slot.  Split partials are added in a fixed
// order by an epilogue kernel (deterministic, no atomics).
#include <algorithm>

#include "bufload.h"
#include "kvalue.h"

namespace higp {
namespace {

constexpr int kWaves = 4;

template <typename T>
struct KArgs {
  const T* Xp;  // npad×P prepared J (column) points: x·xs, rows ≥ n far-away sentinels
  const T* Xq;  // m×d row-major: the row points (X for a square MatVec), unscaled
  const T* V;   // n×k row-major, 16-byte aligned, readable up to nk_pad elements
  const T* sV;  // V for the s·V term (null for a rectangular MatVec)
  T* o1;        // S==1: K̂V (or null); S>1: partial Σ k·v, S×m×k
  T* o2;        // S==1: ∂K̂/∂l·V (or null); S>1: partial Σ k_l·v (GRAD only)
  T* o3;        // S==1: ∂K̂/∂f·V (or null); unused when S>1
  int64_t n;    // J points
  int64_t m;    // rows
  int64_t jchunk;  // J points per split (multiple of the J tile)
  int64_t nk_pad;  // readable elements of V (n·k rounded up to whole 16-byte chunks)
  int k, d, nsplit;
  T xs;          // coordinate pre-scale
  T f2, s;       // K̂ = f²K + sI (epilogue, S==1)
  T cl, cf;      // ∂K̂/∂l = cl·Σk_l v, ∂K̂/∂f = cf·Σk v (epilogue, S==1)
};

constexpr double kFar64 = 1e18;  // squared distance ~1e36: exp underflows to exactly 0

// Padded storage width of an FP64 point with D coordinates (32-byte rows for
// D ≤ 4, then multiples of 4 doubles).
__host__ __device__ constexpr int pad_dim64(int d) {
  return d <= 4 ? 4 : (d <= 8 ? 8 : (d + 3) / 4 * 4);
}

// a1: x̃ = x·xs padded to P doubles; rows n..npad−1 are far-away sentinels.
__global__ void prep_points_f64(int64_t n, int64_t npad, int d, int P,
                                const double* __restrict__ X, double xs,
                                double* __restrict__ Xp) {
  const int64_t count = npad * P;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / P;
    const int c = (int)(e % P);
    Xp[e] = i >= n ? kFar64 : (c < d ? X[i * d + c] * xs : 0.0);
  }
}

// dst[0..count_pad) = src[0..count) followed by zeros.
__global__ void copy_pad_f64(int64_t count, int64_t count_pad, const double* __restrict__ src,
                             double* __restrict__ dst) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count_pad;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = e < count ? src[e] : 0.0;
}

// ---------------------------------------------------------------------------
// FP64: v_mfma_f64_16x16x4f64.  A wave owns 16 rows; per MFMA each lane
// supplies K[i0 + lane%16][j0 + lane/16] (4 J points per step); NB blocks of
// 16 columns.  Output layout: lane l, register r holds row l/16 + 4r,
// column l%16.  With NV = 1 one more column (k = 16·NB + 1, e.g. y plus 16
// or 32 probes) is carried on the VALU: each lane adds its kernel values
// times that column's V, and the 4 lanes of a row are added at the end.
// J tiles of the prepared points and of V are copied global → LDS directly
// (16-byte buffer loads, double-buffered); reads past the end of V return 0
// and the prepared points past n are far away, so a ragged last tile needs
// no branches.  EXACT instances have k = 16·NB + NV, a compile-time V row
// stride.

constexpr int kBJ64 = 64;  // J points per LDS tile (FP64 kernel)

template <int KERN, int D, int NB, int NV, bool GRAD, bool EXACT>
__global__ __launch_bounds__(256) void kmv_f64(KArgs<double> a) {
  constexpr int P = pad_dim64(D);
  constexpr int VC = NB * 16 + NV;
  constexpr int BM = 16 * kWaves;
  __shared__ __attribute__((aligned(16))) double Xs[2][kBJ64 * P];
  __shared__ __attribute__((aligned(16))) double Vs[2][kBJ64 * VC];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int q = lane >> 4;        // which of the 4 J points of the step
  const int l16 = lane & 15;
  const int split = blockIdx.x % a.nsplit;
  const int64_t row0 = (int64_t)(blockIdx.x / a.nsplit) * BM;
  const int64_t jbeg = (int64_t)split * a.jchunk;
  const int64_t jend = min(a.n, jbeg + a.jchunk);
  const int k = EXACT ? VC : a.k;  // V row stride in LDS
  const int d = a.d;

  const int64_t irow = row0 + wave * 16 + l16;
  double xi[D];
#pragma unroll
  for (int c = 0; c < D; ++c)
    xi[c] = (irow < a.m && c < d) ? a.Xq[irow * d + c] * a.xs : 0.0;

  f64x4 acc[NB];
  f64x4 acc2[GRAD ? NB : 1];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    acc[b] = f64x4{0};
    if constexpr (GRAD) acc2[b] = f64x4{0};
  }
  double accx = 0.0, accx2 = 0.0;  // the VALU column (NV = 1)

  // Every wave issues its share of 16-byte chunks, 64 consecutive chunks
  // (1 KB) per instruction.
  constexpr int XC = kBJ64 * P / 2;  // chunks of the X tile
  const int vchunks = kBJ64 * k / 2;  // chunks of the V tile (k·64 doubles)
  auto gload = [&](int64_t j0, int buf) {
    char* xs = reinterpret_cast<char*>(&Xs[buf][0]);
    char* vs = reinterpret_cast<char*>(&Vs[buf][0]);
    const __amdgpu_buffer_rsrc_t rx = make_rsrc(a.Xp + j0 * P, (int64_t)kBJ64 * P * 8);
    for (int m = wave * 64; m < XC; m += 256)
      if (m + lane < XC)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rx, (lds_void_t*)(xs + 16 * m), 16,
                                                 16 * (m + lane), 0, 0, 0);
    const __amdgpu_buffer_rsrc_t rv = make_rsrc(a.V + j0 * k, (a.nk_pad - j0 * k) * 8);
    for (int m = wave * 64; m < vchunks; m += 256)
      if (m + lane < vchunks)
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rv, (lds_void_t*)(vs + 16 * m), 16,
                                                 16 * (m + lane), 0, 0, 0);
  };

  const int64_t ntiles = (jend > jbeg) ? (jend - jbeg + kBJ64 - 1) / kBJ64 : 0;
  if (ntiles > 0) gload(jbeg, 0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  for (int64_t t = 0; t < ntiles; ++t) {
    const int cur = (int)(t & 1);
    if (t + 1 < ntiles) gload(jbeg + (t + 1) * kBJ64, cur ^ 1);

    const double* xs = &Xs[cur][0];
    const double* vs = &Vs[cur][0];
#pragma unroll 4  // about 3% faster than 2 at n = 1e5, k = 33 (Gaussian); same results
    for (int st = 0; st < kBJ64 / 4; ++st) {
      const int j = 4 * st + q;
      double r2 = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double df = xi[c] - xs[j * P + c];
        r2 = fma(df, df, r2);
      }
      double kv, kg;
      kval_f64<KERN, GRAD>(r2, kv, kg);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const double vb = vs[j * k + b * 16 + l16];
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(kv, vb, acc[b], 0, 0, 0);
        if constexpr (GRAD) acc2[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(kg, vb, acc2[b], 0, 0, 0);
      }
      if constexpr (NV == 1) {
        const double vx = vs[j * k + NB * 16];
        accx = fma(kv, vx, accx);
        if constexpr (GRAD) accx2 = fma(kg, vx, accx2);
      }
    }

    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }

  const bool direct = a.nsplit == 1;
  double* p1 = direct ? a.o1 : a.o1 + (int64_t)split * a.m * k;
  double* p2 = a.o2;
  if constexpr (GRAD) {
    if (!direct) p2 = a.o2 + (int64_t)split * a.m * k;
  }
  if constexpr (NV == 1) {
    // Row l16's VALU column: the 4 lanes l16 + 16q hold its J points ≡ q mod 4.
    accx += __shfl_xor(accx, 16);
    accx += __shfl_xor(accx, 32);
    if constexpr (GRAD) {
      accx2 += __shfl_xor(accx2, 16);
      accx2 += __shfl_xor(accx2, 32);
    }
    const int col = NB * 16;
    if (q == 0 && irow < a.m && col < k) {
      const int64_t o = irow * k + col;
      if (direct) {
        if (a.o1) a.o1[o] = fma(a.f2, accx, a.sV ? a.s * a.sV[o] : 0.0);
        if constexpr (GRAD) {
          if (a.o2) a.o2[o] = a.cl * accx2;
          if (a.o3) a.o3[o] = a.cf * accx;
        }
      } else {
        p1[o] = accx;
        if constexpr (GRAD) p2[o] = accx2;
      }
    }
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int col = b * 16 + l16;
    if (col >= k) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + wave * 16 + q + 4 * r;
      if (row >= a.m) continue;
      const int64_t o = row * k + col;
      const double s1 = acc[b][r];
      if (direct) {
        if (a.o1) a.o1[o] = fma(a.f2, s1, a.sV ? a.s * a.sV[o] : 0.0);
        if constexpr (GRAD) {
          if (a.o2) a.o2[o] = a.cl * acc2[b][r];
          if (a.o3) a.o3[o] = a.cf * s1;
        }
      } else {
        p1[o] = s1;
        if constexpr (GRAD) p2[o] = acc2[b][r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Epilogue over S partials: out = f²·Σ_s P1 + s·V (no s·V term when V is
// null) and the derivative outputs.  Partials are added in split order in
// FP64.

template <typename T>
__global__ __launch_bounds__(256) void kmv_epilogue(const T* __restrict__ P1,
                                                    const T* __restrict__ P2,
                                                    const T* __restrict__ V, T* o1, T* o2,
                                                    T* o3, int64_t count, int nsplit, double f2,
                                                    double s, double cl, double cf) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s1 = 0.0, s2 = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) {
      s1 += (double)P1[sp * count + e];
      if (P2) s2 += (double)P2[sp * count + e];
    }
    if (o1) o1[e] = (T)(f2 * s1 + (V ? s * (double)V[e] : 0.0));
    if (o2) o2[e] = (T)(cl * s2);
    if (o3) o3[e] = (T)(cf * s1);
  }
}

template <typename T>
using KFn = void (*)(KArgs<T>);

template <int KERN, int D, bool GRAD>
KFn<double> pick_f64_cols(int k) {
  if (k < 16) return kmv_f64<KERN, D, 1, 0, GRAD, false>;
  if (k == 16) return kmv_f64<KERN, D, 1, 0, GRAD, true>;
  if (k == 17) return kmv_f64<KERN, D, 1, 1, GRAD, true>;
  if (k < 32) return kmv_f64<KERN, D, 2, 0, GRAD, false>;
  if (k == 32) return kmv_f64<KERN, D, 2, 0, GRAD, true>;
  if (k == 33) return kmv_f64<KERN, D, 2, 1, GRAD, true>;
  if (k < 48) return kmv_f64<KERN, D, 3, 0, GRAD, false>;
  if (k == 48) return kmv_f64<KERN, D, 3, 0, GRAD, true>;
  if (k == 49) return kmv_f64<KERN, D, 3, 1, GRAD, true>;
  if (k < 64) return kmv_f64<KERN, D, 4, 0, GRAD, false>;
  return kmv_f64<KERN, D, 4, 0, GRAD, true>;
}

// Compile-time dimension of the instance serving d coordinates.
int f64_dim_code(int d) {
  return d <= 2 ? 2 : d == 3 ? 3 : d == 4 ? 4 : d <= 8 ? 8 : d <= 16 ? 16 : d <= 20 ? 20 : 32;
}

template <int KERN, bool GRAD>
KFn<double> pick_f64_d(int d, int k) {
  switch (f64_dim_code(d)) {
    case 2: return pick_f64_cols<KERN, 2, GRAD>(k);
    case 3: return pick_f64_cols<KERN, 3, GRAD>(k);
    case 4: return pick_f64_cols<KERN, 4, GRAD>(k);
    case 8: return pick_f64_cols<KERN, 8, GRAD>(k);
    case 16: return pick_f64_cols<KERN, 16, GRAD>(k);
    case 20: return pick_f64_cols<KERN, 20, GRAD>(k);
    default: return pick_f64_cols<KERN, 32, GRAD>(k);
  }
}

// Number of J splits S (a power of two ≤ 64) so that the grid has at least
// `want_blocks` workgroups while each split keeps `min_tiles` J tiles
// (n J points, `rows` output rows).
int choose_splits(int64_t n, int64_t rows, int bm, int bj, int min_tiles, int64_t want_blocks) {
  const int64_t row_tiles = (rows + bm - 1) / bm;
  int s = 1;
  while (s < 64 && row_tiles * s < want_blocks && n / (2LL * s) >= (int64_t)min_tiles * bj) s *= 2;
  return s;
}

template <typename T>
int launch_epilogue(const T* P1, const T* P2, const T* V, MatvecOut out, int64_t count, int S,
                    double f2, double s, double cl, double cf, hipStream_t st, int ncus) {
  const int64_t blocks = std::min<int64_t>((count + 255) / 256, 8LL * ncus);
  hipLaunchKernelGGL(kmv_epilogue<T>, dim3((unsigned)blocks), dim3(256), 0, st, P1, P2, V,
                     static_cast<T*>(out.kv), static_cast<T*>(out.dl), static_cast<T*>(out.df),
                     count, S, f2, s, cl, cf);
  return hipGetLastError() == hipSuccess ? HIGP_OK
                                         : set_error(HIGP_ERR_HIP, "epilogue launch failed");
}

// Y = K̂V (Xq null) or the rectangular Y = f²·k(Xq, X)·V with m rows.
int run_f64(const Problem& p, int64_t m, const double* Xq, int k, const void* V, MatvecOut out,
            hipStream_t st, KFn<double> fn, double xs, double cl, int num_cus) {
  constexpr int bm = 16 * kWaves;
  const bool grad = out.dl != nullptr || out.df != nullptr;
  const bool cross = Xq != nullptr;
  const int64_t rows = cross ? m : p.n;
  const int P = pad_dim64(f64_dim_code(p.d));  // the instance's padded width
  KArgs<double> a{};
  a.Xq = cross ? Xq : static_cast<const double*>(p.X);
  a.sV = cross ? nullptr : static_cast<const double*>(V);
  a.n = p.n;
  a.m = rows;
  a.k = k;
  a.d = p.d;
  a.xs = xs;
  a.f2 = p.f * p.f;
  a.s = cross ? 0.0 : p.s;
  a.cl = cl;
  a.cf = 2.0 * p.f;
  const int S = choose_splits(p.n, rows, bm, kBJ64, 1, 4LL * num_cus);
  a.nsplit = S;
  const int64_t tiles_j = (p.n + kBJ64 - 1) / kBJ64;
  a.jchunk = ((tiles_j + S - 1) / S) * kBJ64;
  const int64_t npad = tiles_j * kBJ64;
  const int64_t nblocks = ((rows + bm - 1) / bm) * S;
  if (nblocks > 0x7fffffffLL) return set_error(HIGP_ERR_INVALID_ARG, "n too large");
  // Scratch: prepared points (whole J tiles); a zero-padded copy of V unless
  // V is 16-byte aligned and n·k is even (tiles move 16-byte chunks); the
  // split partials.
  const int64_t nk = p.n * k;
  const bool direct_v = (reinterpret_cast<uintptr_t>(V) & 15) == 0 && nk % 2 == 0;
  const int64_t nk_pad = (nk + 1) / 2 * 2;
  auto rup = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t xp_bytes = rup((size_t)npad * P * 8);
  const size_t v_bytes = direct_v ? 0 : rup((size_t)nk_pad * 8);
  const size_t per = S > 1 ? rup((size_t)rows * k * sizeof(double) * S) : 0;
  void* scratch = nullptr;
  HIGP_TRY(scratch_alloc(&scratch, xp_bytes + v_bytes + per * (grad ? 2 : 1), st));
  char* base = static_cast<char*>(scratch);
  double* Xp = reinterpret_cast<double*>(base);
  a.Xp = Xp;
  a.V = static_cast<const double*>(V);
  a.nk_pad = direct_v ? nk : nk_pad;
  if (!direct_v) {
    double* Vc = reinterpret_cast<double*>(base + xp_bytes);
    const unsigned cb = (unsigned)std::min<int64_t>((nk_pad + 255) / 256, 4096);
    hipLaunchKernelGGL(copy_pad_f64, dim3(cb), dim3(256), 0, st, nk, nk_pad,
                       static_cast<const double*>(V), Vc);
    a.V = Vc;
  }
  {
    const unsigned pb = (unsigned)std::min<int64_t>((npad * P + 255) / 256, 4096);
    hipLaunchKernelGGL(prep_points_f64, dim3(pb), dim3(256), 0, st, p.n, npad, p.d, P,
                       static_cast<const double*>(p.X), xs, Xp);
  }
  if (S == 1) {
    a.o1 = static_cast<double*>(out.kv);
    a.o2 = static_cast<double*>(out.dl);
    a.o3 = static_cast<double*>(out.df);
  } else {
    a.o1 = reinterpret_cast<double*>(base + xp_bytes + v_bytes);
    a.o2 = grad ? reinterpret_cast<double*>(base + xp_bytes + v_bytes + per) : nullptr;
  }
  hipLaunchKernelGGL(fn, dim3((unsigned)nblocks), dim3(256), 0, st, a);
  int rc = hipGetLastError() == hipSuccess ? HIGP_OK
                                           : set_error(HIGP_ERR_HIP, "FP64 MatVec launch failed");
  if (rc == HIGP_OK && S > 1)
    rc = launch_epilogue<double>(a.o1, grad ? a.o2 : nullptr, a.sV, out, rows * k, S, p.f * p.f,
                                 a.s, cl, 2.0 * p.f, st, num_cus);
  scratch_free(scratch, st);
  return rc;
}

}  // namespace

int launch_kmatvec_f64(const Problem& p, int k, const void* V, MatvecOut out, hipStream_t st,
                       int num_cus) {
  const bool grad = out.dl != nullptr || out.df != nullptr;
  KFn<double> fn;
  if (p.kernel == HIGP_GAUSSIAN)
    fn = grad ? pick_f64_d<HIGP_GAUSSIAN, true>(p.d, k) : pick_f64_d<HIGP_GAUSSIAN, false>(p.d, k);
  else
    fn = grad ? pick_f64_d<HIGP_MATERN32, true>(p.d, k) : pick_f64_d<HIGP_MATERN32, false>(p.d, k);
  return run_f64(p, p.n, nullptr, k, V, out, st, fn, coord_scale(p.kernel, HIGP_FP64, p.l),
                 p.f * p.f * dl_factor(p.kernel, HIGP_FP64, p.l), num_cus);
}

int launch_kmatvec_f64_cross(const Problem& p, int64_t m, const void* Xq, int k, const void* V,
                             void* Y, hipStream_t st, int num_cus) {
  KFn<double> fn = p.kernel == HIGP_GAUSSIAN ? pick_f64_d<HIGP_GAUSSIAN, false>(p.d, k)
                                             : pick_f64_d<HIGP_MATERN32, false>(p.d, k);
  MatvecOut out;
  out.kv = Y;
  return run_f64(p, m, static_cast<const double*>(Xq), k, V, out, st, fn,
                 coord_scale(p.kernel, HIGP_FP64, p.l), 0.0, num_cus);
}

}  // namespace higp
