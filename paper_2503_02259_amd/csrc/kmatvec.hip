// On-the-fly kernel MatVec Y = K̂·V and derivative MatVecs for gfx950.
//
// HiGP forms small kernel-matrix blocks, multiplies them into the vectors
// immediately and discards them ("Statement of Need", MatVec paragraph).
// Here one workgroup owns a row tile I and streams column tiles J of the
// points X and vectors V through LDS; each lane forms ‖x̃_i − x̃_j‖² and the
// kernel value in registers, directly in the MFMA A-operand slot, and the
// matrix core multiplies the kernel tile with the V tile held in LDS.  The
// kernel matrix never leaves registers.
//
// Coordinates are pre-scaled while they are staged so that the kernel value
// needs no further multiply:
//   Gaussian   x̃ = x·√(log₂e / (2l²))  →  k = exp2(−‖Δx̃‖²)
//   Matérn-3/2 x̃ = x·√3 / l            →  a = ‖Δx̃‖, k = (1 + a)·exp2(−a·log₂e)
// (FP64 uses natural-exp scalings x̂ = x/(√2·l) and x̃ = x·√3/l.)
//
// Split-J: the J range is cut into S chunks; workgroup b takes chunk b mod S,
// so with S = 8 each XCD (workgroups are dealt to the 8 XCDs round-robin)
// streams only its own eighth of X and V and keeps it in its L2.  Each chunk
// writes raw partial sums; an epilogue kernel adds the S partials in a fixed
// order (deterministic, no atomics) and applies f², s and the derivative
// scales.  With S = 1 the main kernel applies the epilogue itself.
#include <cmath>

#include "common.h"

namespace higp {
namespace {

constexpr float kLog2eF = 1.4426950408889634f;

// ---------------------------------------------------------------------------
// Kernel values on pre-scaled squared distances.

template <int KERN, bool GRAD>
__device__ __forceinline__ void kval_f32(float r2, float& kv, float& kg) {
  if constexpr (KERN == HIGP_GAUSSIAN) {
    kv = __builtin_amdgcn_exp2f(-r2);
    if constexpr (GRAD) kg = kv * r2;  // ∝ ∂k/∂l
  } else {
    const float a = __builtin_amdgcn_sqrtf(r2);
    const float e = __builtin_amdgcn_exp2f(-a * kLog2eF);
    kv = fmaf(a, e, e);                    // (1 + a)·e^{−a}
    if constexpr (GRAD) kg = r2 * e;       // a²·e^{−a} ∝ ∂k/∂l
  }
}

template <int KERN, bool GRAD>
__device__ __forceinline__ void kval_f64(double r2, double& kv, double& kg) {
  if constexpr (KERN == HIGP_GAUSSIAN) {
    kv = exp(-r2);                         // x̂ = x/(√2 l): r̂² = r²/(2l²)
    if constexpr (GRAD) kg = kv * r2;
  } else {
    const double a = sqrt(r2);
    const double e = exp(-a);
    kv = fma(a, e, e);
    if constexpr (GRAD) kg = r2 * e;
  }
}

// ---------------------------------------------------------------------------
// Arguments.

template <typename T>
struct KArgs {
  const T* X;   // n×d row-major
  const T* V;   // n×k row-major
  T* o1;        // S==1: K̂V (or null); S>1: partial Σ k·v, S×n×k
  T* o2;        // S==1: ∂K̂/∂l·V (or null); S>1: partial Σ k_l·v (GRAD only)
  T* o3;        // S==1: ∂K̂/∂f·V (or null); unused when S>1
  int64_t n;
  int64_t jchunk;  // J points per split (multiple of the J tile)
  int k, d, nsplit;
  T xs;          // coordinate pre-scale
  T f2, s;       // K̂ = f²K + sI (epilogue, S==1)
  T cl, cf;      // ∂K̂/∂l = cl·Σk_l v, ∂K̂/∂f = cf·Σk v (epilogue, S==1)
};

// ---------------------------------------------------------------------------
// FP32: v_mfma_f32_32x32x2f32.  A wave owns 32 rows; per MFMA each lane
// supplies K[i0 + lane%32][j0 + lane/32].  NB blocks of 32 columns go through
// the matrix core; NV (≤ 2) trailing columns are accumulated on the VALU
// (k = 33 is 32 MFMA columns plus one VALU column instead of padding to 64).
// Output layout of the 32×32 accumulator: lane l, register r holds row
// 8(r/4) + 4(l/32) + r%4, column l%32.

constexpr int kWaves = 4;
constexpr int kBJ = 64;  // J points per LDS tile

template <int KERN, int D, int NB, int NV, bool GRAD>
__global__ __launch_bounds__(256) void kmv_f32(KArgs<float> a) {
  constexpr int P = D <= 4 ? 4 : 8;       // padded coordinate stride in LDS
  constexpr int VC = NB * 32 + NV;        // V columns held in LDS
  constexpr int VLD = VC;                 // LDS row stride of the V tile
  constexpr int BM = 32 * kWaves;
  __shared__ __attribute__((aligned(16))) float Xs[2][kBJ][P];
  __shared__ float Vs[2][kBJ][VLD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int half = lane >> 5;     // which of the 2 J columns of the MFMA step
  const int l32 = lane & 31;
  const int split = blockIdx.x % a.nsplit;
  const int64_t row0 = (int64_t)(blockIdx.x / a.nsplit) * BM;
  const int64_t jbeg = (int64_t)split * a.jchunk;
  const int64_t jend = min(a.n, jbeg + a.jchunk);
  const int k = a.k, d = a.d;

  // This lane's row point, scaled; padded coordinates are 0.
  const int64_t irow = row0 + wave * 32 + l32;
  float xi[D];
#pragma unroll
  for (int c = 0; c < D; ++c)
    xi[c] = (irow < a.n && c < d) ? a.X[irow * d + c] * a.xs : 0.0f;

  f32x16 acc[NB > 0 ? NB : 1];
  f32x16 acc2[(GRAD && NB > 0) ? NB : 1];
  float accv[NV > 0 ? NV : 1];
  float accv2[(GRAD && NV > 0) ? NV : 1];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    acc[b] = f32x16{0};
    if constexpr (GRAD) acc2[b] = f32x16{0};
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    accv[v] = 0.0f;
    if constexpr (GRAD) accv2[v] = 0.0f;
  }

  // Zero the padded coordinates of both LDS buffers once.
  if constexpr (P > D) {
    for (int e = tid; e < 2 * kBJ * (P - D); e += 256) {
      const int buf = e / (kBJ * (P - D));
      const int rem = e % (kBJ * (P - D));
      Xs[buf][rem / (P - D)][D + rem % (P - D)] = 0.0f;
    }
  }

  // Global → register staging of one J tile.  X: kBJ·D floats, thread t takes
  // (row t/D, coord t%D).  V: thread t takes column t%64 of rows t/64 + 4m.
  constexpr int XPER = (kBJ * D + 255) / 256;
  constexpr int VROWS = kBJ / 4;
  float xr[XPER];
  float vr[VROWS];
  const int vc = tid & 63;
  const int vr0 = tid >> 6;

  auto gload = [&](int64_t jt) {
#pragma unroll
    for (int m = 0; m < XPER; ++m) {
      const int e = tid + 256 * m;
      const int r = e / D, c = e % D;
      float v = 0.0f;
      if (e < kBJ * D && c < d && jt + r < jend) v = a.X[(jt + r) * d + c];
      xr[m] = v;
    }
#pragma unroll
    for (int m = 0; m < VROWS; ++m) {
      const int64_t j = jt + vr0 + 4 * m;
      float v = 0.0f;
      if (vc < k && j < jend) v = a.V[j * k + vc];
      vr[m] = v;
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int m = 0; m < XPER; ++m) {
      const int e = tid + 256 * m;
      if (e < kBJ * D) Xs[buf][e / D][e % D] = xr[m] * a.xs;
    }
    if (vc < VC) {
#pragma unroll
      for (int m = 0; m < VROWS; ++m) Vs[buf][vr0 + 4 * m][vc] = vr[m];
    }
  };

  const int64_t ntiles = (jend > jbeg) ? (jend - jbeg + kBJ - 1) / kBJ : 0;
  if (ntiles > 0) {
    gload(jbeg);
    lstore(0);
  }
  __syncthreads();

  for (int64_t t = 0; t < ntiles; ++t) {
    const int cur = (int)(t & 1);
    const bool more = t + 1 < ntiles;
    if (more) gload(jbeg + (t + 1) * kBJ);

#pragma unroll 4
    for (int st = 0; st < kBJ / 2; ++st) {
      const int j = 2 * st + half;
      float r2 = 0.0f;
      if constexpr (P == 4) {
        const f32x4 xj = *reinterpret_cast<const f32x4*>(&Xs[cur][j][0]);
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const float df = xi[c] - xj[c];
          r2 = fmaf(df, df, r2);
        }
      } else {
        const f32x4 xa = *reinterpret_cast<const f32x4*>(&Xs[cur][j][0]);
        const f32x4 xb = *reinterpret_cast<const f32x4*>(&Xs[cur][j][4]);
#pragma unroll
        for (int c = 0; c < D; ++c) {
          const float df = xi[c] - (c < 4 ? xa[c & 3] : xb[c & 3]);
          r2 = fmaf(df, df, r2);
        }
      }
      float kv, kg;
      kval_f32<KERN, GRAD>(r2, kv, kg);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const float vb = Vs[cur][j][b * 32 + l32];
        acc[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(kv, vb, acc[b], 0, 0, 0);
        if constexpr (GRAD) acc2[b] = __builtin_amdgcn_mfma_f32_32x32x2f32(kg, vb, acc2[b], 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const float vv = Vs[cur][j][NB * 32 + v];
        accv[v] = fmaf(kv, vv, accv[v]);
        if constexpr (GRAD) accv2[v] = fmaf(kg, vv, accv2[v]);
      }
    }

    if (more) lstore(cur ^ 1);
    __syncthreads();
  }

  // VALU columns: lanes l and l+32 hold the two halves of row l%32.
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    accv[v] += __shfl_xor(accv[v], 32);
    if constexpr (GRAD) accv2[v] += __shfl_xor(accv2[v], 32);
  }

  const bool direct = a.nsplit == 1;
  float* p1 = a.o1;
  float* p2 = a.o2;
  if (!direct) {
    p1 = a.o1 + (int64_t)split * a.n * k;
    if constexpr (GRAD) p2 = a.o2 + (int64_t)split * a.n * k;
  }

#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int col = b * 32 + l32;
    if (col >= k) continue;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t row = row0 + wave * 32 + 8 * (r >> 2) + 4 * half + (r & 3);
      if (row >= a.n) continue;
      const int64_t o = row * k + col;
      const float s1 = acc[b][r];
      if (direct) {
        if (a.o1) a.o1[o] = fmaf(a.f2, s1, a.s * a.V[o]);
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
  if (half == 0 && irow < a.n) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int col = NB * 32 + v;
      const int64_t o = irow * k + col;
      if (direct) {
        if (a.o1) a.o1[o] = fmaf(a.f2, accv[v], a.s * a.V[o]);
        if constexpr (GRAD) {
          if (a.o2) a.o2[o] = a.cl * accv2[v];
          if (a.o3) a.o3[o] = a.cf * accv[v];
        }
      } else {
        p1[o] = accv[v];
        if constexpr (GRAD) p2[o] = accv2[v];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// FP64: v_mfma_f64_16x16x4f64.  A wave owns 16 rows; per MFMA each lane
// supplies K[i0 + lane%16][j0 + lane/16] (4 J points per step); NB blocks of
// 16 columns.  Output layout: lane l, register r holds row l/16 + 4r,
// column l%16.

template <int KERN, int D, int NB, bool GRAD>
__global__ __launch_bounds__(256) void kmv_f64(KArgs<double> a) {
  constexpr int P = D <= 4 ? 4 : 8;
  constexpr int VC = NB * 16;
  constexpr int BM = 16 * kWaves;
  __shared__ double Xs[2][kBJ][P];
  __shared__ double Vs[2][kBJ][VC];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int q = lane >> 4;        // which of the 4 J points of the step
  const int l16 = lane & 15;
  const int split = blockIdx.x % a.nsplit;
  const int64_t row0 = (int64_t)(blockIdx.x / a.nsplit) * BM;
  const int64_t jbeg = (int64_t)split * a.jchunk;
  const int64_t jend = min(a.n, jbeg + a.jchunk);
  const int k = a.k, d = a.d;

  const int64_t irow = row0 + wave * 16 + l16;
  double xi[D];
#pragma unroll
  for (int c = 0; c < D; ++c)
    xi[c] = (irow < a.n && c < d) ? a.X[irow * d + c] * a.xs : 0.0;

  f64x4 acc[NB];
  f64x4 acc2[GRAD ? NB : 1];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    acc[b] = f64x4{0};
    if constexpr (GRAD) acc2[b] = f64x4{0};
  }

  constexpr int XPER = (kBJ * D + 255) / 256;
  constexpr int VROWS = kBJ / 4;
  double xr[XPER];
  double vr[VROWS];
  const int vc = tid & 63;
  const int vr0 = tid >> 6;

  auto gload = [&](int64_t jt) {
#pragma unroll
    for (int m = 0; m < XPER; ++m) {
      const int e = tid + 256 * m;
      const int r = e / D, c = e % D;
      double v = 0.0;
      if (e < kBJ * D && c < d && jt + r < jend) v = a.X[(jt + r) * d + c];
      xr[m] = v;
    }
#pragma unroll
    for (int m = 0; m < VROWS; ++m) {
      const int64_t j = jt + vr0 + 4 * m;
      double v = 0.0;
      if (vc < k && j < jend) v = a.V[j * k + vc];
      vr[m] = v;
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int m = 0; m < XPER; ++m) {
      const int e = tid + 256 * m;
      if (e < kBJ * D) Xs[buf][e / D][e % D] = xr[m] * a.xs;
    }
    if (vc < VC) {
#pragma unroll
      for (int m = 0; m < VROWS; ++m) Vs[buf][vr0 + 4 * m][vc] = vr[m];
    }
  };

  if constexpr (P > D) {
    for (int e = tid; e < 2 * kBJ * (P - D); e += 256) {
      const int buf = e / (kBJ * (P - D));
      const int rem = e % (kBJ * (P - D));
      Xs[buf][rem / (P - D)][D + rem % (P - D)] = 0.0;
    }
  }

  const int64_t ntiles = (jend > jbeg) ? (jend - jbeg + kBJ - 1) / kBJ : 0;
  if (ntiles > 0) {
    gload(jbeg);
    lstore(0);
  }
  __syncthreads();

  for (int64_t t = 0; t < ntiles; ++t) {
    const int cur = (int)(t & 1);
    const bool more = t + 1 < ntiles;
    if (more) gload(jbeg + (t + 1) * kBJ);

#pragma unroll 2
    for (int st = 0; st < kBJ / 4; ++st) {
      const int j = 4 * st + q;
      double r2 = 0.0;
#pragma unroll
      for (int c = 0; c < D; ++c) {
        const double df = xi[c] - Xs[cur][j][c];
        r2 = fma(df, df, r2);
      }
      double kv, kg;
      kval_f64<KERN, GRAD>(r2, kv, kg);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const double vb = Vs[cur][j][b * 16 + l16];
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(kv, vb, acc[b], 0, 0, 0);
        if constexpr (GRAD) acc2[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(kg, vb, acc2[b], 0, 0, 0);
      }
    }

    if (more) lstore(cur ^ 1);
    __syncthreads();
  }

  const bool direct = a.nsplit == 1;
  double* p1 = direct ? a.o1 : a.o1 + (int64_t)split * a.n * k;
  double* p2 = a.o2;
  if constexpr (GRAD) {
    if (!direct) p2 = a.o2 + (int64_t)split * a.n * k;
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int col = b * 16 + l16;
    if (col >= k) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = row0 + wave * 16 + q + 4 * r;
      if (row >= a.n) continue;
      const int64_t o = row * k + col;
      const double s1 = acc[b][r];
      if (direct) {
        if (a.o1) a.o1[o] = fma(a.f2, s1, a.s * a.V[o]);
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
// Epilogue over S partials: out = f²·Σ_s P1 + s·V (and the derivative
// outputs).  Partials are added in split order in FP64.

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
    if (o1) o1[e] = (T)(f2 * s1 + s * (double)V[e]);
    if (o2) o2[e] = (T)(cl * s2);
    if (o3) o3[e] = (T)(cf * s1);
  }
}

// ---------------------------------------------------------------------------
// Dispatch.

template <typename T>
using KFn = void (*)(KArgs<T>);

template <int KERN, int D, bool GRAD>
KFn<float> pick_f32_cols(int k) {
  if (k == 1) return kmv_f32<KERN, D, 0, 1, GRAD>;
  if (k == 2) return kmv_f32<KERN, D, 0, 2, GRAD>;
  if (k <= 32) return kmv_f32<KERN, D, 1, 0, GRAD>;
  if (k == 33) return kmv_f32<KERN, D, 1, 1, GRAD>;
  if (k == 34) return kmv_f32<KERN, D, 1, 2, GRAD>;
  return kmv_f32<KERN, D, 2, 0, GRAD>;
}

template <int KERN, bool GRAD>
KFn<float> pick_f32_d(int d, int k) {
  if (d <= 2) return pick_f32_cols<KERN, 2, GRAD>(k);
  if (d == 3) return pick_f32_cols<KERN, 3, GRAD>(k);
  if (d == 4) return pick_f32_cols<KERN, 4, GRAD>(k);
  return pick_f32_cols<KERN, 8, GRAD>(k);
}

template <int KERN, int D, bool GRAD>
KFn<double> pick_f64_cols(int k) {
  if (k <= 16) return kmv_f64<KERN, D, 1, GRAD>;
  if (k <= 32) return kmv_f64<KERN, D, 2, GRAD>;
  if (k <= 48) return kmv_f64<KERN, D, 3, GRAD>;
  return kmv_f64<KERN, D, 4, GRAD>;
}

template <int KERN, bool GRAD>
KFn<double> pick_f64_d(int d, int k) {
  if (d <= 2) return pick_f64_cols<KERN, 2, GRAD>(k);
  if (d == 3) return pick_f64_cols<KERN, 3, GRAD>(k);
  if (d == 4) return pick_f64_cols<KERN, 4, GRAD>(k);
  return pick_f64_cols<KERN, 8, GRAD>(k);
}

int g_num_cus = 0;

int num_cus() {
  if (g_num_cus == 0) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    g_num_cus = cus;
  }
  return g_num_cus;
}

// Number of J splits: enough workgroups to fill every CU several times, a
// divisor of 8 so that a split maps onto whole XCDs, and every split at least
// a few J tiles long.
int choose_splits(int64_t n, int bm) {
  const int64_t row_tiles = (n + bm - 1) / bm;
  const int64_t want = 4LL * num_cus();
  int s = 1;
  while (s < 8 && row_tiles * s < want && n / (2 * s) >= 4 * kBJ) s *= 2;
  return s;
}

template <typename T>
int run(const Problem& p, int k, const void* V, MatvecOut out, hipStream_t st, int bm,
        KFn<T> fn, double xs, double cl) {
  const bool grad = out.dl != nullptr || out.df != nullptr;
  KArgs<T> a{};
  a.X = static_cast<const T*>(p.X);
  a.V = static_cast<const T*>(V);
  a.n = p.n;
  a.k = k;
  a.d = p.d;
  a.xs = (T)xs;
  a.f2 = (T)(p.f * p.f);
  a.s = (T)p.s;
  a.cl = (T)cl;
  a.cf = (T)(2.0 * p.f);
  const int S = choose_splits(p.n, bm);
  a.nsplit = S;
  const int64_t tiles_j = (p.n + kBJ - 1) / kBJ;
  a.jchunk = ((tiles_j + S - 1) / S) * kBJ;
  const int64_t row_tiles = (p.n + bm - 1) / bm;
  const int64_t nblocks = row_tiles * S;
  if (nblocks > 0x7fffffffLL) return set_error(HIGP_ERR_INVALID_ARG, "n too large");

  void* scratch = nullptr;
  if (S == 1) {
    a.o1 = static_cast<T*>(out.kv);
    a.o2 = static_cast<T*>(out.dl);
    a.o3 = static_cast<T*>(out.df);
  } else {
    const size_t per = (size_t)p.n * k * sizeof(T) * S;
    HIGP_TRY(scratch_alloc(&scratch, per * (grad ? 2 : 1), st));
    a.o1 = static_cast<T*>(scratch);
    a.o2 = grad ? reinterpret_cast<T*>(static_cast<char*>(scratch) + per) : nullptr;
  }
  hipLaunchKernelGGL(fn, dim3((unsigned)nblocks), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && S > 1) {
    const int64_t count = p.n * k;
    const int64_t blocks = std::min<int64_t>((count + 255) / 256, 8LL * num_cus());
    hipLaunchKernelGGL(kmv_epilogue<T>, dim3((unsigned)blocks), dim3(256), 0, st, a.o1,
                       grad ? a.o2 : (const T*)nullptr, a.V, static_cast<T*>(out.kv),
                       static_cast<T*>(out.dl), static_cast<T*>(out.df), count, S,
                       p.f * p.f, p.s, cl, 2.0 * p.f);
    e = hipGetLastError();
  }
  if (scratch) scratch_free(scratch, st);
  if (e != hipSuccess)
    return set_error(HIGP_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(e));
  return HIGP_OK;
}

}  // namespace

int launch_kmatvec(const Problem& p, int k, const void* V, MatvecOut out, hipStream_t st,
                   int prec_override) {
  const int prec = prec_override >= 0 ? prec_override : p.prec;
  const bool grad = out.dl != nullptr || out.df != nullptr;
  const double l = p.l;
  if (prec == HIGP_FP64) {
    // Gaussian: x̂ = x/(√2 l), k = exp(−r̂²), ∂k/∂l = k·r̂²·(2/l).
    // Matérn:   x̃ = x·√3/l,   k = (1+a)e^{−a}, ∂k/∂l = a²e^{−a}/l.
    const double xs = p.kernel == HIGP_GAUSSIAN ? 1.0 / (std::sqrt(2.0) * l) : std::sqrt(3.0) / l;
    const double dk = p.kernel == HIGP_GAUSSIAN ? 2.0 / l : 1.0 / l;
    KFn<double> fn;
    if (p.kernel == HIGP_GAUSSIAN)
      fn = grad ? pick_f64_d<HIGP_GAUSSIAN, true>(p.d, k) : pick_f64_d<HIGP_GAUSSIAN, false>(p.d, k);
    else
      fn = grad ? pick_f64_d<HIGP_MATERN32, true>(p.d, k) : pick_f64_d<HIGP_MATERN32, false>(p.d, k);
    return run<double>(p, k, V, out, st, 16 * kWaves, fn, xs, p.f * p.f * dk);
  }
  if (prec == HIGP_FP32) {
    // Gaussian: x̃ = x·√(log₂e/(2l²)), k = exp2(−r̃²), ∂k/∂l = k·r̃²·2/(l·log₂e).
    // Matérn:   x̃ = x·√3/l,           k = (1+a)e^{−a}, ∂k/∂l = a²e^{−a}/l.
    const double log2e = 1.4426950408889634;
    const double xs = p.kernel == HIGP_GAUSSIAN ? std::sqrt(log2e / (2.0 * l * l)) : std::sqrt(3.0) / l;
    const double dk = p.kernel == HIGP_GAUSSIAN ? 2.0 / (l * log2e) : 1.0 / l;
    KFn<float> fn;
    if (p.kernel == HIGP_GAUSSIAN)
      fn = grad ? pick_f32_d<HIGP_GAUSSIAN, true>(p.d, k) : pick_f32_d<HIGP_GAUSSIAN, false>(p.d, k);
    else
      fn = grad ? pick_f32_d<HIGP_MATERN32, true>(p.d, k) : pick_f32_d<HIGP_MATERN32, false>(p.d, k);
    return run<float>(p, k, V, out, st, 32 * kWaves, fn, xs, p.f * p.f * dk);
  }
  return set_error(HIGP_ERR_UNSUPPORTED, "precision %d is not implemented for this MatVec", prec);
}

}  // namespace higp
