// Nyström preconditioner for PCG.  The paper's preconditioner (AFN) rests on
// a Nyström approximation of the kernel matrix on selected points, and on
// evaluating many small kernel matrices ("Statement of Need"); this is the
// generic form:
//
//   landmarks  r points by farthest-point sampling (first point 0; each next
//              one maximises the squared distance to the nearest landmark,
//              lowest index on ties; distances in FP64);
//   M          s·I + f²·K_nr·(K_rr + εI)⁻¹·K_rn, ε = 1e-8 (keeps K_rr
//              invertible when landmarks sit closer than the length-scale;
//              K_rr is evaluated in FP64, and ε grows ×100 up to 1e-2 only if
//              the factorisation still fails);
//   factor     K_rr + εI = RRᵀ (Cholesky), L = K_nr·R⁻ᵀ, so M = s·I + f²·LLᵀ;
//   M⁻¹R       (R − L·C⁻¹·LᵀR)/s,  C = (s/f²)·I + LᵀL  (Woodbury; the
//              eigenvalues of C are ≥ s/f², so C is well conditioned even
//              when K_rr is not).
//
// Build: r − 1 fused "update nearest distance + argmax" launches; K_nr in
// the problem's precision (n×r, row-major); R⁻¹ by a host Cholesky
// factorisation and triangular inverse (r ≤ 2048); L by a tiled product with
// R⁻ᵀ (FP64 accumulation, stored in the problem's precision); C accumulated
// in FP64 from that stored L; C⁻¹ on the host, stored in FP64.  Apply (once
// per PCG iteration): T = LᵀR by row chunks with FP64 partial sums added in
// chunk order, u = C⁻¹T, Z = (R − L·u)/s.  Everything is deterministic.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <vector>

#include "kvalue.h"
#include "nystrom.h"

namespace higp {
namespace {

constexpr int kThreads = 256;
constexpr double kNysJitter = 1e-8;  // ε added to the diagonal of K_rr

// dmin[i] = min(dmin[i], ‖x_i − x_p‖²) with p = sel[j − 1]; then the block
// argmax (largest dmin, lowest index); the last block combines the blocks
// and writes sel[j].
template <typename T>
__global__ __launch_bounds__(kThreads) void fps_step(int64_t n, int d, const T* __restrict__ X,
                                                     int* sel, int j, double* dmin,
                                                     double* bval, int64_t* bidx,
                                                     unsigned* counter) {
  __shared__ double sv[kThreads];
  __shared__ int64_t si[kThreads];
  const int p = sel[j - 1];
  double best = -1.0;
  int64_t bi = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kThreads) {
    double dist = 0.0;
    for (int c = 0; c < d; ++c) {
      const double df = (double)X[i * d + c] - (double)X[(int64_t)p * d + c];
      dist = dist + df * df;
    }
    const double m = fmin(dmin[i], dist);
    dmin[i] = m;
    if (m > best) {  // i increases along the loop: ties keep the lower index
      best = m;
      bi = i;
    }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double v2 = sv[threadIdx.x + s];
      const int64_t i2 = si[threadIdx.x + s];
      if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x])) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    bval[blockIdx.x] = sv[0];
    bidx[blockIdx.x] = si[0];
  }
  __threadfence();
  __syncthreads();
  __shared__ unsigned ticket;
  if (threadIdx.x == 0) ticket = atomicAdd(counter, 1u);
  __syncthreads();
  if (ticket != gridDim.x - 1) return;
  __threadfence();
  // The last block: every thread takes the block winners b ≡ tid, then the
  // same tree as above (the largest value, lowest index on ties: the result
  // does not depend on the order of the comparisons).
  double v = -1.0;
  int64_t idx = 0;
  for (unsigned b = threadIdx.x; b < gridDim.x; b += kThreads) {
    const double vb = __hip_atomic_load(&bval[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t ib = __hip_atomic_load(&bidx[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (vb > v || (vb == v && ib < idx)) {
      v = vb;
      idx = ib;
    }
  }
  sv[threadIdx.x] = v;
  si[threadIdx.x] = idx;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double v2 = sv[threadIdx.x + s];
      const int64_t i2 = si[threadIdx.x + s];
      if (v2 > sv[threadIdx.x] || (v2 == sv[threadIdx.x] && i2 < si[threadIdx.x])) {
        sv[threadIdx.x] = v2;
        si[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    sel[j] = (int)si[0];
    *counter = 0u;
  }
}

__global__ void fill_inf(int64_t n, double* a) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = HUGE_VAL;
}

// W[i][a] = k(x_i, x_sel[a]) in the problem's precision (pre-scaled points).
template <typename T, int KERN>
__global__ void nys_kernel_matrix(int64_t n, int r, int d, const T* __restrict__ X,
                                  const int* __restrict__ sel, double xs, T* __restrict__ W) {
  const int64_t total = n * r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / r;
    const int a = (int)(e % r);
    const int64_t p = sel[a];
    if constexpr (sizeof(T) == 8) {
      double r2 = 0.0;
      for (int c = 0; c < d; ++c) {
        const double df = (X[i * d + c] - X[p * d + c]) * xs;
        r2 = fma(df, df, r2);
      }
      double kv, kg;
      kval_f64<KERN, false>(r2, kv, kg);
      W[e] = (T)kv;
    } else {
      const float xsf = (float)xs;
      float r2 = 0.0f;
      for (int c = 0; c < d; ++c) {
        const float df = ((float)X[i * d + c] - (float)X[p * d + c]) * xsf;
        r2 = fmaf(df, df, r2);
      }
      float kv, kg;
      kval_f32<KERN, false>(r2, kv, kg);
      W[e] = (T)kv;
    }
  }
}

// part[s][a][b] = Σ_{i in chunk s} W[i][a]·W[i][b] for a 16×16 tile (FP64).
constexpr int kGT = 16;   // tile edge
constexpr int kGI = 32;   // rows staged per step
template <typename T>
__global__ __launch_bounds__(256) void nys_gram(int64_t n, int r, const T* __restrict__ W,
                                                int64_t chunk, double* __restrict__ part) {
  __shared__ double wa[kGI][kGT];
  __shared__ double wb[kGI][kGT];
  const int ta = threadIdx.x % kGT, tb = threadIdx.x / kGT;
  const int a0 = blockIdx.x * kGT, b0 = blockIdx.y * kGT;
  const int s = blockIdx.z;
  const int64_t beg = (int64_t)s * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  double acc = 0.0;
  for (int64_t i0 = beg; i0 < end; i0 += kGI) {
    for (int e = threadIdx.x; e < kGI * kGT; e += 256) {
      const int ii = e / kGT, cc = e % kGT;
      const int64_t i = i0 + ii;
      wa[ii][cc] = (i < end && a0 + cc < r) ? (double)W[i * r + a0 + cc] : 0.0;
      wb[ii][cc] = (i < end && b0 + cc < r) ? (double)W[i * r + b0 + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll 8
    for (int ii = 0; ii < kGI; ++ii) acc = fma(wa[ii][ta], wb[ii][tb], acc);
    __syncthreads();
  }
  if (a0 + ta < r && b0 + tb < r) part[((int64_t)s * r + a0 + ta) * r + b0 + tb] = acc;
}

// C[a][b] = Σ_s part[s][a][b] + (a == b ? s/f² : 0).
__global__ void nys_gram_finish(int r, int S, const double* __restrict__ part, double sf2,
                                double* __restrict__ C) {
  const int64_t total = (int64_t)r * r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    double acc = 0.0;
    for (int s = 0; s < S; ++s) acc += part[(int64_t)s * total + e];
    const int a = (int)(e / r), b = (int)(e % r);
    C[e] = acc + (a == b ? sf2 : 0.0);
  }
}

// Krr[a][b] = k(x_sel[a], x_sel[b]) evaluated in FP64 from the (possibly
// FP32) coordinates, so that its Cholesky factor is not spoiled by the FP32
// rounding of K_nr; xs is the FP64 coordinate scale.
template <typename T, int KERN>
__global__ void nys_krr_f64(int r, int d, const T* __restrict__ X, const int* __restrict__ sel,
                            double xs, double* __restrict__ Krr) {
  const int64_t total = (int64_t)r * r;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pa = sel[e / r], pb = sel[e % r];
    double r2 = 0.0;
    for (int c = 0; c < d; ++c) {
      const double df = ((double)X[pa * d + c] - (double)X[pb * d + c]) * xs;
      r2 = fma(df, df, r2);
    }
    double kv, kg;
    kval_f64<KERN, false>(r2, kv, kg);
    Krr[e] = kv;
  }
}

// L[i][a] = Σ_{b ≤ a} W[i][b]·Rinv[a][b] (L = W·R⁻ᵀ; Rinv lower triangular
// with zeros above the diagonal).  64×64 output tiles, 4×4 per thread, b in
// chunks of 16 up to the tile's last column.
template <typename T>
__global__ __launch_bounds__(256) void nys_tri_gemm(int64_t n, int r, const T* __restrict__ W,
                                                    const double* __restrict__ Rinv,
                                                    T* __restrict__ L) {
  __shared__ double ws[16][65];
  __shared__ double rs[16][65];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  const int a0 = blockIdx.y * 64;
  double acc[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[q][t] = 0.0;
  const int bmax = a0 + 64 < r ? a0 + 64 : r;
  for (int b0 = 0; b0 < bmax; b0 += 16) {
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int bb = e % 16, rr = e / 16;
      const int64_t i = i0 + rr;
      const int b = b0 + bb, a = a0 + rr;
      ws[bb][rr] = (i < n && b < r) ? (double)W[i * r + b] : 0.0;
      rs[bb][rr] = (a < r && b < r) ? Rinv[(int64_t)a * r + b] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int bb = 0; bb < 16; ++bb) {
      double wv[4], rv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        wv[q] = ws[bb][ty * 4 + q];
        rv[q] = rs[bb][tx * 4 + q];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[q][t] = fma(wv[q], rv[t], acc[q][t]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t i = i0 + ty * 4 + q;
      const int a = a0 + tx * 4 + t;
      if (i < n && a < r) L[i * r + a] = (T)acc[q][t];
    }
}

// Row splits of WᵀR: enough blocks for several per CU (at k ≥ 4 a split has
// ⌈r/64⌉ blocks) while each split keeps at least 512 rows.
// Row chunks S of the LᵀR pass: enough that the grid (⌈r/256⌉ landmark
// blocks × S) has about 1024 workgroups, each chunk at least 64 rows, and
// the S·r·kmax FP64 partials at most 64 MB.
int wtr_splits(int64_t n, int r, int kmax) {
  const int64_t bx = (r + 255) / 256;
  int64_t s = (1024 + bx - 1) / bx;
  s = std::min<int64_t>(s, std::max<int64_t>(1, n / 64));
  s = std::min<int64_t>(s, std::max<int64_t>(1, (64LL << 20) / ((int64_t)r * kmax * 8)));
  return (int)std::max<int64_t>(1, s);
}

// Tm[e] = Σ_s part[s][e]: eight lanes per output, lane j adding the chunks
// s ≡ j (mod 8) in order with eight loads in flight, then the lanes combined
// by a fixed butterfly.  32 outputs per block of 256.
__global__ __launch_bounds__(256) void nys_reduce_parts(int rk, int S,
                                                        const double* __restrict__ part,
                                                        double* __restrict__ Tm) {
  const int j = threadIdx.x & 7;
  const int e = blockIdx.x * 32 + (threadIdx.x >> 3);
  double acc = 0.0;
  if (e < rk) {
    int s = j;
    for (; s + 56 < S; s += 64) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = part[(int64_t)(s + 8 * u) * rk + e];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; s < S; s += 8) acc += part[(int64_t)s * rk + e];
  }
  acc += __shfl_xor(acc, 1);
  acc += __shfl_xor(acc, 2);
  acc += __shfl_xor(acc, 4);
  if (e < rk && j == 0) Tm[e] = acc;
}

// u = C⁻¹·T (r×r times r×k): one wave per row a of C⁻¹.  Lane l takes the
// entries b ≡ l (mod 64) of the row (coalesced), for 16 columns at a time,
// and the 64 lane sums of a column are added by a fixed butterfly.
__global__ __launch_bounds__(256) void nys_cinv_t(int r, int k, const double* __restrict__ Cinv,
                                                  const double* __restrict__ Tm,
                                                  double* __restrict__ u) {
  const int lane = threadIdx.x & 63;
  const int a = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (a >= r) return;  // whole waves: no barrier follows
  const double* row = Cinv + (int64_t)a * r;
  for (int c0 = 0; c0 < k; c0 += 16) {
    double acc[16];
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) acc[cc] = 0.0;
    for (int b = lane; b < r; b += 64) {
      const double cv = row[b];
#pragma unroll
      for (int cc = 0; cc < 16; ++cc)
        if (c0 + cc < k) acc[cc] = fma(cv, Tm[(int64_t)b * k + c0 + cc], acc[cc]);
    }
#pragma unroll
    for (int cc = 0; cc < 16; ++cc) {
      double v = acc[cc];
#pragma unroll
      for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
      if (lane == 0 && c0 + cc < k) u[(int64_t)a * k + c0 + cc] = v;
    }
  }
}

// The apply's two passes on v_mfma_f64_16x16x4f64 (NB = ⌈k/16⌉ blocks of 16
// columns; one column costs a whole block, but the passes are bound by
// reading L and by latency, not by MFMA time; lane layout: A[m][kk] from lane kk·16 + m, B[kk][c] from lane
// kk·16 + c, result register e of lane l is C[l/16 + 4e][l%16]).
//
// part[s][a][c] = Σ_{i in chunk s} W[i][a]·R[i][c]: A = Wᵀ (16 landmarks ×
// 4 rows), B = R (4 rows × 16 columns).  A wave covers 64 landmarks as 4
// MFMA tiles (tile t: landmarks a0 + 16t + m) and walks its chunk 4 rows at a
// time, the next group's loads issued before the current group's MFMAs.
template <typename T, int NB>
__global__ __launch_bounds__(256) void nys_wtr_mfma(int64_t n, int r, int k,
                                                    const T* __restrict__ W,
                                                    const double* __restrict__ R, int64_t chunk,
                                                    double* __restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, q = lane >> 4;
  const int a0 = (blockIdx.x * 4 + wave) * 64;
  if (a0 >= r) return;
  const int s = blockIdx.y;
  const int64_t beg = (int64_t)s * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  f64x4 acc[4][NB];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[t][b] = f64x4{0};
  auto load = [&](int64_t i0, double (&w)[4], double (&v)[NB]) {
    const int64_t i = i0 + q;
    const bool ok = i < end;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int a = a0 + 16 * t + m;
      w[t] = ok && a < r ? (double)W[i * r + a] : 0.0;
    }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int c = 16 * b + m;
      v[b] = ok && c < k ? R[i * k + c] : 0.0;
    }
  };
  double w[4], v[NB];
  if (beg < end) load(beg, w, v);
  for (int64_t i0 = beg; i0 < end; i0 += 4) {
    double wn[4], vn[NB];
    if (i0 + 4 < end) load(i0 + 4, wn, vn);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int b = 0; b < NB; ++b)
        acc[t][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(w[t], v[b], acc[t][b], 0, 0, 0);
    if (i0 + 4 < end) {
#pragma unroll
      for (int t = 0; t < 4; ++t) w[t] = wn[t];
#pragma unroll
      for (int b = 0; b < NB; ++b) v[b] = vn[b];
    }
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int c = 16 * b + m;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int a = a0 + 16 * t + q + 4 * e;
        if (a < r && c < k) part[((int64_t)s * r + a) * k + c] = acc[t][b][e];
      }
    }
}

// Z = (R − W·u)/s: A = W (16 rows × 4 landmarks), B = u (4 landmarks × 16
// columns).  A wave owns 16 rows and walks the landmarks 16 at a time: lane
// (q, m) loads landmarks a0 + 4q .. a0 + 4q + 3 of row m, and step t takes
// landmark a0 + 4q + t as its reduction index q.
template <typename T, int NB>
__global__ __launch_bounds__(256) void nys_apply_z_mfma(int64_t n, int r, int k,
                                                        const T* __restrict__ W,
                                                        const double* __restrict__ u,
                                                        const double* __restrict__ R,
                                                        double inv_s, double* __restrict__ Z) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int m = lane & 15, q = lane >> 4;
  const int64_t i0 = ((int64_t)blockIdx.x * 4 + wave) * 16;
  if (i0 >= n) return;
  const int64_t i = i0 + m;  // the row this lane loads
  f64x4 acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = f64x4{0};
  auto load = [&](int a0, double (&w)[4], double (&v)[4][NB]) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int a = a0 + 4 * q + t;
      const bool ok = a < r;
      w[t] = ok && i < n ? (double)W[i * r + a] : 0.0;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int c = 16 * b + m;
        v[t][b] = ok && c < k ? u[(int64_t)a * k + c] : 0.0;
      }
    }
  };
  double w[4], v[4][NB];
  load(0, w, v);
  for (int a0 = 0; a0 < r; a0 += 16) {
    double wn[4], vn[4][NB];
    if (a0 + 16 < r) load(a0 + 16, wn, vn);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int b = 0; b < NB; ++b)
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(w[t], v[t][b], acc[b], 0, 0, 0);
    if (a0 + 16 < r) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        w[t] = wn[t];
#pragma unroll
        for (int b = 0; b < NB; ++b) v[t][b] = vn[t][b];
      }
    }
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int c = 16 * b + m;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t row = i0 + q + 4 * e;
      if (row < n && c < k) Z[row * k + c] = (R[row * k + c] - acc[b][e]) * inv_s;
    }
  }
}

// Lower Cholesky factor of the SPD matrix A (r×r, row-major; zeros above
// the diagonal).  Returns false if A is not numerically positive definite.
// Dot product with eight independent partial sums combined in a fixed order
// (vectorisable, and the same result on every run).
double dot8(const double* a, const double* b, int n) {
  double s[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int q = 0;
  for (; q + 8 <= n; q += 8)
    for (int t = 0; t < 8; ++t) s[t] += a[q + t] * b[q + t];
  double tot = ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
  for (; q < n; ++q) tot += a[q] * b[q];
  return tot;
}

// f(i) for i in [0, n) on the host's threads, in contiguous static chunks
// (each output is computed by one thread, so results do not depend on the
// thread count).
template <typename F>
void host_parallel_for(int n, F f) {
  const int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (nt == 1 || n < 64) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> team;
  const int chunk = (n + nt - 1) / nt;
  for (int t = 0; t < nt; ++t) {
    const int b = t * chunk, e = std::min(n, b + chunk);
    if (b >= e) break;
    team.emplace_back([=, &f] {
      for (int i = b; i < e; ++i) f(i);
    });
  }
  for (auto& th : team) th.join();
}

// Sense-reversing spin barrier for a team of host threads.
class SpinBarrier {
 public:
  explicit SpinBarrier(int n) : n_(n) {}
  void wait() {
    const int gen = gen_.load(std::memory_order_acquire);
    if (count_.fetch_add(1, std::memory_order_acq_rel) == n_ - 1) {
      count_.store(0, std::memory_order_relaxed);
      gen_.store(gen + 1, std::memory_order_release);
    } else {
      while (gen_.load(std::memory_order_acquire) == gen) std::this_thread::yield();
    }
  }

 private:
  const int n_;
  std::atomic<int> count_{0};
  std::atomic<int> gen_{0};
};

// Column j of the factor: L[i][j] = (A[i][j] − Σ_{k<j} L[i][k]·L[j][k]) / L[j][j]
// for i > j, with L[j][j] = √(A[j][j] − Σ_{k<j} L[j][k]²).  Every entry is
// computed by the same dot8 whether the columns' rows are shared out among
// threads or not, so the factor does not depend on the thread count.
bool chol_lower(const std::vector<double>& A, int r, std::vector<double>& L) {
  L.assign((size_t)r * r, 0.0);
  const int nt = r < 512 ? 1 : (int)std::max(1u, std::min(8u, std::thread::hardware_concurrency()));
  auto diag = [&](int j) { return A[(size_t)j * r + j] - dot8(&L[(size_t)j * r], &L[(size_t)j * r], j); };
  if (nt == 1) {
    for (int j = 0; j < r; ++j) {
      const double s = diag(j);
      if (!(s > 0.0)) return false;
      const double d = std::sqrt(s);
      L[(size_t)j * r + j] = d;
      const double* lj = &L[(size_t)j * r];
      for (int i = j + 1; i < r; ++i)
        L[(size_t)i * r + j] = (A[(size_t)i * r + j] - dot8(&L[(size_t)i * r], lj, j)) / d;
    }
    return true;
  }
  // One barrier per column: each thread forms the diagonal itself (the same
  // value in every thread), thread 0 stores it, and the rows below are
  // shared out in a fixed interleave.
  SpinBarrier bar(nt);
  std::atomic<bool> ok{true};
  auto work = [&](int t) {
    for (int j = 0; j < r; ++j) {
      const double s = diag(j);
      if (!(s > 0.0)) {
        if (t == 0) ok.store(false);
        return;  // every thread sees the same s and leaves at the same column
      }
      const double d = std::sqrt(s);
      if (t == 0) L[(size_t)j * r + j] = d;
      const double* lj = &L[(size_t)j * r];
      for (int i = j + 1 + t; i < r; i += nt)
        L[(size_t)i * r + j] = (A[(size_t)i * r + j] - dot8(&L[(size_t)i * r], lj, j)) / d;
      bar.wait();
    }
  };
  std::vector<std::thread> team;
  for (int t = 1; t < nt; ++t) team.emplace_back(work, t);
  work(0);
  for (auto& th : team) th.join();
  return ok.load();
}

// Inverse of the lower-triangular L, returned transposed: Mt[j][i] =
// (L⁻¹)[i][j] (so column j of L⁻¹ is contiguous), zeros elsewhere.
void tri_inverse_t(const std::vector<double>& L, int r, std::vector<double>& Mt) {
  Mt.assign((size_t)r * r, 0.0);
  host_parallel_for(r, [&](int j) {  // columns of L⁻¹ are independent
    double* mj = &Mt[(size_t)j * r];
    mj[j] = 1.0 / L[(size_t)j * r + j];
    for (int i = j + 1; i < r; ++i) {
      const double* li = &L[(size_t)i * r];
      mj[i] = -dot8(li + j, mj + j, i - j) / li[i];
    }
  });
}

// In-place inverse of the SPD matrix A (r×r, row-major): A = LLᵀ,
// A⁻¹ = L⁻ᵀL⁻¹.  Returns false if A is not numerically positive definite.
bool spd_inverse(std::vector<double>& A, int r) {
  std::vector<double> L, Mt;
  if (!chol_lower(A, r, L)) return false;
  tri_inverse_t(L, r, Mt);
  // A⁻¹[a][b] = Σ_{i ≥ max(a,b)} L⁻¹[i][a]·L⁻¹[i][b] = Σ_i Mt[a][i]·Mt[b][i].
  host_parallel_for(r, [&](int a) {
    const double* ma = &Mt[(size_t)a * r];
    for (int b = 0; b <= a; ++b) {
      const double s = dot8(ma + a, &Mt[(size_t)b * r] + a, r - a);
      A[(size_t)a * r + b] = s;
      A[(size_t)b * r + a] = s;
    }
  });
  return true;
}

unsigned grid_for(int64_t count) {
  const int64_t b = (count + 255) / 256;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

// Farthest-point landmarks into sel (device, r ints); dmin n doubles, bval/
// bidx `blocks` slots each, counter one zero-initialised uint.
template <typename T>
int fps_select(const Problem& p, int r, int* sel, double* dmin, double* bval, int64_t* bidx,
               unsigned* counter, int blocks, hipStream_t st) {
  const int64_t n = p.n;
  if (hipMemsetAsync(sel, 0, 4, st) != hipSuccess || hipMemsetAsync(counter, 0, 4, st) != hipSuccess)
    return set_error(HIGP_ERR_HIP, "hipMemsetAsync failed");
  hipLaunchKernelGGL(fill_inf, dim3(grid_for(n)), dim3(256), 0, st, n, dmin);
  for (int j = 1; j < r; ++j)
    hipLaunchKernelGGL((fps_step<T>), dim3(blocks), dim3(kThreads), 0, st, n, p.d,
                       static_cast<const T*>(p.X), sel, j, dmin, bval, bidx, counter);
  return hipGetLastError() == hipSuccess ? HIGP_OK
                                         : set_error(HIGP_ERR_HIP, "landmark selection failed");
}

template <typename T>
int build_impl(const Problem& p, int r, int kmax, NysPrec* P, hipStream_t st) {
  const int64_t n = p.n;
  auto rup = [](size_t b) { return (b + 255) / 256 * 256; };
  const int fps_blocks = (int)std::min<int64_t>(256, (n + kThreads - 1) / kThreads);
  const int S = wtr_splits(n, r, kmax);
  const int64_t chunk = (n + S - 1) / S;
  // Persistent part: L, C⁻¹, sel.  Work part (apply): partials, T, u.
  const size_t l_bytes = rup((size_t)n * r * sizeof(T));
  const size_t rr_bytes = rup((size_t)r * r * 8);
  const size_t sel_bytes = rup((size_t)r * 4);
  const size_t part_bytes = rup((size_t)S * r * kmax * 8);
  const size_t t_bytes = rup((size_t)r * kmax * 8);
  const size_t keep = l_bytes + rr_bytes + sel_bytes + part_bytes + 2 * t_bytes;
  // Build-only scratch: K_nr, dmin, block argmax slots, K_rr / R⁻¹ / C
  // (one r×r FP64 slot, reused), Gram partials.
  const int gS = (int)std::max<int64_t>(1, std::min<int64_t>(8, n / 8192));
  const int64_t gchunk = (n + gS - 1) / gS;
  const size_t o_w = 0, o_dmin = o_w + l_bytes, o_bv = o_dmin + rup((size_t)n * 8),
               o_cnt = o_bv + rup((size_t)fps_blocks * 16), o_rr = o_cnt + 256,
               o_gp = o_rr + rr_bytes, tmp_bytes = o_gp + rup((size_t)gS * r * r * 8);
  void* mem = nullptr;
  HIGP_TRY(scratch_alloc(&mem, keep, st));
  void* tmp = nullptr;
  if (int rc = scratch_alloc(&tmp, tmp_bytes, st)) {
    scratch_free(mem, st);
    return rc;
  }
  char* base = static_cast<char*>(mem);
  P->mem = mem;
  P->n = n;
  P->r = r;
  P->kmax = kmax;
  P->prec = p.prec;
  P->s = p.s;
  P->S = S;
  P->chunk = chunk;
  P->W = base;
  P->Cinv = reinterpret_cast<double*>(base + l_bytes);
  P->sel = reinterpret_cast<int*>(base + l_bytes + rr_bytes);
  P->part = reinterpret_cast<double*>(base + l_bytes + rr_bytes + sel_bytes);
  P->Tm = reinterpret_cast<double*>(base + l_bytes + rr_bytes + sel_bytes + part_bytes);
  P->u = P->Tm + t_bytes / 8;
  char* tb = static_cast<char*>(tmp);
  T* Knr = reinterpret_cast<T*>(tb + o_w);
  double* dmin = reinterpret_cast<double*>(tb + o_dmin);
  double* bval = reinterpret_cast<double*>(tb + o_bv);
  int64_t* bidx = reinterpret_cast<int64_t*>(bval + fps_blocks);
  unsigned* counter = reinterpret_cast<unsigned*>(tb + o_cnt);
  double* RR = reinterpret_cast<double*>(tb + o_rr);
  double* gpart = reinterpret_cast<double*>(tb + o_gp);
  auto fail = [&](int rc) {
    scratch_free(tmp, st);
    scratch_free(mem, st);
    P->mem = nullptr;
    return rc;
  };
  const T* X = static_cast<const T*>(p.X);
  if (int rc = fps_select<T>(p, r, P->sel, dmin, bval, bidx, counter, fps_blocks, st))
    return fail(rc);
  // K_nr = k(X, landmarks).
  const double xs = coord_scale(p.kernel, sizeof(T) == 8 ? HIGP_FP64 : HIGP_FP32, p.l);
  if (p.kernel == HIGP_GAUSSIAN)
    hipLaunchKernelGGL((nys_kernel_matrix<T, HIGP_GAUSSIAN>), dim3(grid_for(n * r)), dim3(256), 0,
                       st, n, r, p.d, X, (const int*)P->sel, xs, Knr);
  else
    hipLaunchKernelGGL((nys_kernel_matrix<T, HIGP_MATERN32>), dim3(grid_for(n * r)), dim3(256),
                       0, st, n, r, p.d, X, (const int*)P->sel, xs, Knr);
  // K_rr + εI = RRᵀ on the host, R⁻¹ back to the device.
  const double xs64 = coord_scale(p.kernel, HIGP_FP64, p.l);
  if (p.kernel == HIGP_GAUSSIAN)
    hipLaunchKernelGGL((nys_krr_f64<T, HIGP_GAUSSIAN>), dim3(grid_for((int64_t)r * r)), dim3(256),
                       0, st, r, p.d, X, (const int*)P->sel, xs64, RR);
  else
    hipLaunchKernelGGL((nys_krr_f64<T, HIGP_MATERN32>), dim3(grid_for((int64_t)r * r)), dim3(256),
                       0, st, r, p.d, X, (const int*)P->sel, xs64, RR);
  if (hipGetLastError() != hipSuccess)
    return fail(set_error(HIGP_ERR_HIP, "preconditioner build launch failed"));
  std::vector<double> A((size_t)r * r), F, Mt;
  if (hipMemcpyAsync(A.data(), RR, A.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(set_error(HIGP_ERR_HIP, "copy of the landmark block failed"));
  // ε = 1e-8; should rounding still leave K_rr + εI indefinite (landmarks
  // that coincide), ε grows by 100× up to 1e-2.
  bool ok = false;
  for (double eps = kNysJitter; !ok && eps <= 1e-2 * 1.0001; eps *= 100.0) {
    std::vector<double> Aj = A;
    for (int a = 0; a < r; ++a) Aj[(size_t)a * r + a] += eps;
    ok = chol_lower(Aj, r, F);
  }
  if (!ok)
    return fail(set_error(HIGP_ERR_INVALID_ARG, "landmark kernel block is not positive definite"));
  tri_inverse_t(F, r, Mt);
  for (int a = 0; a < r; ++a)  // R⁻¹[a][b] = Mt[b][a] (lower triangular)
    for (int b = 0; b < r; ++b) A[(size_t)a * r + b] = b <= a ? Mt[(size_t)b * r + a] : 0.0;
  if (hipMemcpyAsync(RR, A.data(), A.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess)
    return fail(set_error(HIGP_ERR_HIP, "upload of the landmark factor failed"));
  // L = K_nr·R⁻ᵀ, then C = (s/f²)·I + LᵀL.
  hipLaunchKernelGGL((nys_tri_gemm<T>), dim3((unsigned)((n + 63) / 64), (r + 63) / 64), dim3(256),
                     0, st, n, r, (const T*)Knr, (const double*)RR, static_cast<T*>(P->W));
  const int tiles = (r + kGT - 1) / kGT;
  hipLaunchKernelGGL((nys_gram<T>), dim3(tiles, tiles, gS), dim3(256), 0, st, n, r,
                     (const T*)P->W, gchunk, gpart);
  hipLaunchKernelGGL(nys_gram_finish, dim3(grid_for((int64_t)r * r)), dim3(256), 0, st, r, gS,
                     (const double*)gpart, p.s / (p.f * p.f), RR);
  if (hipGetLastError() != hipSuccess)
    return fail(set_error(HIGP_ERR_HIP, "preconditioner build launch failed"));
  if (hipMemcpyAsync(A.data(), RR, A.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(set_error(HIGP_ERR_HIP, "copy of the Nyström core failed"));
  if (!spd_inverse(A, r))
    return fail(set_error(HIGP_ERR_INVALID_ARG, "Nyström core matrix is not positive definite"));
  if (hipMemcpyAsync(P->Cinv, A.data(), A.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(set_error(HIGP_ERR_HIP, "upload of the Nyström core failed"));
  scratch_free(tmp, st);
  return HIGP_OK;
}

template <typename T, int NB>
void launch_wtr_mfma(const NysPrec& P, int k, const double* R, hipStream_t st) {
  hipLaunchKernelGGL((nys_wtr_mfma<T, NB>), dim3((P.r + 255) / 256, P.S), dim3(256), 0, st, P.n,
                     P.r, k, static_cast<const T*>(P.W), R, P.chunk, P.part);
}

template <typename T, int NB>
void launch_apply_z_mfma(const NysPrec& P, int k, const double* R, double* Z, hipStream_t st) {
  hipLaunchKernelGGL((nys_apply_z_mfma<T, NB>), dim3((unsigned)((P.n + 63) / 64)), dim3(256), 0,
                     st, P.n, P.r, k, static_cast<const T*>(P.W), (const double*)P.u, R,
                     1.0 / P.s, Z);
}

template <typename T>
int apply_impl(const NysPrec& P, int k, const double* R, double* Z, hipStream_t st) {
  const int nb = (k + 15) / 16;
  if (nb == 1) launch_wtr_mfma<T, 1>(P, k, R, st);
  else if (nb == 2) launch_wtr_mfma<T, 2>(P, k, R, st);
  else if (nb == 3) launch_wtr_mfma<T, 3>(P, k, R, st);
  else launch_wtr_mfma<T, 4>(P, k, R, st);
  const int rk = P.r * k;
  hipLaunchKernelGGL(nys_reduce_parts, dim3((unsigned)((rk + 31) / 32)), dim3(256), 0, st, rk,
                     P.S, (const double*)P.part, P.Tm);
  hipLaunchKernelGGL(nys_cinv_t, dim3((unsigned)((P.r + 3) / 4)), dim3(256), 0, st, P.r, k,
                     (const double*)P.Cinv, (const double*)P.Tm, P.u);
  if (nb == 1) launch_apply_z_mfma<T, 1>(P, k, R, Z, st);
  else if (nb == 2) launch_apply_z_mfma<T, 2>(P, k, R, Z, st);
  else if (nb == 3) launch_apply_z_mfma<T, 3>(P, k, R, Z, st);
  else launch_apply_z_mfma<T, 4>(P, k, R, Z, st);
  return hipGetLastError() == hipSuccess ? HIGP_OK
                                         : set_error(HIGP_ERR_HIP, "preconditioner apply failed");
}

}  // namespace

int nys_build(const Problem& p, int rank, int kmax, NysPrec* P, hipStream_t st) {
  *P = NysPrec{};
  const int r = (int)std::min<int64_t>(rank, p.n);
  if (r < 1 || kmax < 1 || kmax > 64)
    return set_error(HIGP_ERR_INVALID_ARG, "bad Nyström rank or width");
  if (!(p.s > 0.0))
    return set_error(HIGP_ERR_INVALID_ARG, "the Nyström preconditioner needs s > 0");
  if (p.prec == HIGP_FP64) return build_impl<double>(p, r, kmax, P, st);
  return build_impl<float>(p, r, kmax, P, st);
}

int nys_apply(const NysPrec& P, int k, const double* R, double* Z, hipStream_t st) {
  if (k > P.kmax) return set_error(HIGP_ERR_INVALID_ARG, "Nyström apply wider than built");
  if (P.prec == HIGP_FP64) return apply_impl<double>(P, k, R, Z, st);
  return apply_impl<float>(P, k, R, Z, st);
}

size_t nys_bytes(int64_t n, int rank, int kmax, int prec) {
  const int r = (int)std::min<int64_t>(rank, n);
  const int S = wtr_splits(n, r, kmax);
  auto rup = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t es = prec == HIGP_FP64 ? 8 : 4;
  return rup((size_t)n * r * es) + rup((size_t)r * r * 8) + rup((size_t)r * 4) +
         rup((size_t)S * r * kmax * 8) + 2 * rup((size_t)r * kmax * 8);
}

int fps_landmarks(const Problem& p, int rank, int* sel_host, hipStream_t st) {
  const int r = (int)std::min<int64_t>(rank, p.n);
  const int blocks = (int)std::min<int64_t>(256, (p.n + kThreads - 1) / kThreads);
  auto rup = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t bytes = rup((size_t)r * 4) + rup((size_t)p.n * 8) + rup((size_t)blocks * 16) + 256;
  void* mem = nullptr;
  HIGP_TRY(scratch_alloc(&mem, bytes, st));
  char* b = static_cast<char*>(mem);
  int* sel = reinterpret_cast<int*>(b);
  double* dmin = reinterpret_cast<double*>(b + rup((size_t)r * 4));
  double* bval = reinterpret_cast<double*>(b + rup((size_t)r * 4) + rup((size_t)p.n * 8));
  int64_t* bidx = reinterpret_cast<int64_t*>(bval + blocks);
  unsigned* counter = reinterpret_cast<unsigned*>(b + rup((size_t)r * 4) + rup((size_t)p.n * 8) +
                                                  rup((size_t)blocks * 16));
  int rc = p.prec == HIGP_FP64
               ? fps_select<double>(p, r, sel, dmin, bval, bidx, counter, blocks, st)
               : fps_select<float>(p, r, sel, dmin, bval, bidx, counter, blocks, st);
  if (rc == HIGP_OK &&
      (hipMemcpyAsync(sel_host, sel, (size_t)r * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
       hipStreamSynchronize(st) != hipSuccess))
    rc = set_error(HIGP_ERR_HIP, "landmark copy failed");
  scratch_free(mem, st);
  return rc;
}

void nys_free(NysPrec& P, hipStream_t st) {
  if (P.mem) scratch_free(P.mem, st);
  P.mem = nullptr;
}

}  // namespace higp
