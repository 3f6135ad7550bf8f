// Lanczos kernels shared by the single-call SLQ (higp_slq_logdet) and the
// serving engine.  N probe columns advance together; the breakdown decision
// (β_j ≤ 1e-12·max_{i≤j}|α_i|) is taken on the device in FP64, so a run needs
// no host round trip per step.  Step j of a live column c:
//     w = A q_j;  α_j = q_jᵀw;  w ← w − α_j q_j − β_{j−1} q_{j−1};
//     (full reorthogonalisation) w ← w − Σ_{t≤j} (q_tᵀw) q_t;  β_j = ‖w‖;
//     q_{j+1} = w/β_j
// with A = isq²·K̂ (isq = 1/√(f²+s) with Jacobi, 1 without).  α_j and β_j are
// recorded in hist arrays; steps[c] counts the recorded α's (the size of T).
#pragma once

#include "reduce.h"

namespace higp {
namespace {

constexpr int kCoefBlocks = 128;  // row blocks of the reorthogonalisation dots

struct LzState {
  double* Q;         // (m+1) blocks of n×N, FP64 Lanczos vectors
  double* W;         // n×N FP64 work vector
  double* alpha;     // N: α of the current step
  double* beta;      // N: β of the current step
  double* beta_prev; // N
  double* amax;      // N: max |α| so far
  double* ahist;     // m×N recorded α
  double* bhist;     // m×N recorded β
  double* coef;      // (m+1)×64 reorthogonalisation coefficients
  double* part;      // (m+1)×kCoefBlocks×64 partial dots
  double* work;      // reduction partials (red_grid(n).blocks × 64)
  int* live;         // N
  int* steps;        // N
  int* nlive;        // 1
  unsigned* counter; // 1, zero-initialised
  volatile int* nlive_host;  // optional pinned host mirror of *nlive
};

// W = isq·WW; α = Σ q_j·W per column.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void lz_alpha(int64_t n, int N, int64_t chunk,
                                                        const T* __restrict__ WW, double isq,
                                                        const double* __restrict__ Qj,
                                                        LzState S) {
  __shared__ double sh[kRedThreads];
  const ColLanes L = col_lanes(N);
  const int c = L.c;
  const int r0 = L.r0;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  double acc = 0.0;
  if (c < N)
    for (int64_t i = beg + r0; i < end; i += L.step) {
      const int64_t o = i * N + c;
      const double w = isq * (double)WW[o];
      S.W[o] = w;
      acc += Qj[o] * w;
    }
  (void)block_colsum_finish(acc, N, S.work, S.counter, sh,
                            [&](int col, double tot) { S.alpha[col] = tot; });
}

// W ← W − α q_j − β_prev q_{j−1}.
__global__ void lz_three_term(int64_t count, int N, const double* __restrict__ Qj,
                              const double* __restrict__ Qjm1, LzState S) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % N);
    double w = S.W[e] - S.alpha[c] * Qj[e];
    if (Qjm1) w -= S.beta_prev[c] * Qjm1[e];
    S.W[e] = w;
  }
}

// part[t][b][c] = Σ_{i in row block b} Q_t[i][c]·W[i][c]; grid (blocks, j+1).
__global__ __launch_bounds__(kRedThreads) void lz_coef(int64_t n, int N, int64_t chunk, LzState S) {
  __shared__ double sh[kRedThreads];
  const ColLanes L = col_lanes(N);
  const int c = L.c;
  const int r0 = L.r0;
  const int t = blockIdx.y;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  const double* Qt = S.Q + (int64_t)t * n * N;
  double acc = 0.0;
  if (c < N)
    for (int64_t i = beg + r0; i < end; i += L.step) acc += Qt[i * N + c] * S.W[i * N + c];
  block_colsum(acc, N, sh);
  if ((int)threadIdx.x < N) S.part[((int64_t)t * gridDim.x + blockIdx.x) * 64 + threadIdx.x] = sh[threadIdx.x];
}

// coef[t][c] = Σ_b part[t][b][c] in block order; one block per t.
__global__ void lz_coef_final(int nb, LzState S) {
  const int t = blockIdx.x;
  const int c = threadIdx.x;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += S.part[((int64_t)t * nb + b) * 64 + c];
  S.coef[t * 64 + c] = s;
}

// W ← W − Σ_{t<nt} coef[t]·Q_t, β = ‖W‖; then record α_j, β_j and decide
// breakdown / end for every live column (last block).
__global__ __launch_bounds__(kRedThreads) void lz_reorth_norm(int64_t n, int N, int64_t chunk,
                                                              int nt, int j, int m, LzState S) {
  __shared__ double sh[kRedThreads];
  const ColLanes L = col_lanes(N);
  const int c = L.c;
  const int r0 = L.r0;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  double acc = 0.0;
  if (c < N)
    for (int64_t i = beg + r0; i < end; i += L.step) {
      const int64_t o = i * N + c;
      double w = S.W[o];
      for (int t = 0; t < nt; ++t) w -= S.coef[t * 64 + c] * S.Q[(int64_t)t * n * N + o];
      S.W[o] = w;
      acc += w * w;
    }
  const bool last = block_colsum_finish(acc, N, S.work, S.counter, sh, [&](int col, double tot) {
    const double b = sqrt(tot);
    S.beta[col] = b;
    if (!S.live[col]) return;
    const double a = S.alpha[col];
    const double am = fmax(S.amax[col], fabs(a));
    S.amax[col] = am;
    S.ahist[(int64_t)j * N + col] = a;
    S.steps[col] = j + 1;
    if (j == m - 1 || b <= 1e-12 * am) {
      S.live[col] = 0;
    } else {
      S.bhist[(int64_t)j * N + col] = b;
    }
  });
  if (last && threadIdx.x == 0) {
    int nl = 0;
    for (int col = 0; col < N; ++col) nl += S.live[col];
    *S.nlive = nl;
    if (S.nlive_host) *S.nlive_host = nl;
  }
}

// Q_{j+1} = live ? W/β : 0; QW = isq·Q_{j+1} in the MatVec precision;
// β_prev = live ? β : 0.
template <typename T>
__global__ void lz_next(int64_t count, int N, double* __restrict__ Qn, T* __restrict__ QW,
                        double isq, LzState S) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % N);
    const bool lv = S.live[c] != 0;
    const double q = lv ? S.W[e] / S.beta[c] : 0.0;
    Qn[e] = q;
    QW[e] = (T)(isq * q);
    if (e < N) S.beta_prev[e] = S.live[e] ? S.beta[e] : 0.0;
  }
}

// Q_0 = z/‖z‖ (zn2 = ‖z‖²), QW = isq·Q_0; resets the per-column state.
template <typename T>
__global__ void lz_first(int64_t count, int N, const T* __restrict__ Z,
                         const double* __restrict__ zn2, T* __restrict__ QW, double isq,
                         LzState S) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % N);
    const double q = zn2[c] > 0.0 ? (double)Z[e] / sqrt(zn2[c]) : 0.0;
    S.Q[e] = q;
    QW[e] = (T)(isq * q);
    if (e < N) {
      S.live[e] = zn2[e] > 0.0 ? 1 : 0;
      S.steps[e] = 0;
      S.amax[e] = 0.0;
      S.beta_prev[e] = 0.0;
    }
    if (e == 0) *S.nlive = N;
  }
}

inline unsigned lz_blocks(int64_t count) {
  const int64_t b = (count + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

// Bytes of device state for n points, N probes, m steps (besides QW/WW).
inline size_t lz_state_bytes(int64_t n, int N, int m) {
  const size_t nN = (size_t)n * N;
  const RedGrid g = red_grid(n);
  auto r = [](size_t b) { return (b + 255) / 256 * 256; };
  return r((size_t)(m + 1) * nN * 8) + r(nN * 8) + r(4 * 64 * 8) + 2 * r((size_t)m * 64 * 8) +
         r((size_t)(m + 1) * 64 * 8) + r((size_t)(m + 1) * kCoefBlocks * 64 * 8) +
         r((size_t)g.blocks * 64 * 8) + r(3 * 64 * 4) + r(8);
}

// Carve an LzState out of `base` (lz_state_bytes bytes).
inline LzState lz_carve(char* base, int64_t n, int N, int m) {
  const size_t nN = (size_t)n * N;
  const RedGrid g = red_grid(n);
  size_t off = 0;
  auto take = [&](size_t b) {
    char* p = base + off;
    off += (b + 255) / 256 * 256;
    return p;
  };
  LzState S{};
  S.Q = (double*)take((size_t)(m + 1) * nN * 8);
  S.W = (double*)take(nN * 8);
  double* sc = (double*)take(4 * 64 * 8);
  S.alpha = sc;
  S.beta = sc + 64;
  S.beta_prev = sc + 128;
  S.amax = sc + 192;
  S.ahist = (double*)take((size_t)m * 64 * 8);
  S.bhist = (double*)take((size_t)m * 64 * 8);
  S.coef = (double*)take((size_t)(m + 1) * 64 * 8);
  S.part = (double*)take((size_t)(m + 1) * kCoefBlocks * 64 * 8);
  S.work = (double*)take((size_t)g.blocks * 64 * 8);
  int* in = (int*)take(3 * 64 * 4);
  S.live = in;
  S.steps = in + 64;
  S.nlive = in + 128;
  S.counter = (unsigned*)take(8);
  S.nlive_host = nullptr;
  return S;
}

// Kernels of Lanczos step j (after the MatVec WW = K̂·QW of this step).
template <typename T>
inline void lz_launch_step(int64_t n, int N, int j, int m, bool reorth, double isq,
                           const T* WW, T* QW, LzState S, hipStream_t st) {
  const size_t nN = (size_t)n * N;
  const RedGrid g = red_grid(n);
  const int64_t cchunk = ((n + kCoefBlocks - 1) / kCoefBlocks + 3) / 4 * 4;
  const int cblocks = (int)((n + cchunk - 1) / cchunk);
  double* Qj = S.Q + (size_t)j * nN;
  hipLaunchKernelGGL((lz_alpha<T>), dim3(g.blocks), dim3(kRedThreads), 0, st, n, N, g.chunk, WW,
                     isq, (const double*)Qj, S);
  hipLaunchKernelGGL(lz_three_term, dim3(lz_blocks(nN)), dim3(256), 0, st, (int64_t)nN, N,
                     (const double*)Qj, j > 0 ? (const double*)(Qj - nN) : nullptr, S);
  if (reorth) {
    hipLaunchKernelGGL(lz_coef, dim3(cblocks, j + 1), dim3(kRedThreads), 0, st, n, N, cchunk, S);
    hipLaunchKernelGGL(lz_coef_final, dim3(j + 1), dim3(64), 0, st, cblocks, S);
  }
  hipLaunchKernelGGL(lz_reorth_norm, dim3(g.blocks), dim3(kRedThreads), 0, st, n, N, g.chunk,
                     reorth ? j + 1 : 0, j, m, S);
  if (j + 1 < m)
    hipLaunchKernelGGL((lz_next<T>), dim3(lz_blocks(nN)), dim3(256), 0, st, (int64_t)nN, N,
                       Qj + nN, QW, isq, S);
}

}  // namespace
}  // namespace higp
