// Stochastic Lanczos quadrature for log|K̂| (eq. (1) of the paper with the
// SLQ estimator of Ubaru et al. 2017, "Gaussian Processes" section).
//
// log|K̂| = log|M| + log|M^{-1/2} K̂ M^{-1/2}|.  With M = diag(K̂) = (f²+s)·I
// (stationary kernels) the operator is K̂/(f²+s) and log|M| = n·log(f²+s);
// without preconditioning M = I.  For each probe z the Lanczos process runs
// from q₀ = z/‖z‖:
//     w = A q_j;  α_j = q_jᵀ w;  w ← w − α_j q_j − β_{j−1} q_{j−1};
//     (full reorthogonalisation) w ← w − Σ_{t≤j} (q_tᵀw) q_t;  β_j = ‖w‖;
//     q_{j+1} = w / β_j,
// stopping after nsteps steps or when β_j ≤ 1e-12·max_{i≤j}|α_i|.  The
// quadrature is ‖z‖²·Σ_k τ_k²·log θ_k with θ, τ the eigenvalues and first
// eigenvector components of the tridiagonal T, computed in FP64 on the host.
//
// All probes advance together: one MatVec with k = nprobe columns per step.
// Lanczos vectors are kept in FP64 on the device ((nsteps+1)·n·nprobe·8 B);
// the MatVec input is the probe block rounded to the problem's precision.
#include <cmath>
#include <vector>

#include "reduce.h"

namespace higp {
namespace {

constexpr int kCoefBlocks = 128;  // row blocks of the reorthogonalisation dots

// W = isq·WW; α = Σ q_j·W per column.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void lz_alpha(int64_t n, int N, int64_t chunk,
                                                        const T* __restrict__ WW, double isq,
                                                        const double* __restrict__ Qj,
                                                        double* __restrict__ W, double* alpha,
                                                        double* work, unsigned* counter) {
  __shared__ double sh[kRedThreads];
  const int c = threadIdx.x & 63;
  const int r0 = threadIdx.x >> 6;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  double acc = 0.0;
  if (c < N)
    for (int64_t i = beg + r0; i < end; i += 4) {
      const int64_t o = i * N + c;
      const double w = isq * (double)WW[o];
      W[o] = w;
      acc += Qj[o] * w;
    }
  (void)block_colsum_finish(acc, N, work, counter, sh,
                            [&](int col, double tot) { alpha[col] = tot; });
}

// W ← W − α q_j − β_prev q_{j−1}.
__global__ void lz_three_term(int64_t count, int N, double* __restrict__ W,
                              const double* __restrict__ Qj, const double* __restrict__ Qjm1,
                              const double* __restrict__ alpha,
                              const double* __restrict__ beta_prev) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % N);
    double w = W[e] - alpha[c] * Qj[e];
    if (Qjm1) w -= beta_prev[c] * Qjm1[e];
    W[e] = w;
  }
}

// partial[t][b][c] = Σ_{i in row block b} Q_t[i][c]·W[i][c]; grid (blocks, j+1).
__global__ __launch_bounds__(kRedThreads) void lz_coef(int64_t n, int N, int64_t chunk,
                                                       const double* __restrict__ Q,
                                                       const double* __restrict__ W,
                                                       double* __restrict__ partial) {
  __shared__ double sh[kRedThreads];
  const int c = threadIdx.x & 63;
  const int r0 = threadIdx.x >> 6;
  const int t = blockIdx.y;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  const double* Qt = Q + (int64_t)t * n * N;
  double acc = 0.0;
  if (c < N)
    for (int64_t i = beg + r0; i < end; i += 4) acc += Qt[i * N + c] * W[i * N + c];
  sh[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x < 64) {
    const int tid = threadIdx.x;
    partial[((int64_t)t * gridDim.x + blockIdx.x) * 64 + tid] =
        ((sh[tid] + sh[tid + 64]) + sh[tid + 128]) + sh[tid + 192];
  }
}

// coef[t][c] = Σ_b partial[t][b][c] in block order; one block per t.
__global__ void lz_coef_final(int nb, const double* __restrict__ partial, double* coef) {
  const int t = blockIdx.x;
  const int c = threadIdx.x;
  double s = 0.0;
  for (int b = 0; b < nb; ++b) s += partial[((int64_t)t * nb + b) * 64 + c];
  coef[t * 64 + c] = s;
}

// W ← W − Σ_{t≤j} coef[t]·Q_t (if reorth), then β = ‖W‖ per column.
__global__ __launch_bounds__(kRedThreads) void lz_reorth_norm(
    int64_t n, int N, int64_t chunk, const double* __restrict__ Q, int nt,
    const double* __restrict__ coef, double* __restrict__ W, double* beta, double* work,
    unsigned* counter) {
  __shared__ double sh[kRedThreads];
  const int c = threadIdx.x & 63;
  const int r0 = threadIdx.x >> 6;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  double acc = 0.0;
  if (c < N)
    for (int64_t i = beg + r0; i < end; i += 4) {
      const int64_t o = i * N + c;
      double w = W[o];
      for (int t = 0; t < nt; ++t) w -= coef[t * 64 + c] * Q[(int64_t)t * n * N + o];
      W[o] = w;
      acc += w * w;
    }
  (void)block_colsum_finish(acc, N, work, counter, sh,
                            [&](int col, double tot) { beta[col] = sqrt(tot); });
}

// Q_{j+1} = live ? W/β : 0; QW = isq·Q_{j+1} in the MatVec precision;
// β_prev = live ? β : 0 for the next three-term step.
template <typename T>
__global__ void lz_next(int64_t count, int N, const double* __restrict__ W,
                        const double* __restrict__ beta, const int* __restrict__ live,
                        double* __restrict__ Qn, T* __restrict__ QW, double* beta_prev,
                        double isq) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % N);
    const double q = live[c] ? W[e] / beta[c] : 0.0;
    Qn[e] = q;
    QW[e] = (T)(isq * q);
    if (e < N) beta_prev[e] = live[e] ? beta[e] : 0.0;
  }
}

// Q_0 = z/‖z‖, QW = isq·Q_0.
template <typename T>
__global__ void lz_first(int64_t count, int N, const T* __restrict__ Z,
                         const double* __restrict__ zn2, double* __restrict__ Q0,
                         T* __restrict__ QW, double isq) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % N);
    const double q = zn2[c] > 0.0 ? (double)Z[e] / sqrt(zn2[c]) : 0.0;
    Q0[e] = q;
    QW[e] = (T)(isq * q);
  }
}

unsigned eblocks(int64_t count) {
  const int64_t b = (count + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

template <typename T>
int slq_impl(const Problem& p, int N, int m, const void* Zv, int reorth, int precond,
             double* logdet, double* per_probe, hipStream_t st) {
  const int64_t n = p.n;
  const size_t nN = (size_t)n * N;
  const RedGrid g = red_grid(n);
  const int64_t cchunk = ((n + kCoefBlocks - 1) / kCoefBlocks + 3) / 4 * 4;
  const int cblocks = (int)((n + cchunk - 1) / cchunk);
  const double isq = precond ? 1.0 / std::sqrt(p.f * p.f + p.s) : 1.0;
  const double logm = precond ? (double)n * std::log(p.f * p.f + p.s) : 0.0;
  const int wp = p.prec == HIGP_FP64 ? 0 : 1;

  size_t bytes = 0;
  auto take = [&](size_t b) {
    size_t off = bytes;
    bytes += (b + 255) / 256 * 256;
    return off;
  };
  const size_t o_q = take((size_t)(m + 1) * nN * 8), o_w = take(nN * 8),
               o_qw = take(nN * sizeof(T)), o_ww = take(nN * sizeof(T)),
               o_sc = take(4 * 64 * 8), o_coef = take((size_t)(m + 1) * 64 * 8),
               o_part = take(reorth ? (size_t)(m + 1) * cblocks * 64 * 8 : 8),
               o_work = take((size_t)g.blocks * 64 * 8), o_live = take(64 * 4), o_cnt = take(8);
  void* mem = nullptr;
  HIGP_TRY(scratch_alloc(&mem, bytes, st));
  char* base = static_cast<char*>(mem);
  double* Q = (double*)(base + o_q);
  double* W = (double*)(base + o_w);
  T* QW = (T*)(base + o_qw);
  T* WW = (T*)(base + o_ww);
  double* sc = (double*)(base + o_sc);
  double* zn2 = sc;
  double* alpha = sc + 64;
  double* beta = sc + 128;
  double* beta_prev = sc + 192;
  double* coef = (double*)(base + o_coef);
  double* part = (double*)(base + o_part);
  double* work = (double*)(base + o_work);
  int* live_d = (int*)(base + o_live);
  unsigned* counter = (unsigned*)(base + o_cnt);

  auto fail = [&](int code) {
    (void)hipStreamSynchronize(st);
    scratch_free(mem, st);
    return code;
  };
  auto chk = [&]() -> int {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
      return set_error(HIGP_ERR_HIP, "launch failed: %s", hipGetErrorString(e));
    return HIGP_OK;
  };
  int rc;
  std::vector<int> live(N, 1);
  if (hipMemsetAsync(counter, 0, 8, st) != hipSuccess ||
      hipMemsetAsync(beta_prev, 0, 64 * 8, st) != hipSuccess ||
      hipMemcpyAsync(live_d, live.data(), N * sizeof(int), hipMemcpyHostToDevice, st) !=
          hipSuccess)
    return fail(set_error(HIGP_ERR_HIP, "initialisation failed"));

  rc = launch_coldot(n, N, Zv, wp, Zv, wp, zn2, work, counter, st);
  if (rc) return fail(rc);
  hipLaunchKernelGGL((lz_first<T>), dim3(eblocks(nN)), dim3(256), 0, st, (int64_t)nN, N,
                     (const T*)Zv, zn2, Q, QW, isq);
  if ((rc = chk())) return fail(rc);

  std::vector<std::vector<double>> al(N), be(N);
  std::vector<double> amax(N, 0.0), ah(N), bh(N), zn2h(N);
  if (hipMemcpyAsync(zn2h.data(), zn2, N * 8, hipMemcpyDeviceToHost, st) != hipSuccess)
    return fail(set_error(HIGP_ERR_HIP, "copy failed"));

  for (int j = 0; j < m; ++j) {
    double* Qj = Q + (size_t)j * nN;
    MatvecOut mo;
    mo.kv = WW;
    rc = launch_kmatvec(p, N, QW, mo, st);
    if (rc) return fail(rc);
    hipLaunchKernelGGL((lz_alpha<T>), dim3(g.blocks), dim3(kRedThreads), 0, st, n, N, g.chunk,
                       (const T*)WW, isq, (const double*)Qj, W, alpha, work, counter);
    hipLaunchKernelGGL(lz_three_term, dim3(eblocks(nN)), dim3(256), 0, st, (int64_t)nN, N, W,
                       (const double*)Qj, j > 0 ? (const double*)(Qj - nN) : nullptr,
                       (const double*)alpha, (const double*)beta_prev);
    if ((rc = chk())) return fail(rc);
    if (reorth) {
      hipLaunchKernelGGL(lz_coef, dim3(cblocks, j + 1), dim3(kRedThreads), 0, st, n, N, cchunk,
                         (const double*)Q, (const double*)W, part);
      hipLaunchKernelGGL(lz_coef_final, dim3(j + 1), dim3(64), 0, st, cblocks,
                         (const double*)part, coef);
    }
    hipLaunchKernelGGL(lz_reorth_norm, dim3(g.blocks), dim3(kRedThreads), 0, st, n, N, g.chunk,
                       (const double*)Q, reorth ? j + 1 : 0, (const double*)coef, W, beta, work,
                       counter);
    if ((rc = chk())) return fail(rc);
    if (hipMemcpyAsync(ah.data(), alpha, N * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipMemcpyAsync(bh.data(), beta, N * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(set_error(HIGP_ERR_HIP, "synchronisation failed"));
    bool any = false;
    for (int c = 0; c < N; ++c) {
      if (!live[c]) continue;
      amax[c] = std::max(amax[c], std::fabs(ah[c]));
      al[c].push_back(ah[c]);
    }
    if (j == m - 1) break;
    for (int c = 0; c < N; ++c) {
      if (!live[c]) continue;
      if (bh[c] <= 1e-12 * amax[c]) {
        live[c] = 0;
      } else {
        be[c].push_back(bh[c]);
        any = true;
      }
    }
    if (!any) break;
    if (hipMemcpyAsync(live_d, live.data(), N * sizeof(int), hipMemcpyHostToDevice, st) !=
        hipSuccess)
      return fail(set_error(HIGP_ERR_HIP, "copy failed"));
    hipLaunchKernelGGL((lz_next<T>), dim3(eblocks(nN)), dim3(256), 0, st, (int64_t)nN, N,
                       (const double*)W, (const double*)beta, (const int*)live_d,
                       Q + (size_t)(j + 1) * nN, QW, beta_prev, isq);
    if ((rc = chk())) return fail(rc);
  }
  if (hipStreamSynchronize(st) != hipSuccess)
    return fail(set_error(HIGP_ERR_HIP, "synchronisation failed"));
  scratch_free(mem, st);

  double total = 0.0;
  std::vector<double> th, tau;
  for (int c = 0; c < N; ++c) {
    const int mc = (int)al[c].size();
    th.assign(mc, 0.0);
    tau.assign(mc, 0.0);
    rc = higp_tridiag_eig(mc, al[c].data(), be[c].data(), th.data(), tau.data());
    if (rc) return rc;
    double q = 0.0;
    for (int i = 0; i < mc; ++i) q += tau[i] * tau[i] * std::log(th[i]);
    const double v = logm + zn2h[c] * q;
    if (per_probe) per_probe[c] = v;
    total += v;
  }
  *logdet = total / N;
  if (hipStreamSynchronize(st) != hipSuccess)
    return set_error(HIGP_ERR_HIP, "synchronisation failed");
  return HIGP_OK;
}

}  // namespace

int run_slq(const Problem& p, int N, int m, const void* Z, int reorth, int precond,
            double* logdet, double* per_probe, hipStream_t st) {
  if (p.prec == HIGP_FP64) return slq_impl<double>(p, N, m, Z, reorth, precond, logdet, per_probe, st);
  return slq_impl<float>(p, N, m, Z, reorth, precond, logdet, per_probe, st);
}

}  // namespace higp

// ---------------------------------------------------------------------------
// Host FP64 eigen-solve of a symmetric tridiagonal matrix: implicit symmetric
// QR steps with the Wilkinson shift and Givens bulge chasing (Golub & Van
// Loan, "Matrix Computations", symmetric tridiagonal QR algorithm).  Only the
// first row of the eigenvector matrix is accumulated, which is all the
// quadrature needs.
extern "C" int higp_tridiag_eig(int32_t m, const double* a, const double* b, double* theta,
                                double* tau) {
  if (m < 1 || !a || !theta || !tau || (m > 1 && !b))
    return higp::set_error(HIGP_ERR_INVALID_ARG, "higp_tridiag_eig: bad arguments (m=%d)", m);
  std::vector<double> d(a, a + m), e(m, 0.0), z(m, 0.0);
  for (int i = 0; i + 1 < m; ++i) e[i] = b[i];
  z[0] = 1.0;
  const double eps = 2.220446049250313e-16;
  int guard = 0;
  for (int hi = m - 1; hi > 0;) {
    if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
      e[hi - 1] = 0.0;
      --hi;
      continue;
    }
    if (++guard > 60 * m)
      return higp::set_error(HIGP_ERR_UNSUPPORTED, "higp_tridiag_eig: no convergence");
    int lo = hi - 1;
    while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) --lo;
    // Wilkinson shift: the eigenvalue of the trailing 2×2 block closer to d[hi].
    const double dd = 0.5 * (d[hi - 1] - d[hi]);
    const double bb = e[hi - 1];
    const double sg = dd >= 0.0 ? 1.0 : -1.0;
    const double mu = d[hi] - bb * bb / (dd + sg * std::hypot(dd, bb));
    double x = d[lo] - mu, y = e[lo];
    for (int k = lo; k < hi; ++k) {
      // Givens rotation G = [[c, s], [−s, c]] with (GᵀT G) zeroing y against x.
      const double r = std::hypot(x, y);
      double c = 1.0, s = 0.0;
      if (r > 0.0) {
        c = x / r;
        s = -y / r;
      }
      if (k > lo) e[k - 1] = r;
      const double ak = d[k], bk = e[k], ck = d[k + 1];
      d[k] = c * c * ak - 2.0 * c * s * bk + s * s * ck;
      d[k + 1] = s * s * ak + 2.0 * c * s * bk + c * c * ck;
      e[k] = c * s * (ak - ck) + (c * c - s * s) * bk;
      if (k + 1 < hi) {
        y = -s * e[k + 1];
        e[k + 1] = c * e[k + 1];
        x = e[k];
      }
      const double z0 = z[k], z1 = z[k + 1];
      z[k] = c * z0 - s * z1;
      z[k + 1] = s * z0 + c * z1;
    }
  }
  for (int i = 0; i < m; ++i) {
    theta[i] = d[i];
    tau[i] = z[i];
  }
  return HIGP_OK;
}
