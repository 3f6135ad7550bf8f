// Stochastic Lanczos quadrature for log|K̂| (eq. (1) of the paper with the
// SLQ estimator of Ubaru et al. 2017, "Gaussian Processes" section).
//
// log|K̂| = log|M| + log|M^{-1/2} K̂ M^{-1/2}|.  With M = diag(K̂) = (f²+s)·I
// (stationary kernels) the operator is K̂/(f²+s) and log|M| = n·log(f²+s);
// without preconditioning M = I.  Every probe runs the Lanczos process of
// lanczos_kernels.h from z/‖z‖ (all probes share one MatVec per step); the
// quadrature is ‖z‖²·Σ_k τ_k²·log θ_k with θ, τ the eigenvalues and first
// eigenvector components of the tridiagonal T, computed in FP64 on the host.
// Lanczos vectors are kept in FP64 on the device ((nsteps+1)·n·nprobe·8 B).
#include <cmath>
#include <vector>

#include "lanczos_kernels.h"

namespace higp {
namespace {

template <typename T>
int slq_impl(const Problem& p, int N, int m, const void* Zv, int reorth, int precond,
             double* logdet, double* per_probe, hipStream_t st) {
  const int64_t n = p.n;
  const size_t nN = (size_t)n * N;
  const double isq = precond ? 1.0 / std::sqrt(p.f * p.f + p.s) : 1.0;
  const double logm = precond ? (double)n * std::log(p.f * p.f + p.s) : 0.0;
  const int wp = p.prec == HIGP_FP64 ? 0 : 1;

  const size_t sbytes = lz_state_bytes(n, N, m);
  const size_t qw_bytes = (nN * sizeof(T) + 255) / 256 * 256;
  void* mem = nullptr;
  HIGP_TRY(scratch_alloc(&mem, sbytes + 2 * qw_bytes + 64 * 8, st));
  char* base = static_cast<char*>(mem);
  LzState S = lz_carve(base, n, N, m);
  T* QW = (T*)(base + sbytes);
  T* WW = (T*)(base + sbytes + qw_bytes);
  double* zn2 = (double*)(base + sbytes + 2 * qw_bytes);
  auto fail = [&](int code) {
    (void)hipStreamSynchronize(st);
    scratch_free(mem, st);
    return code;
  };
  int rc;
  if (hipMemsetAsync(S.counter, 0, 8, st) != hipSuccess)
    return fail(set_error(HIGP_ERR_HIP, "initialisation failed"));
  rc = launch_coldot(n, N, Zv, wp, Zv, wp, zn2, S.work, S.counter, st);
  if (rc) return fail(rc);
  hipLaunchKernelGGL((lz_first<T>), dim3(lz_blocks(nN)), dim3(256), 0, st, (int64_t)nN, N,
                     (const T*)Zv, (const double*)zn2, QW, isq, S);

  // Poll the number of live probes every few steps so that a run whose
  // probes all broke down early stops early.
  int nlive_h = N;
  for (int j = 0; j < m; ++j) {
    MatvecOut mo;
    mo.kv = WW;
    rc = launch_kmatvec(p, N, QW, mo, st);
    if (rc) break;
    lz_launch_step<T>(n, N, j, m, reorth != 0, isq, WW, QW, S, st);
    if (hipGetLastError() != hipSuccess) {
      rc = set_error(HIGP_ERR_HIP, "Lanczos launch failed");
      break;
    }
    if ((j % 8) == 7 && j + 1 < m) {
      if (hipMemcpyAsync(&nlive_h, S.nlive, sizeof(int), hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) {
        rc = set_error(HIGP_ERR_HIP, "synchronisation failed");
        break;
      }
      if (nlive_h == 0) break;
    }
  }
  std::vector<double> ah((size_t)m * N), bh((size_t)m * N), zn2h(N);
  std::vector<int> steps(N);
  if (rc == HIGP_OK &&
      (hipMemcpyAsync(ah.data(), S.ahist, (size_t)m * N * 8, hipMemcpyDeviceToHost, st) !=
           hipSuccess ||
       hipMemcpyAsync(bh.data(), S.bhist, (size_t)m * N * 8, hipMemcpyDeviceToHost, st) !=
           hipSuccess ||
       hipMemcpyAsync(steps.data(), S.steps, N * sizeof(int), hipMemcpyDeviceToHost, st) !=
           hipSuccess ||
       hipMemcpyAsync(zn2h.data(), zn2, N * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
       hipStreamSynchronize(st) != hipSuccess))
    rc = set_error(HIGP_ERR_HIP, "result copy failed");
  if (rc) return fail(rc);
  scratch_free(mem, st);

  double total = 0.0;
  std::vector<double> a, b, th, tau;
  for (int c = 0; c < N; ++c) {
    const int mc = steps[c];
    if (mc < 1) return set_error(HIGP_ERR_INVALID_ARG, "probe %d is zero", c);
    a.resize(mc);
    b.resize(mc > 1 ? mc - 1 : 1);
    for (int i = 0; i < mc; ++i) a[i] = ah[(size_t)i * N + c];
    for (int i = 0; i + 1 < mc; ++i) b[i] = bh[(size_t)i * N + c];
    th.assign(mc, 0.0);
    tau.assign(mc, 0.0);
    rc = higp_tridiag_eig(mc, a.data(), b.data(), th.data(), tau.data());
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
