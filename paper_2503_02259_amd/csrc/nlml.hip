// Negative log marginal likelihood and its hand-coded gradient ("Gaussian
// Processes": L(Θ), ∂L/∂θ, eq. (1), eq. (2), SLQ and Hutchinson), composed of
// the library's own PCG, SLQ, derivative MatVec and column-dot kernels.
//
// log|K̂| comes either from SLQ (a Lanczos pass over the probes after the
// solve) or from the tridiagonals the PCG run on [y | Z] builds implicitly for
// the probe columns (CG–Lanczos correspondence, Saad 2003 §6.7.3; GPyTorch's
// mBCG): with the step lengths α_j and direction coefficients β_j,
//   T_00 = 1/α_0,  T_jj = 1/α_j + β_{j−1}/α_{j−1},  T_{j,j+1} = √β_j/α_j,
// the Lanczos matrix of M^{-1/2}K̂M^{-1/2} from z/‖z‖ for the constant Jacobi
// M (or M = I).  The trace term of eq. (2) uses Hutchinson's estimator here
// and Hutch++ in hutchpp.hip.
#include <cmath>
#include <vector>

#include "reduce.h"

namespace higp {

int run_nlml_hutchpp(const Problem& p, const void* y, int N, const void* Z,
                     const higp_nlml_opts& o, double* loss, double* grad, double* logdet,
                     int32_t* iters, hipStream_t st);

// Probe quadrature ‖z‖²·e₁ᵀlog(T)e₁ with T from m PCG steps (α, β host
// arrays of m and m − 1 entries).  A zero step length (an exactly zero
// residual) ends T there.
int cg_quadrature(int m, const double* alpha, const double* beta, double zn2, double* out) {
  int mm = 0;
  while (mm < m && alpha[mm] > 0.0) ++mm;
  if (mm < 1) return set_error(HIGP_ERR_INVALID_ARG, "a probe column has no CG step");
  std::vector<double> a(mm), b(mm > 1 ? mm - 1 : 1), th(mm), tau(mm);
  for (int j = 0; j < mm; ++j) {
    a[j] = 1.0 / alpha[j];
    if (j > 0) a[j] += beta[j - 1] / alpha[j - 1];
    if (j + 1 < mm) b[j] = std::sqrt(beta[j]) / alpha[j];
  }
  HIGP_TRY(higp_tridiag_eig(mm, a.data(), b.data(), th.data(), tau.data()));
  double q = 0.0;
  for (int j = 0; j < mm; ++j) q += tau[j] * tau[j] * std::log(th[j]);
  *out = zn2 * q;
  return HIGP_OK;
}

int run_slq(const Problem& p, int N, int m, const void* Z, int reorth, int precond,
            double* logdet, double* per_probe, hipStream_t st);

// Host copy of k column dots (FP64, deterministic).
int host_coldot(int64_t n, int k, const void* A, int ta, const void* B, int tb, double* out,
                hipStream_t st) {
  size_t bytes = dot_work_doubles(n, k) * 8 + 64 * 8 + 256;
  void* mem = nullptr;
  HIGP_TRY(scratch_alloc(&mem, bytes, st));
  double* d_out = static_cast<double*>(mem);
  unsigned* counter = reinterpret_cast<unsigned*>(d_out + 64);
  double* work = d_out + 96;
  int rc = HIGP_OK;
  if (hipMemsetAsync(counter, 0, 4, st) != hipSuccess)
    rc = set_error(HIGP_ERR_HIP, "hipMemsetAsync failed");
  if (rc == HIGP_OK) rc = launch_coldot(n, k, A, ta, B, tb, d_out, work, counter, st);
  if (rc == HIGP_OK &&
      (hipMemcpyAsync(out, d_out, k * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
       hipStreamSynchronize(st) != hipSuccess))
    rc = set_error(HIGP_ERR_HIP, "column dot copy failed");
  scratch_free(mem, st);
  return rc;
}

namespace {

// B[:, 0] = y, B[:, 1..N] = Z  (row-major n×(N+1)).
template <typename T>
__global__ void pack_rhs(int64_t n, int N, const T* __restrict__ y, const T* __restrict__ Z,
                         T* __restrict__ B) {
  const int k = N + 1;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * k;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / k;
    const int c = (int)(e % k);
    B[e] = c == 0 ? y[i] : Z[i * N + c - 1];
  }
}

// A[:, 0] = α (from the FP64 iterate, rounded to T), A[:, 1..N] = Z.
template <typename T>
__global__ void pack_grad_input(int64_t n, int N, const double* __restrict__ W,
                                const T* __restrict__ Z, T* __restrict__ A) {
  const int k = N + 1;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n * k;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / k;
    const int c = (int)(e % k);
    A[e] = c == 0 ? (T)W[e] : Z[i * N + c - 1];
  }
}

unsigned blocks_for(int64_t count) {
  const int64_t b = (count + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

template <typename T>
int nlml_impl(const Problem& p, const void* y, int N, const void* Z, const higp_nlml_opts& o,
              double* loss, double* grad, double* logdet_out, int32_t* iters_out,
              hipStream_t st) {
  const int64_t n = p.n;
  const int k = N + 1;
  const size_t nk = (size_t)n * k;
  const int tt = p.prec == HIGP_FP64 ? 0 : 1;  // element type code of T
  size_t bytes = 0;
  auto take = [&](size_t b) {
    size_t off = bytes;
    bytes += (b + 255) / 256 * 256;
    return off;
  };
  const bool from_cg = o.logdet_mode == 1;
  const size_t hist = from_cg ? (size_t)o.max_iter * k * 8 : 0;
  const size_t o_b = take(nk * sizeof(T)), o_x = take(nk * sizeof(T)), o_w = take(nk * 8),
               o_a = take(nk * sizeof(T)), o_dl = take(nk * sizeof(T)),
               o_df = take(nk * sizeof(T)), o_ah = take(hist), o_bh = take(hist);
  void* mem = nullptr;
  HIGP_TRY(scratch_alloc(&mem, bytes, st));
  char* base = static_cast<char*>(mem);
  T* B = (T*)(base + o_b);
  T* Xs = (T*)(base + o_x);
  double* W = (double*)(base + o_w);
  T* A = (T*)(base + o_a);
  T* DL = (T*)(base + o_dl);
  T* DF = (T*)(base + o_df);
  double* ahist = from_cg ? (double*)(base + o_ah) : nullptr;
  double* bhist = from_cg ? (double*)(base + o_bh) : nullptr;
  auto done = [&](int rc) {
    (void)hipStreamSynchronize(st);
    scratch_free(mem, st);
    return rc;
  };

  // 1. K̂⁻¹[y | Z] by PCG (FP64 iterate kept).
  hipLaunchKernelGGL((pack_rhs<T>), dim3(blocks_for(nk)), dim3(256), 0, st, n, N,
                     (const T*)y, (const T*)Z, B);
  higp_pcg_opts po{};
  po.tol = o.tol;
  po.max_iter = o.max_iter;
  po.precond = o.precond;
  po.refine_every = o.refine_every;
  po.use_x0 = 0;
  po.check_every = 0;
  po.refine_prec = HIGP_FP64;
  po.x_fp64 = W;
  std::vector<int32_t> its(k);
  std::vector<double> rel(k);
  std::vector<int32_t> conv(k);
  higp_pcg_info info{its.data(), rel.data(), conv.data()};
  int rc = run_pcg(p, k, B, Xs, po, &info, st, ahist, bhist);
  if (rc) return done(rc);
  int itmax = 0;
  for (int c = 0; c < k; ++c) itmax = its[c] > itmax ? its[c] : itmax;

  // 2. log|K̂| by eq. (1): SLQ over Z, or the PCG tridiagonals of the Z
  //    columns (quadratures formed below, once ‖z‖² is known).
  double logdet = 0.0;
  std::vector<double> ah, bh;
  if (from_cg) {
    ah.assign((size_t)itmax * k, 0.0);
    bh.assign((size_t)itmax * k, 0.0);
    if (itmax > 0 &&
        (hipMemcpyAsync(ah.data(), ahist, ah.size() * 8, hipMemcpyDeviceToHost, st) !=
             hipSuccess ||
         hipMemcpyAsync(bh.data(), bhist, bh.size() * 8, hipMemcpyDeviceToHost, st) !=
             hipSuccess))
      return done(set_error(HIGP_ERR_HIP, "coefficient copy failed"));
  } else {
    rc = run_slq(p, N, o.nsteps, Z, o.reorth, o.precond, &logdet, nullptr, st);
    if (rc) return done(rc);
  }

  // 3. ∂K̂/∂θ·[α | Z] by one fused derivative MatVec.
  hipLaunchKernelGGL((pack_grad_input<T>), dim3(blocks_for(nk)), dim3(256), 0, st, n, N,
                     (const double*)W, (const T*)Z, A);
  MatvecOut mo;
  mo.dl = DL;
  mo.df = DF;
  rc = launch_kmatvec(p, k, A, mo, st);
  if (rc) return done(rc);

  // 4. Inner products (FP64): [αᵀ∂K̂α, W_iᵀ∂K̂z_i] for l and f; [αᵀα, W_iᵀz_i]
  //    for s (∂K̂/∂s = I); yᵀα and ‖z_i‖² from [y | Z].
  std::vector<double> dl(k), df(k), ds(k), by(k), bb(k);
  if ((rc = host_coldot(n, k, W, 0, DL, tt, dl.data(), st)) ||
      (rc = host_coldot(n, k, W, 0, DF, tt, df.data(), st)) ||
      (rc = host_coldot(n, k, W, 0, A, tt, ds.data(), st)) ||
      (rc = host_coldot(n, k, W, 0, B, tt, by.data(), st)) ||
      (rc = host_coldot(n, k, B, tt, B, tt, bb.data(), st)))
    return done(rc);
  done(HIGP_OK);
  if (from_cg) {
    const double logm = o.precond ? (double)n * std::log(p.f * p.f + p.s) : 0.0;
    std::vector<double> a(itmax), b(itmax);
    for (int c = 1; c < k; ++c) {
      const int m = its[c];
      for (int j = 0; j < m; ++j) {
        a[j] = ah[(size_t)j * k + c];
        b[j] = bh[(size_t)j * k + c];
      }
      double q = 0.0;
      rc = cg_quadrature(m, a.data(), b.data(), bb[c], &q);
      if (rc) return rc;
      logdet += logm + q;
    }
    logdet /= N;
  }

  // Eq. (2) with M = diag(K̂) = (f²+s)·I: tr(M⁻¹∂M) − (1/N) Σ z_iᵀM⁻¹∂M z_i;
  // ∂M/∂l = 0, ∂M/∂f = 2f·I, ∂M/∂s = I.  Without preconditioning M = I.
  const double m = p.f * p.f + p.s;
  double zz = 0.0;
  for (int c = 1; c < k; ++c) zz += bb[c];
  zz /= N;
  const double cv_f = o.precond ? 2.0 * p.f / m * ((double)n - zz) : 0.0;
  const double cv_s = o.precond ? 1.0 / m * ((double)n - zz) : 0.0;
  double h[3] = {0.0, 0.0, 0.0};
  for (int c = 1; c < k; ++c) {
    h[0] += dl[c];
    h[1] += df[c];
    h[2] += ds[c];
  }
  for (int t = 0; t < 3; ++t) h[t] /= N;
  grad[0] = 0.5 * (-dl[0] + h[0]);
  grad[1] = 0.5 * (-df[0] + h[1] + cv_f);
  grad[2] = 0.5 * (-ds[0] + h[2] + cv_s);
  *loss = 0.5 * (by[0] + logdet + (double)n * std::log(2.0 * M_PI));
  if (logdet_out) *logdet_out = logdet;
  if (iters_out) *iters_out = itmax;
  return HIGP_OK;
}

}  // namespace

int run_nlml(const Problem& p, const void* y, int N, const void* Z, const higp_nlml_opts& o,
             double* loss, double* grad, double* logdet, int32_t* iters, hipStream_t st) {
  if (o.trace_mode == 1) return run_nlml_hutchpp(p, y, N, Z, o, loss, grad, logdet, iters, st);
  if (p.prec == HIGP_FP64) return nlml_impl<double>(p, y, N, Z, o, loss, grad, logdet, iters, st);
  return nlml_impl<float>(p, y, N, Z, o, loss, grad, logdet, iters, st);
}

}  // namespace higp
