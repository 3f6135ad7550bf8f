// Negative log marginal likelihood and its hand-coded gradient ("Gaussian
// Processes": L(Θ), ∂L/∂θ, eq. (1), eq. (2), SLQ and Hutchinson), composed of
// the library's own PCG, SLQ, derivative MatVec and column-dot kernels.
#include <cmath>
#include <vector>

#include "reduce.h"

namespace higp {

int run_pcg(const Problem& p, int k, const void* B, void* X, const higp_pcg_opts& o,
            higp_pcg_info* info, hipStream_t st);
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
  const size_t o_b = take(nk * sizeof(T)), o_x = take(nk * sizeof(T)), o_w = take(nk * 8),
               o_a = take(nk * sizeof(T)), o_dl = take(nk * sizeof(T)),
               o_df = take(nk * sizeof(T));
  void* mem = nullptr;
  HIGP_TRY(scratch_alloc(&mem, bytes, st));
  char* base = static_cast<char*>(mem);
  T* B = (T*)(base + o_b);
  T* Xs = (T*)(base + o_x);
  double* W = (double*)(base + o_w);
  T* A = (T*)(base + o_a);
  T* DL = (T*)(base + o_dl);
  T* DF = (T*)(base + o_df);
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
  int rc = run_pcg(p, k, B, Xs, po, &info, st);
  if (rc) return done(rc);
  int itmax = 0;
  for (int c = 0; c < k; ++c) itmax = its[c] > itmax ? its[c] : itmax;

  // 2. log|K̂| by eq. (1) and SLQ over Z.
  double logdet = 0.0;
  rc = run_slq(p, N, o.nsteps, Z, o.reorth, o.precond, &logdet, nullptr, st);
  if (rc) return done(rc);

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
  if (p.prec == HIGP_FP64) return nlml_impl<double>(p, y, N, Z, o, loss, grad, logdet, iters, st);
  return nlml_impl<float>(p, y, N, Z, o, loss, grad, logdet, iters, st);
}

}  // namespace higp
