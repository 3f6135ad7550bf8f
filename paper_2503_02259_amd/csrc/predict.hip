// GP regression prediction (the `gpr_prediction` call of Listing 1): the
// predictive mean and latent variance of the textbook GP posterior, composed
// of the library's PCG, rectangular on-the-fly MatVec and column dots.  The
// rectangular MatVec evaluates K(X*, X) block by block exactly like the square
// one ("Statement of Need", on-the-fly evaluation).
//
//   mean_q = f²·k(x_q, X)·α,       α = K̂⁻¹y
//   var_q  = f² − k*_qᵀ K̂⁻¹ k*_q,  k*_q = f²·k(X, x_q)
//
// The variance solves run 64 query points at a time: K* = f²·k(X, X*_b) is
// formed as the rectangular MatVec of the identity (n×64), PCG solves
// K̂W = K*, and the column dots of K* and W give the 64 quadratic forms.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"

namespace higp {

int host_coldot(int64_t n, int k, const void* A, int ta, const void* B, int tb, double* out,
                hipStream_t st);
int launch_kmatvec_cross(const Problem& p, int64_t m, const void* Xq, int k, const void* V,
                         void* Y, hipStream_t st);

namespace {

constexpr int kVarBlock = 64;

template <typename T>
__global__ void eye_kernel(int B, T* __restrict__ E) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < B * B; e += gridDim.x * blockDim.x)
    E[e] = (e / B == e % B) ? (T)1 : (T)0;
}

template <typename T>
int predict_impl(const Problem& p, const void* y, int64_t m, const void* Xq,
                 const higp_predict_opts& o, void* mean, void* var, int32_t* pcg_iters,
                 hipStream_t st) {
  const int64_t n = p.n;
  const int tcode = sizeof(T) == 8 ? 0 : 1;
  auto rup = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t a_bytes = rup((size_t)n * sizeof(T));
  const size_t e_bytes = o.want_var ? rup((size_t)kVarBlock * kVarBlock * sizeof(T)) : 0;
  const size_t k_bytes = o.want_var ? rup((size_t)n * kVarBlock * sizeof(T)) : 0;
  void* mem = nullptr;
  HIGP_TRY(scratch_alloc(&mem, a_bytes + e_bytes + 2 * k_bytes, st));
  char* base = static_cast<char*>(mem);
  T* alpha = reinterpret_cast<T*>(base);
  T* E = reinterpret_cast<T*>(base + a_bytes);
  T* Kxq = reinterpret_cast<T*>(base + a_bytes + e_bytes);
  T* W = reinterpret_cast<T*>(base + a_bytes + e_bytes + k_bytes);
  auto fail = [&](int rc) {
    scratch_free(mem, st);
    return rc;
  };

  higp_pcg_opts po{};
  po.tol = o.tol;
  po.max_iter = o.max_iter;
  po.precond = o.precond;
  po.rank = o.rank;
  po.refine_prec = HIGP_FP64;
  std::vector<int32_t> it(kVarBlock);
  std::vector<double> rel(kVarBlock);
  std::vector<int32_t> conv(kVarBlock);
  higp_pcg_info info{it.data(), rel.data(), conv.data()};

  // α = K̂⁻¹y, then the mean.
  int rc = run_pcg(p, 1, y, alpha, po, &info, st);
  if (rc) return fail(rc);
  if (pcg_iters) *pcg_iters = it[0];
  rc = launch_kmatvec_cross(p, m, Xq, 1, alpha, mean, st);
  if (rc) return fail(rc);

  if (o.want_var) {
    const double f2 = p.f * p.f;
    std::vector<double> dots(kVarBlock);
    std::vector<T> vh(kVarBlock);
    for (int64_t q0 = 0; q0 < m; q0 += kVarBlock) {
      const int B = (int)std::min<int64_t>(kVarBlock, m - q0);
      hipLaunchKernelGGL((eye_kernel<T>), dim3((B * B + 255) / 256), dim3(256), 0, st, B, E);
      if (hipGetLastError() != hipSuccess)
        return fail(set_error(HIGP_ERR_HIP, "identity launch failed"));
      // K* = f²·k(X, X*_b)·I: the query block takes the role of the J points.
      Problem pb = p;
      pb.X = static_cast<const char*>(Xq) + (size_t)q0 * p.d * sizeof(T);
      pb.n = B;
      rc = launch_kmatvec_cross(pb, n, p.X, B, E, Kxq, st);
      if (rc) return fail(rc);
      rc = run_pcg(p, B, Kxq, W, po, &info, st);
      if (rc) return fail(rc);
      rc = host_coldot(n, B, Kxq, tcode, W, tcode, dots.data(), st);
      if (rc) return fail(rc);
      // The exact value is ≥ 0; a solve stopped at its tolerance can leave a
      // tiny negative remainder, which is reported as 0.
      for (int c = 0; c < B; ++c) vh[c] = (T)std::max(0.0, f2 - dots[c]);
      if (hipMemcpyAsync(static_cast<T*>(var) + q0, vh.data(), B * sizeof(T),
                         hipMemcpyHostToDevice, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return fail(set_error(HIGP_ERR_HIP, "variance copy failed"));
    }
  }
  if (hipStreamSynchronize(st) != hipSuccess)
    return fail(set_error(HIGP_ERR_HIP, "synchronisation failed"));
  scratch_free(mem, st);
  return HIGP_OK;
}

}  // namespace

int run_predict(const Problem& p, const void* y, int64_t m, const void* Xq,
                const higp_predict_opts& o, void* mean, void* var, int32_t* pcg_iters,
                hipStream_t st) {
  if (p.prec == HIGP_FP64) return predict_impl<double>(p, y, m, Xq, o, mean, var, pcg_iters, st);
  return predict_impl<float>(p, y, m, Xq, o, mean, var, pcg_iters, st);
}

}  // namespace higp
