// Preconditioned conjugate gradients for K̂·X = B with k right-hand sides.
//
// HiGP approximates K̂⁻¹y with PCG and a preconditioner M ≈ K̂ ("Gaussian
// Processes" section, citing Saad 2003).  Here the k columns are k
// independent CG recurrences that share one k-column MatVec per iteration.
// All CG scalars live on the device in FP64 and are updated by the kernels
// themselves (no host round trip per iteration); x and r are FP64 vectors;
// the search direction p is stored in the problem's precision because it is
// the MatVec input.  A column stops when its recursively updated residual
// satisfies ‖r‖₂ ≤ tol·‖b‖₂ (checked after every iteration) or when it has
// taken max_iter iterations; it is then frozen.  The host only polls the
// number of active columns every `check_every` iterations, which decides
// when the call returns but never changes a result.
//
// Jacobi preconditioning uses M = diag(K̂).  For the stationary kernels
// supported here diag(K̂) = f²·k(0) + s = f² + s for every row, so M⁻¹ is the
// scalar 1/(f² + s).
//
// Residual replacement (refine_every = R): after every R-th iteration the
// recursive residual is replaced by b − K̂x.  With refine_prec = FP64 the
// iterate x (kept in FP64) enters an FP64 MatVec over the points widened to
// double, so the replaced residual is the true residual to FP64 accuracy and
// the stopping test then holds for the true residual (mixed-precision
// iterative refinement: cheap MatVecs inside CG, an accurate residual every R
// iterations).  With refine_prec = FP32, x is rounded to float and the FP32
// MatVec is used; the residual is then only as accurate as the FP32 floor.
#include <vector>

#include "nystrom.h"
#include "pcg_kernels.h"

namespace higp {
namespace {

template <typename T>
int pcg_impl(const Problem& p, int k, const void* Bv, void* Xv, const higp_pcg_opts& o,
             higp_pcg_info* info, hipStream_t st, double* ahist, double* bhist) {
  const int64_t n = p.n;
  const size_t nk = (size_t)n * k;
  const RedGrid g = red_grid(n);
  const int wp = p.prec == HIGP_FP64 ? 0 : 1;  // MatVec element type
  const int refine_prec = (p.prec == HIGP_BF16 || p.prec == HIGP_BF16X3) ? HIGP_FP32 : p.prec;
  const T* B = static_cast<const T*>(Bv);
  T* Xout = static_cast<T*>(Xv);

  // Scratch layout.
  const size_t nwork = (size_t)g.blocks * 64;
  size_t bytes = 0;
  auto take = [&](size_t b) {
    size_t off = bytes;
    bytes += (b + 255) / 256 * 256;
    return off;
  };
  const bool refine = o.refine_every > 0;
  const bool refine64 = refine && (o.refine_prec == HIGP_FP64 || p.prec == HIGP_FP64);
  const bool widen = refine64 && p.prec != HIGP_FP64;  // FP64 copy of the points
  const bool nys = o.precond == 2;                      // Nyström preconditioner
  const size_t o_x = take(nk * 8), o_r = take(nk * 8), o_p = take(nk * sizeof(T)),
               o_q = take(nk * sizeof(T)),
               o_q2 = take(refine ? nk * (refine64 ? 8 : sizeof(T)) : 0),
               o_xd = take(widen ? (size_t)n * p.d * 8 : 0),
               o_z = take(nys ? nk * 8 : 0), o_sc = take(10 * 64 * 8),
               o_int = take(4 * 64 * 4),
               o_work = take(nwork * 8 * 2), o_cnt = take(2 * 4);
  void* mem = nullptr;
  HIGP_TRY(scratch_alloc(&mem, bytes, st));
  char* base = static_cast<char*>(mem);
  PcgState S{};
  S.x = (double*)(base + o_x);
  S.r = (double*)(base + o_r);
  T* P = (T*)(base + o_p);
  T* Q = (T*)(base + o_q);
  void* Q2 = base + o_q2;
  Problem p64 = p;  // the problem seen by an FP64 replacement MatVec
  if (refine64) {
    p64.prec = HIGP_FP64;
    if (widen) p64.X = base + o_xd;
  }
  double* sc = (double*)(base + o_sc);
  S.rho = sc;
  S.pq = sc + 64;
  S.beta = sc + 128;
  S.bnorm = sc + 192;
  S.relres = sc + 256;
  S.lastrep = sc + 448;
  double* bb = sc + 320;
  double* rr0 = sc + 384;
  double* pr = sc + 512;  // pᵀr on the iteration after a replacement
  int* in = (int*)(base + o_int);
  S.active = in;
  S.iters = in + 64;
  S.nactive = in + 128;
  S.norepl = in + 192;
  S.work = (double*)(base + o_work);
  double* work2 = S.work + nwork;
  S.counter = (unsigned*)(base + o_cnt);
  unsigned* counter2 = S.counter + 1;
  S.ahist = ahist;
  S.bhist = bhist;

  PcgScalars ps;
  ps.tol = o.tol;
  ps.max_iter = o.max_iter;
  ps.k = k;
  ps.minv = o.precond == 1 ? 1.0 / (p.f * p.f + p.s) : 1.0;
  ps.general_m = nys ? 1 : 0;
  // Stopping only on a replaced residual is sound when the replacement is
  // accurate (FP64).  An FP32 replacement has a floor u₃₂·‖|K̂||x|‖/‖b‖ that
  // is usually above the tolerance; a column held open by it keeps taking
  // replacements whose noise grows with |x|, so there the recursive residual
  // decides as without refinement.
  ps.replaced_only = refine64 ? 1 : 0;
  ps.stall_off = refine && !refine64 ? 1 : 0;

  int rc = HIGP_OK;
  NysPrec NP;
  auto fail = [&](int code) {
    nys_free(NP, st);
    scratch_free(mem, st);
    return code;
  };
  double* Z = nys ? (double*)(base + o_z) : nullptr;
  double* rz = (double*)(base + o_sc) + 576;
  if (nys) {
    rc = nys_build(p, o.rank > 0 ? o.rank : (int)std::min<int64_t>(n, 1024), k, &NP, st);
    if (rc) return fail(rc);
  }
  if (hipMemsetAsync(S.counter, 0, 8, st) != hipSuccess)
    return fail(set_error(HIGP_ERR_HIP, "hipMemsetAsync failed"));
  if (widen) {
    rc = launch_cast_scale(n * p.d, p.X, 1, base + o_xd, 0, 1.0, st);
    if (rc) return fail(rc);
  }

  // r0 = b − K̂x0 needs a MatVec of x0 when a warm start is given.
  const T* q0 = nullptr;
  if (o.use_x0) {
    MatvecOut mo;
    mo.kv = Q;
    rc = launch_kmatvec(p, k, Xout, mo, st, refine_prec);
    if (rc) return fail(rc);
    q0 = Q;
  }
  hipLaunchKernelGGL((pcg_start_norms<T>), dim3(g.blocks), dim3(kRedThreads), 0, st, n, k,
                     g.chunk, B, o.use_x0 ? (const T*)Xout : (const T*)nullptr, q0, S, bb,
                     work2, counter2);
  if (hipGetLastError() != hipSuccess) return fail(set_error(HIGP_ERR_HIP, "launch failed"));
  rc = launch_coldot(n, k, S.r, 0, S.r, 0, rr0, S.work, S.counter, st);
  if (rc) return fail(rc);
  hipLaunchKernelGGL(pcg_start_finish, dim3(1), dim3(64), 0, st, k, S, ps, bb, rr0);
  if (nys) {
    // z₀ = M⁻¹r₀, ρ = r₀ᵀz₀, p = z₀.
    rc = nys_apply(NP, k, S.r, Z, st);
    if (rc == HIGP_OK) rc = launch_coldot(n, k, S.r, 0, Z, 0, rz, S.work, S.counter, st);
    if (rc) return fail(rc);
    hipLaunchKernelGGL(pcg_rho_beta, dim3(1), dim3(64), 0, st, k, S, (const double*)rz, 1);
    rc = launch_cast_scale((int64_t)nk, Z, 0, P, wp, 1.0, st);
    if (rc) return fail(rc);
  } else {
    hipLaunchKernelGGL((pcg_pinit<T>), dim3(elem_blocks(nk)), dim3(256), 0, st, n, k, P, S.r,
                       ps.minv);
  }
  if (hipGetLastError() != hipSuccess) return fail(set_error(HIGP_ERR_HIP, "launch failed"));

  int check = o.check_every > 0 ? o.check_every : (n >= 20000 ? 1 : 8);
  int nact = 0;
  if (hipMemcpyAsync(&nact, S.nactive, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(set_error(HIGP_ERR_HIP, "synchronisation failed"));

  bool after_replace = false;
  for (int it = 1; it <= o.max_iter && nact > 0; ++it) {
    MatvecOut mo;
    mo.kv = Q;
    rc = launch_kmatvec(p, k, P, mo, st);
    if (rc) return fail(rc);
    rc = launch_coldot(n, k, P, wp, Q, wp, S.pq, S.work, S.counter, st);
    if (rc) return fail(rc);
    if (after_replace) {
      rc = launch_coldot(n, k, P, wp, S.r, 0, pr, S.work, S.counter, st);
      if (rc) return fail(rc);
    }
    const bool replace = o.refine_every > 0 && it % o.refine_every == 0;
    hipLaunchKernelGGL((pcg_update<T>), dim3(g.blocks), dim3(kRedThreads), 0, st, n, k, g.chunk,
                       (const T*)P, (const T*)Q, S, ps, replace ? 0 : 1,
                       after_replace ? (const double*)pr : nullptr);
    if (hipGetLastError() != hipSuccess) return fail(set_error(HIGP_ERR_HIP, "launch failed"));
    if (replace) {
      MatvecOut m2;
      m2.kv = Q2;
      if (refine64) {
        // r = b − K̂x with x in FP64 and an FP64 MatVec.
        rc = launch_kmatvec(p64, k, S.x, m2, st);
        if (rc) return fail(rc);
        hipLaunchKernelGGL((pcg_replace<T, double>), dim3(g.blocks), dim3(kRedThreads), 0, st, n,
                           k, g.chunk, B, (const double*)Q2, S, ps);
      } else {
        // r = b − K̂x with x rounded to the MatVec precision and the FP32 MatVec.
        rc = launch_cast_scale((int64_t)nk, S.x, 0, Q, wp, 1.0, st);
        if (rc) return fail(rc);
        rc = launch_kmatvec(p, k, Q, m2, st, refine_prec);
        if (rc) return fail(rc);
        hipLaunchKernelGGL((pcg_replace<T, T>), dim3(g.blocks), dim3(kRedThreads), 0, st, n, k,
                           g.chunk, B, (const T*)Q2, S, ps);
      }
      if (hipGetLastError() != hipSuccess) return fail(set_error(HIGP_ERR_HIP, "launch failed"));
    }
    after_replace = replace;
    if (nys) {
      rc = nys_apply(NP, k, S.r, Z, st);
      if (rc == HIGP_OK) rc = launch_coldot(n, k, S.r, 0, Z, 0, rz, S.work, S.counter, st);
      if (rc) return fail(rc);
      hipLaunchKernelGGL(pcg_rho_beta, dim3(1), dim3(64), 0, st, k, S, (const double*)rz, 0);
      hipLaunchKernelGGL((pcg_pupdate_z<T>), dim3(elem_blocks(nk)), dim3(256), 0, st, n, k, P,
                         (const double*)Z, S);
    } else {
      hipLaunchKernelGGL((pcg_pupdate<T>), dim3(elem_blocks(nk)), dim3(256), 0, st, n, k, P, S,
                         ps.minv);
    }
    if (hipGetLastError() != hipSuccess) return fail(set_error(HIGP_ERR_HIP, "launch failed"));
    if (it % check == 0 || it == o.max_iter) {
      if (hipMemcpyAsync(&nact, S.nactive, sizeof(int), hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return fail(set_error(HIGP_ERR_HIP, "synchronisation failed"));
    }
  }

  // Results.
  rc = launch_cast_scale((int64_t)nk, S.x, 0, Xout, wp, 1.0, st);
  if (rc) return fail(rc);
  if (o.x_fp64 &&
      hipMemcpyAsync(o.x_fp64, S.x, nk * 8, hipMemcpyDeviceToDevice, st) != hipSuccess)
    return fail(set_error(HIGP_ERR_HIP, "copy of the FP64 iterate failed"));
  std::vector<int> it_h(k);
  std::vector<double> rel_h(k);
  if (hipMemcpyAsync(it_h.data(), S.iters, k * sizeof(int), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipMemcpyAsync(rel_h.data(), S.relres, k * sizeof(double), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(set_error(HIGP_ERR_HIP, "result copy failed"));
  nys_free(NP, st);
  scratch_free(mem, st);
  for (int c = 0; c < k; ++c) {
    if (info && info->iters) info->iters[c] = it_h[c];
    if (info && info->relres) info->relres[c] = rel_h[c];
    if (info && info->converged) info->converged[c] = rel_h[c] <= o.tol ? 1 : 0;
  }
  if (hipStreamSynchronize(st) != hipSuccess)
    return set_error(HIGP_ERR_HIP, "synchronisation failed");
  return HIGP_OK;
}

}  // namespace

int run_pcg(const Problem& p, int k, const void* B, void* X, const higp_pcg_opts& o,
            higp_pcg_info* info, hipStream_t st, double* ahist, double* bhist) {
  if (p.prec == HIGP_FP64) return pcg_impl<double>(p, k, B, X, o, info, st, ahist, bhist);
  return pcg_impl<float>(p, k, B, X, o, info, st, ahist, bhist);
}

}  // namespace higp
