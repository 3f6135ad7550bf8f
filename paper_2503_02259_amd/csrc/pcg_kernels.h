// PCG kernels shared by the single-call solver (higp_pcg) and the serving
// engine.  CG scalars are FP64 on the device; x and r are FP64 vectors; the
// search direction p is stored in the MatVec precision.  Column c stops when
// its recursive ‖r_c‖₂ ≤ tol·‖b_c‖₂ (checked after every iteration) or after
// max_iter iterations, and is frozen from then on.  With an FP64 residual
// replacement (`replaced_only`) the tolerance is tested only on a replaced
// residual b − K̂x, so that it holds for the recomputed residual and not for
// a recursive one that has drifted from it; the cap applies at every
// iteration.  An FP32 replacement is accurate only to the floor
// u₃₂·‖|K̂||x|‖/‖b‖; replacing at that level breaks the orthogonality CG relies
// on (β stays near 1, p accumulates) and the iteration runs away.  So with
// `stall_off` a column takes no further replacements once one fails to lower
// its residual below the previous replacement's, and continues as plain
// recursive CG (the idea of van der Vorst and Ye's residual replacement: stop
// replacing when it no longer helps).  Any column whose residual is not
// finite or exceeds 1e8·‖b‖ stops as diverged.
#pragma once

#include "reduce.h"

namespace higp {
namespace {

struct PcgState {
  double* x;       // n×k FP64
  double* r;       // n×k FP64
  double* rho;     // k
  double* pq;      // k
  double* beta;    // k
  double* bnorm;   // k
  double* relres;  // k
  double* lastrep;  // k: relres after the last replacement (stall_off only)
  int* norepl;      // k: 1 = no further replacements for this column
  int* active;     // k
  int* iters;      // k
  int* nactive;    // 1
  double* work;    // reduction partials
  unsigned* counter;
  volatile int* nactive_host;  // optional pinned host copy of *nactive
  double* ahist;   // optional max_iter×k: α_j of each column (row j)
  double* bhist;   // optional max_iter×k: β_j of each column (row j)
};

struct PcgScalars {
  double tol;
  double minv;
  int max_iter;
  int k;              // columns (row length of the coefficient histories)
  int replaced_only;  // 1: stop on tol only after a residual replacement
  int stall_off;      // 1: stop replacing a column once a replacement stalls
  int general_m;      // 1: ρ = rᵀM⁻¹r comes from a separate dot (pcg_rho_beta)
};

// Finalisation shared by the update and replacement kernels: from ‖r_c‖²
// compute relres, count the iteration, freeze converged or capped columns,
// and form ρ' = rᵀM⁻¹r and β = ρ'/ρ.
__device__ __forceinline__ void pcg_finish_col(const PcgState& S, const PcgScalars& P, int c,
                                               double rr, bool count_iter, bool replaced) {
  if (!S.active[c]) {
    S.beta[c] = 0.0;
    return;
  }
  const int it = S.iters[c] + (count_iter ? 1 : 0);
  S.iters[c] = it;
  const double rel = S.bnorm[c] > 0.0 ? sqrt(rr) / S.bnorm[c] : 0.0;
  S.relres[c] = rel;
  if (!P.general_m) {
    const double rho_new = P.minv * rr;
    S.beta[c] = S.rho[c] != 0.0 ? rho_new / S.rho[c] : 0.0;
    S.rho[c] = rho_new;
  }
  const bool tol_ok = rel <= P.tol && (replaced || !P.replaced_only);
  if (tol_ok || it >= P.max_iter || !(rel < 1e8)) S.active[c] = 0;
  else if (S.bhist && !P.general_m) S.bhist[(size_t)(it - 1) * P.k + c] = S.beta[c];
}

__device__ __forceinline__ void pcg_count_active(const PcgState& S, int k) {
  if (threadIdx.x == 0) {
    int na = 0;
    for (int c = 0; c < k; ++c) na += S.active[c];
    *S.nactive = na;
    if (S.nactive_host) *S.nactive_host = na;  // pinned host mirror (may be null)
  }
}

// x += αp, r −= αq for active columns, then ‖r‖² and finish (finish = 0
// before a replacement, which finishes instead).  α = ρ/pᵀq, or with `pr`
// (pᵀr per column) the line-search step α = pᵀr/pᵀq.  The two agree while
// pᵀr = ρ; a residual replacement breaks that (p was built from the old
// residual), and one line-search step right after it restores it: the new
// r is orthogonal to the step taken, so the next p again has pᵀr = ρ.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void pcg_update(int64_t n, int k, int64_t chunk,
                                                          const T* __restrict__ p,
                                                          const T* __restrict__ q, PcgState S,
                                                          PcgScalars P, int finish,
                                                          const double* __restrict__ pr) {
  __shared__ double sh[kRedThreads];
  const ColLanes L = col_lanes(k);
  const int c = L.c;
  const int r0 = L.r0;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  double acc = 0.0;
  if (c < k && S.active[c]) {
    // α = 0 once the residual is exactly zero (pᵀq = 0): x and r stay put.
    const double num = pr ? pr[c] : S.rho[c];
    const double alpha = S.pq[c] != 0.0 ? num / S.pq[c] : 0.0;
    // The column's iteration count is raised only by the last block, after
    // every block has passed this point.
    if (S.ahist && blockIdx.x == 0 && r0 == 0) S.ahist[(size_t)S.iters[c] * k + c] = alpha;
    // kRowBatch rows' loads in flight; the same arithmetic, ‖r‖² added in
    // row order.
    int64_t i = beg + r0;
    for (; i + (kRowBatch - 1) * L.step < end; i += kRowBatch * L.step) {
      double xv[kRowBatch], pv[kRowBatch], rv[kRowBatch], qv[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        const int64_t o = (i + u * L.step) * k + c;
        xv[u] = S.x[o];
        pv[u] = (double)p[o];
        rv[u] = S.r[o];
        qv[u] = (double)q[o];
      }
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        const int64_t o = (i + u * L.step) * k + c;
        S.x[o] = xv[u] + alpha * pv[u];
        const double rn = rv[u] - alpha * qv[u];
        S.r[o] = rn;
        acc += rn * rn;
      }
    }
    for (; i < end; i += L.step) {
      const int64_t o = i * k + c;
      S.x[o] += alpha * (double)p[o];
      const double rn = S.r[o] - alpha * (double)q[o];
      S.r[o] = rn;
      acc += rn * rn;
    }
  }
  if (!finish) return;
  const bool last = block_colsum_finish(acc, k, S.work, S.counter, sh, [&](int col, double tot) {
    pcg_finish_col(S, P, col, tot, true, false);
  });
  if (last) pcg_count_active(S, k);
}

// r = b − q (true residual) for active columns that still take replacements
// (the others keep their recursive r), then ‖r‖² and finish.
template <typename T, typename TQ>
__global__ __launch_bounds__(kRedThreads) void pcg_replace(int64_t n, int k, int64_t chunk,
                                                           const T* __restrict__ b,
                                                           const TQ* __restrict__ q, PcgState S,
                                                           PcgScalars P) {
  __shared__ double sh[kRedThreads];
  const ColLanes L = col_lanes(k);
  const int c = L.c;
  const int r0 = L.r0;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  double acc = 0.0;
  if (c < k && S.active[c]) {
    const bool keep = S.norepl && S.norepl[c];
    for (int64_t i = beg + r0; i < end; i += L.step) {
      const int64_t o = i * k + c;
      const double rn = keep ? S.r[o] : (double)b[o] - (double)q[o];
      S.r[o] = rn;
      acc += rn * rn;
    }
  }
  const bool last = block_colsum_finish(acc, k, S.work, S.counter, sh, [&](int col, double tot) {
    const bool repl = !(S.norepl && S.norepl[col]);
    const bool was_active = S.active[col] != 0;
    pcg_finish_col(S, P, col, tot, true, repl);
    if (P.stall_off && repl && was_active) {
      if (S.relres[col] >= S.lastrep[col]) S.norepl[col] = 1;
      S.lastrep[col] = S.relres[col];
    }
  });
  if (last) pcg_count_active(S, k);
}

// General preconditioner: with rz = rᵀz (z = M⁻¹r), β = rz/ρ and ρ = rz for
// the active columns (start: ρ = rz only).
__global__ void pcg_rho_beta(int k, PcgState S, const double* __restrict__ rz, int start) {
  const int c = threadIdx.x;
  if (c < k && (start || S.active[c])) {
    S.beta[c] = (!start && S.rho[c] != 0.0) ? rz[c] / S.rho[c] : 0.0;
    S.rho[c] = rz[c];
  }
}

// p = z + βp for active columns (general preconditioner; z FP64).
template <typename T>
__global__ void pcg_pupdate_z(int64_t n, int k, T* __restrict__ p, const double* __restrict__ z,
                              PcgState S) {
  const int64_t count = n * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % k);
    if (S.active[c]) p[e] = (T)(z[e] + S.beta[c] * (double)p[e]);
  }
}

// p = M⁻¹r + βp for active columns (p in the MatVec precision).
template <typename T>
__global__ void pcg_pupdate(int64_t n, int k, T* __restrict__ p, PcgState S, double minv) {
  const int64_t count = n * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % k);
    if (S.active[c]) p[e] = (T)(minv * S.r[e] + S.beta[c] * (double)p[e]);
  }
}

// Start: x = x0 or 0; r = b − K̂x0 or b; ‖b‖, ‖r‖; p = M⁻¹r.
template <typename T>
__global__ __launch_bounds__(kRedThreads) void pcg_start_norms(int64_t n, int k, int64_t chunk,
                                                               const T* __restrict__ b,
                                                               const T* __restrict__ x0,
                                                               const T* __restrict__ q0,
                                                               PcgState S, double* bb_out,
                                                               double* work2,
                                                               unsigned* counter2) {
  __shared__ double sh[kRedThreads];
  const ColLanes L = col_lanes(k);
  const int c = L.c;
  const int r0 = L.r0;
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  double acc = 0.0;
  if (c < k) {
    for (int64_t i = beg + r0; i < end; i += L.step) {
      const int64_t o = i * k + c;
      const double bv = (double)b[o];
      S.x[o] = x0 ? (double)x0[o] : 0.0;
      S.r[o] = q0 ? bv - (double)q0[o] : bv;
      acc += bv * bv;
    }
  }
  (void)block_colsum_finish(acc, k, work2, counter2, sh,
                            [&](int col, double tot) { bb_out[col] = tot; });
}

__global__ void pcg_start_finish(int k, PcgState S, PcgScalars P, const double* bb,
                                 const double* rr) {
  const int c = threadIdx.x;
  if (c < k) {
    const double bn = sqrt(bb[c]);
    S.bnorm[c] = bn;
    const double rel = bn > 0.0 ? sqrt(rr[c]) / bn : 0.0;
    S.relres[c] = rel;
    S.rho[c] = P.minv * rr[c];
    S.iters[c] = 0;
    S.beta[c] = 0.0;
    S.active[c] = (rel > P.tol && P.max_iter > 0) ? 1 : 0;
    if (S.norepl) S.norepl[c] = 0;
    if (S.lastrep) S.lastrep[c] = __builtin_huge_val();
  }
  __syncthreads();
  pcg_count_active(S, k);
}

template <typename T>
__global__ void pcg_pinit(int64_t n, int k, T* __restrict__ p, const double* __restrict__ r,
                          double minv) {
  const int64_t count = n * k;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x)
    p[e] = (T)(minv * r[e]);
}

inline unsigned elem_blocks(int64_t count) {
  const int64_t b = (count + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

}  // namespace
}  // namespace higp
