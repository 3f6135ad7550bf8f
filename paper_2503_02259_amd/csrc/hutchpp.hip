// Hutch++ for the trace term of eq. (2) (Meyer, Musco, Musco & Woodruff
// 2021, cited beside Hutchinson's estimator in "Gaussian Processes").
//
// For each θ ∈ {l, f, s} the matrix whose trace eq. (2) estimates is
//   A_θ = K̂⁻¹·∂K̂/∂θ − c_θ·I,  c_θ = tr-weight of M⁻¹∂M/∂θ,
// with M = diag(K̂) = (f²+s)·I (c_l = 0, c_f = 2f/(f²+s), c_s = 1/(f²+s)) or
// M = I (all c_θ = 0).  The probe block Z (n×N) gives the sketch
// S = Z[:, :N/2] and the Hutchinson probes G = Z[:, N/2:], and
//   tr(A_θ) ≈ tr(Q_θᵀA_θQ_θ) + (1/|G|)·tr(G_θ'ᵀA_θG_θ'),
//   Q_θ = orth(A_θS),  G_θ' = (I − Q_θQ_θᵀ)G.
// Because K̂ is symmetric, qᵀA_θq = (K̂⁻¹q)ᵀ(∂K̂/∂θ·q) − c_θ‖q‖², so every
// term is a column dot of a PCG solution with a derivative MatVec.
//
// Work, all on the device with the library's own kernels:
//   1. ∂K̂/∂θ·S by one fused derivative MatVec;
//   2. one PCG on [y | ∂K̂/∂l·S | ∂K̂/∂f·S | S] (1 + 3|S| ≤ 64 columns);
//   3. Q_θ = orth(A_θS): Gram matrix YᵀY (FP64, fixed-order), its symmetric
//      eigen-decomposition on the host (cyclic Jacobi), Y·VΛ^{-1/2} keeping
//      the directions with σ > 1e-7·σ_max, and a second identical pass that
//      restores orthogonality to rounding level;
//   4. G_θ' = G − Q_θ(Q_θᵀG);
//   5. PCG and the derivative MatVec on [Q_l | Q_f | Q_s | G_l' | G_f' | G_s']
//      in chunks of ≤ 63 columns, then the column dots.
// log|K̂| is SLQ over all of Z as with Hutchinson's estimator.
#include <algorithm>
#include <cmath>
#include <vector>

#include "reduce.h"

namespace higp {

int run_slq(const Problem& p, int N, int m, const void* Z, int reorth, int precond,
            double* logdet, double* per_probe, hipStream_t st);
int host_coldot(int64_t n, int k, const void* A, int ta, const void* B, int tb, double* out,
                hipStream_t st);

namespace {

// Columns c0, c0+1, … of a row-major block with leading dimension ld.
struct Cols {
  const void* p;
  int64_t ld;
  int c0;
  int type;  // 0 = double, 1 = float
};

__device__ __forceinline__ double get(const Cols& B, int64_t i, int c) {
  const int64_t o = i * B.ld + B.c0 + c;
  return B.type ? (double)static_cast<const float*>(B.p)[o] : static_cast<const double*>(B.p)[o];
}

__device__ __forceinline__ void put(const Cols& B, int64_t i, int c, double v) {
  const int64_t o = i * B.ld + B.c0 + c;
  if (B.type)
    static_cast<float*>(const_cast<void*>(B.p))[o] = (float)v;
  else
    static_cast<double*>(const_cast<void*>(B.p))[o] = v;
}

// D = a·A + b·B over nc columns (B.p may be null).
__global__ void hpp_axpby(int64_t n, int nc, Cols A, double a, Cols B, double b, Cols D) {
  const int64_t count = n * nc;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / nc;
    const int c = (int)(e % nc);
    double v = a * get(A, i, c);
    if (B.p) v += b * get(B, i, c);
    put(D, i, c, v);
  }
}

// Gram partials part[blk][p·nb + q] = Σ_{i ∈ chunk blk} A[i][p]·B[i][q]; the
// rows of a chunk are staged through LDS 32 at a time.
constexpr int kGramRows = 32;
__global__ __launch_bounds__(256) void hpp_gram_part(int64_t n, int64_t chunk, int na, Cols A,
                                                     int nb, Cols B, double* __restrict__ part) {
  __shared__ double sa[kGramRows][64];
  __shared__ double sb[kGramRows][64];
  const int64_t beg = (int64_t)blockIdx.x * chunk;
  const int64_t end = beg + chunk < n ? beg + chunk : n;
  const int nab = na * nb;
  double acc[16];
  for (int t = 0; t < 16; ++t) acc[t] = 0.0;
  for (int64_t i0 = beg; i0 < end; i0 += kGramRows) {
    const int rows = (int)(end - i0 < kGramRows ? end - i0 : kGramRows);
    __syncthreads();
    for (int e = threadIdx.x; e < rows * 64; e += blockDim.x) {
      const int r = e / 64, c = e % 64;
      sa[r][c] = c < na ? get(A, i0 + r, c) : 0.0;
      sb[r][c] = c < nb ? get(B, i0 + r, c) : 0.0;
    }
    __syncthreads();
    for (int t = 0; t < 16; ++t) {
      const int e = threadIdx.x + t * 256;
      if (e >= nab) break;
      const int pa = e / nb, qb = e % nb;
      double s = acc[t];
      for (int r = 0; r < rows; ++r) s += sa[r][pa] * sb[r][qb];
      acc[t] = s;
    }
  }
  double* out = part + (size_t)blockIdx.x * nab;
  for (int t = 0; t < 16; ++t) {
    const int e = threadIdx.x + t * 256;
    if (e < nab) out[e] = acc[t];
  }
}

__global__ void hpp_gram_sum(int nparts, int nab, const double* __restrict__ part,
                             double* __restrict__ out) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < nab; e += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += part[(size_t)b * nab + e];
    out[e] = s;
  }
}

// D = Base + sgn·A·C with C (na×nr, row-major, device FP64); Base.p may be
// null (then D = sgn·A·C).
__global__ void hpp_gemm(int64_t n, int na, Cols A, int nr, const double* __restrict__ C,
                         Cols Base, double sgn, Cols D) {
  const int64_t count = n * nr;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / nr;
    const int c = (int)(e % nr);
    double acc = 0.0;
    for (int q = 0; q < na; ++q) acc += get(A, i, q) * C[q * nr + c];
    put(D, i, c, (Base.p ? get(Base, i, c) : 0.0) + sgn * acc);
  }
}

unsigned grid1(int64_t count) {
  const int64_t b = (count + 255) / 256;
  return (unsigned)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

constexpr int kGramParts = 256;

// Eigen-decomposition of the symmetric m×m matrix A (row-major, destroyed)
// by cyclic Jacobi rotations (Golub & Van Loan, "Matrix Computations", the
// cyclic Jacobi method); w: eigenvalues, V: eigenvectors as columns.
void sym_eig(int m, std::vector<double>& A, std::vector<double>& w, std::vector<double>& V) {
  V.assign((size_t)m * m, 0.0);
  for (int i = 0; i < m; ++i) V[(size_t)i * m + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < m; ++j) {
        const double a2 = A[(size_t)i * m + j] * A[(size_t)i * m + j];
        tot += a2;
        if (i != j) off += a2;
      }
    if (off <= 1e-30 * tot || off == 0.0) break;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[(size_t)p * m + q];
        if (apq == 0.0) continue;
        const double app = A[(size_t)p * m + p], aqq = A[(size_t)q * m + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) /
                         (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        // A ← JᵀAJ with the rotation J in the (p, q) plane.
        for (int k = 0; k < m; ++k) {
          const double akp = A[(size_t)k * m + p], akq = A[(size_t)k * m + q];
          A[(size_t)k * m + p] = c * akp - s * akq;
          A[(size_t)k * m + q] = s * akp + c * akq;
        }
        for (int k = 0; k < m; ++k) {
          const double apk = A[(size_t)p * m + k], aqk = A[(size_t)q * m + k];
          A[(size_t)p * m + k] = c * apk - s * aqk;
          A[(size_t)q * m + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < m; ++k) {
          const double vkp = V[(size_t)k * m + p], vkq = V[(size_t)k * m + q];
          V[(size_t)k * m + p] = c * vkp - s * vkq;
          V[(size_t)k * m + q] = s * vkp + c * vkq;
        }
      }
  }
  w.resize(m);
  for (int i = 0; i < m; ++i) w[i] = A[(size_t)i * m + i];
}

struct Ctx {
  int64_t n;
  hipStream_t st;
  double* part;    // kGramParts × 64 × 64
  double* dsmall;  // 64 × 64 device matrix (Gram result or uploaded factor)
  std::vector<double> host;
};

// AᵀB (na×nb ≤ 64×64) into ctx.host.
int gram(Ctx& x, int na, Cols A, int nb, Cols B) {
  const int64_t chunk = (x.n + kGramParts - 1) / kGramParts;
  const int parts = (int)((x.n + chunk - 1) / chunk);
  hipLaunchKernelGGL(hpp_gram_part, dim3(parts), dim3(256), 0, x.st, x.n, chunk, na, A, nb, B,
                     x.part);
  hipLaunchKernelGGL(hpp_gram_sum, dim3(grid1(na * nb)), dim3(256), 0, x.st, parts, na * nb,
                     (const double*)x.part, x.dsmall);
  x.host.assign((size_t)na * nb, 0.0);
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(x.host.data(), x.dsmall, (size_t)na * nb * 8, hipMemcpyDeviceToHost,
                     x.st) != hipSuccess ||
      hipStreamSynchronize(x.st) != hipSuccess)
    return set_error(HIGP_ERR_HIP, "Gram matrix failed");
  return HIGP_OK;
}

// D = Base + sgn·A·C with the host matrix C (na×nr) uploaded first.
int gemm(Ctx& x, int na, Cols A, int nr, const std::vector<double>& C, Cols Base, double sgn,
         Cols D) {
  if (hipMemcpyAsync(x.dsmall, C.data(), (size_t)na * nr * 8, hipMemcpyHostToDevice, x.st) !=
      hipSuccess)
    return set_error(HIGP_ERR_HIP, "upload failed");
  hipLaunchKernelGGL(hpp_gemm, dim3(grid1(x.n * nr)), dim3(256), 0, x.st, x.n, na, A, nr,
                     (const double*)x.dsmall, Base, sgn, D);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(x.st) != hipSuccess)
    return set_error(HIGP_ERR_HIP, "block product failed");
  return HIGP_OK;
}

// One orthonormalisation pass: from the Gram matrix YᵀY = VΛVᵀ, the factor
// C = V_r Λ_r^{-1/2} over the directions with λ > cut·λ_max (cut = 0: all
// positive ones).  Returns the kept count r.
int orth_factor(int m, std::vector<double> G, double cut, std::vector<double>& C) {
  std::vector<double> w, V;
  sym_eig(m, G, w, V);
  double wmax = 0.0;
  for (double v : w) wmax = std::max(wmax, v);
  std::vector<int> keep;
  for (int i = 0; i < m; ++i)
    if (wmax > 0.0 && w[i] > cut * wmax && w[i] > 0.0) keep.push_back(i);
  const int r = (int)keep.size();
  C.assign((size_t)m * std::max(r, 1), 0.0);
  for (int j = 0; j < r; ++j) {
    const double sc = 1.0 / std::sqrt(w[keep[j]]);
    for (int i = 0; i < m; ++i) C[(size_t)i * r + j] = V[(size_t)i * m + keep[j]] * sc;
  }
  return r;
}

template <typename T>
int hutchpp_impl(const Problem& p, const void* y, int N, const void* Z, const higp_nlml_opts& o,
                 double* loss, double* grad, double* logdet_out, int32_t* iters_out,
                 hipStream_t st) {
  const int64_t n = p.n;
  const int tt = p.prec == HIGP_FP64 ? 0 : 1;
  const int ns = N / 2, ng = N - ns;
  const int k1 = 1 + 3 * ns;
  const int k2max = 3 * N;
  constexpr int kChunk = 63;
  size_t bytes = 0;
  auto take = [&](size_t b) {
    size_t off = bytes;
    bytes += (b + 255) / 256 * 256;
    return off;
  };
  const size_t es = sizeof(T);
  const size_t o_s = take(n * ns * es), o_dls = take(n * ns * es), o_dfs = take(n * ns * es),
               o_b1 = take(n * k1 * es), o_x1 = take(n * k1 * es), o_w1 = take(n * k1 * 8),
               o_y = take(n * ns * 8), o_qt = take(n * ns * 8), o_b2 = take(n * k2max * 8),
               o_bc = take(n * kChunk * es), o_xc = take(n * kChunk * es),
               o_wc = take(n * kChunk * 8), o_dlc = take(n * kChunk * es),
               o_dfc = take(n * kChunk * es), o_at = take(n * es), o_ad = take(n * 8),
               o_dla = take(n * es), o_dfa = take(n * es),
               o_part = take((size_t)kGramParts * 64 * 64 * 8), o_small = take(64 * 64 * 8);
  void* mem = nullptr;
  HIGP_TRY(scratch_alloc(&mem, bytes, st));
  char* base = static_cast<char*>(mem);
  auto at = [&](size_t off) { return static_cast<void*>(base + off); };
  auto done = [&](int rc) {
    (void)hipStreamSynchronize(st);
    scratch_free(mem, st);
    return rc;
  };
  Ctx x{n, st, (double*)at(o_part), (double*)at(o_small), {}};
  auto view = [](const void* ptr, int64_t ld, int c0, int type) { return Cols{ptr, ld, c0, type}; };
  const Cols none{nullptr, 0, 0, 0};
  auto axpby = [&](int nc, Cols A, double a, Cols B, double b, Cols D) {
    hipLaunchKernelGGL(hpp_axpby, dim3(grid1(n * nc)), dim3(256), 0, st, n, nc, A, a, B, b, D);
    return hipGetLastError() == hipSuccess ? HIGP_OK
                                           : set_error(HIGP_ERR_HIP, "block copy failed");
  };

  higp_pcg_opts po{};
  po.tol = o.tol;
  po.max_iter = o.max_iter;
  po.precond = o.precond;
  po.refine_every = o.refine_every;
  po.refine_prec = HIGP_FP64;
  std::vector<int32_t> its(64);
  std::vector<double> rel(64);
  std::vector<int32_t> conv(64);
  higp_pcg_info info{its.data(), rel.data(), conv.data()};
  int itmax = 0;
  auto solve = [&](int k, const void* B, void* X, double* W) {
    po.x_fp64 = W;
    int rc = run_pcg(p, k, B, X, po, &info, st);
    for (int c = 0; c < k; ++c) itmax = std::max(itmax, its[c]);
    return rc;
  };

  const double m = p.f * p.f + p.s;
  const double cth[3] = {0.0, o.precond ? 2.0 * p.f / m : 0.0, o.precond ? 1.0 / m : 0.0};
  int rc;

  // 1–2. ∂K̂/∂θ·S and the first solve.
  const Cols zc = view(Z, N, 0, tt);
  if ((rc = axpby(ns, zc, 1.0, none, 0.0, view(at(o_s), ns, 0, tt)))) return done(rc);
  {
    MatvecOut mo;
    mo.dl = at(o_dls);
    mo.df = at(o_dfs);
    if ((rc = launch_kmatvec(p, ns, at(o_s), mo, st))) return done(rc);
  }
  if ((rc = axpby(1, view(y, 1, 0, tt), 1.0, none, 0.0, view(at(o_b1), k1, 0, tt))) ||
      (rc = axpby(ns, view(at(o_dls), ns, 0, tt), 1.0, none, 0.0, view(at(o_b1), k1, 1, tt))) ||
      (rc = axpby(ns, view(at(o_dfs), ns, 0, tt), 1.0, none, 0.0,
                  view(at(o_b1), k1, 1 + ns, tt))) ||
      (rc = axpby(ns, view(at(o_s), ns, 0, tt), 1.0, none, 0.0,
                  view(at(o_b1), k1, 1 + 2 * ns, tt))))
    return done(rc);
  if ((rc = solve(k1, at(o_b1), at(o_x1), (double*)at(o_w1)))) return done(rc);

  // 3. Q_θ = orth(A_θS) into the leading columns of the FP64 block B2.
  int r[3], qoff[3];
  int rt = 0;
  std::vector<double> C1, C2;
  for (int t = 0; t < 3; ++t) {
    // Y = K̂⁻¹(∂K̂/∂θ·S) − c_θ·S
    if ((rc = axpby(ns, view(at(o_w1), k1, 1 + t * ns, 0), 1.0, view(at(o_s), ns, 0, tt),
                    -cth[t], view(at(o_y), ns, 0, 0))))
      return done(rc);
    const Cols yv = view(at(o_y), ns, 0, 0);
    if ((rc = gram(x, ns, yv, ns, yv))) return done(rc);
    const int r1 = orth_factor(ns, x.host, 1e-14, C1);
    if (r1 == 0) {
      r[t] = 0;
      qoff[t] = rt;
      continue;
    }
    const Cols qt = view(at(o_qt), ns, 0, 0);
    if ((rc = gemm(x, ns, yv, r1, C1, none, 1.0, qt))) return done(rc);
    const Cols q1 = view(at(o_qt), ns, 0, 0);
    if ((rc = gram(x, r1, q1, r1, q1))) return done(rc);
    const int r2 = orth_factor(r1, x.host, 0.0, C2);
    if (r2 != r1)
      return done(set_error(HIGP_ERR_UNSUPPORTED,
                            "Hutch++: the sketch lost rank in its second orthonormalisation"));
    qoff[t] = rt;
    r[t] = r2;
    if ((rc = gemm(x, r1, q1, r2, C2, none, 1.0, view(at(o_b2), k2max, rt, 0)))) return done(rc);
    rt += r2;
  }
  // 4. G_θ' = G − Q_θ(Q_θᵀG) after the Q columns.
  const Cols gv = view(Z, N, ns, tt);
  const int goff = rt;
  for (int t = 0; t < 3; ++t) {
    const Cols dst = view(at(o_b2), k2max, goff + t * ng, 0);
    if (r[t] == 0) {
      if ((rc = axpby(ng, gv, 1.0, none, 0.0, dst))) return done(rc);
      continue;
    }
    const Cols qv = view(at(o_b2), k2max, qoff[t], 0);
    if ((rc = gram(x, r[t], qv, ng, gv))) return done(rc);
    if ((rc = gemm(x, r[t], qv, ng, x.host, gv, -1.0, dst))) return done(rc);
  }
  const int k2 = rt + 3 * ng;

  // 5. Solves and derivative MatVecs of B2 in chunks; column dots.
  double top[3] = {0.0, 0.0, 0.0}, rest[3] = {0.0, 0.0, 0.0};
  std::vector<double> dl(kChunk), df(kChunk), ds(kChunk), nn(kChunk);
  for (int cb = 0; cb < k2; cb += kChunk) {
    const int kc = std::min(kChunk, k2 - cb);
    if ((rc = axpby(kc, view(at(o_b2), k2max, cb, 0), 1.0, none, 0.0, view(at(o_bc), kc, 0, tt))))
      return done(rc);
    if ((rc = solve(kc, at(o_bc), at(o_xc), (double*)at(o_wc)))) return done(rc);
    MatvecOut mo;
    mo.dl = at(o_dlc);
    mo.df = at(o_dfc);
    if ((rc = launch_kmatvec(p, kc, at(o_bc), mo, st))) return done(rc);
    if ((rc = host_coldot(n, kc, at(o_wc), 0, at(o_dlc), tt, dl.data(), st)) ||
        (rc = host_coldot(n, kc, at(o_wc), 0, at(o_dfc), tt, df.data(), st)) ||
        (rc = host_coldot(n, kc, at(o_wc), 0, at(o_bc), tt, ds.data(), st)) ||
        (rc = host_coldot(n, kc, at(o_bc), tt, at(o_bc), tt, nn.data(), st)))
      return done(rc);
    for (int c = 0; c < kc; ++c) {
      const int g = cb + c;
      int t;
      bool is_q;
      if (g < goff) {
        is_q = true;
        t = g < qoff[1] ? 0 : (g < qoff[2] ? 1 : 2);
      } else {
        is_q = false;
        t = (g - goff) / ng;
      }
      const double quad = (t == 0 ? dl[c] : (t == 1 ? df[c] : ds[c])) - cth[t] * nn[c];
      if (is_q)
        top[t] += quad;
      else
        rest[t] += quad;
    }
  }

  // α = K̂⁻¹y and its terms: αᵀ∂K̂/∂θα, yᵀα.
  if ((rc = axpby(1, view(at(o_w1), k1, 0, 0), 1.0, none, 0.0, view(at(o_ad), 1, 0, 0))) ||
      (rc = axpby(1, view(at(o_w1), k1, 0, 0), 1.0, none, 0.0, view(at(o_at), 1, 0, tt))))
    return done(rc);
  {
    MatvecOut mo;
    mo.dl = at(o_dla);
    mo.df = at(o_dfa);
    if ((rc = launch_kmatvec(p, 1, at(o_at), mo, st))) return done(rc);
  }
  double qa[3], ya;
  if ((rc = host_coldot(n, 1, at(o_ad), 0, at(o_dla), tt, &qa[0], st)) ||
      (rc = host_coldot(n, 1, at(o_ad), 0, at(o_dfa), tt, &qa[1], st)) ||
      (rc = host_coldot(n, 1, at(o_ad), 0, at(o_at), tt, &qa[2], st)) ||
      (rc = host_coldot(n, 1, at(o_ad), 0, y, tt, &ya, st)))
    return done(rc);

  double logdet = 0.0;
  if ((rc = run_slq(p, N, o.nsteps, Z, o.reorth, o.precond, &logdet, nullptr, st)))
    return done(rc);
  done(HIGP_OK);

  for (int t = 0; t < 3; ++t)
    grad[t] = 0.5 * (-qa[t] + cth[t] * (double)n + top[t] + rest[t] / ng);
  *loss = 0.5 * (ya + logdet + (double)n * std::log(2.0 * M_PI));
  if (logdet_out) *logdet_out = logdet;
  if (iters_out) *iters_out = itmax;
  return HIGP_OK;
}

}  // namespace

int run_nlml_hutchpp(const Problem& p, const void* y, int N, const void* Z,
                     const higp_nlml_opts& o, double* loss, double* grad, double* logdet,
                     int32_t* iters, hipStream_t st) {
  if (p.prec == HIGP_FP64) return hutchpp_impl<double>(p, y, N, Z, o, loss, grad, logdet, iters, st);
  if (p.prec == HIGP_FP32) return hutchpp_impl<float>(p, y, N, Z, o, loss, grad, logdet, iters, st);
  return set_error(HIGP_ERR_UNSUPPORTED, "Hutch++ runs in FP64 or FP32");
}

}  // namespace higp
