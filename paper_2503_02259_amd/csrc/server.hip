// Continuous-batching serving of independent GP solves.
//
// Each request is one GP problem (FP32 points X, targets y, probes Z) for
// which the server computes K̂⁻¹y by CG (Jacobi-preconditioned, to a
// tolerance on the recursive residual) and log|K̂| by eq. (1) with SLQ over
// the probes — the two quantities of the negative log marginal likelihood
// ("Gaussian Processes").  Requests are admitted from a FIFO queue while a
// slot is free and their device state fits in the HBM budget; admitted
// requests keep X, their vectors and all CG/Lanczos state resident.  Every
// round runs ONE batched MatVec for all active requests (the CG column and
// the live Lanczos columns of each request form its k ≤ 32 columns), then
// each request's CG and Lanczos updates (scalars stay on the device; the
// host only reads two pinned status words per request per round).  Finished
// requests are retired and their memory returned before the next admission.
//
// A request's arithmetic — its split counts, reduction orders, scalars — is a
// function of that request alone, so its results are bitwise the same whether
// it runs alone or among others.
#include <cmath>
#include <deque>
#include <memory>
#include <vector>

#include "lanczos_kernels.h"
#include "nystrom.h"
#include "pcg_kernels.h"

namespace higp {
namespace {

// Vin[i][0] = p[i] (CG) and Vin[i][c0 + c] = QW[i][c] (Lanczos), zero beyond.
__global__ void srv_pack(int64_t n, int kr, int cg, int N, const float* __restrict__ p,
                         const float* __restrict__ QW, float* __restrict__ Vin, int64_t count_pad) {
  const int64_t count = n * kr;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count_pad;
       e += (int64_t)gridDim.x * blockDim.x) {
    float v = 0.0f;
    if (e < count) {
      const int64_t i = e / kr;
      const int c = (int)(e % kr);
      v = (cg && c == 0) ? p[i] : QW[i * N + (c - cg)];
    }
    Vin[e] = v;
  }
}

// q[i] = Vout[i][0] (CG), WW[i][c] = Vout[i][cg + c] (Lanczos).
__global__ void srv_unpack(int64_t n, int kr, int cg, int N, int lz, const float* __restrict__ Vout,
                           float* __restrict__ q, float* __restrict__ WW) {
  const int64_t count = n * kr;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / kr;
    const int c = (int)(e % kr);
    if (cg && c == 0) q[i] = Vout[e];
    else if (lz) WW[i * N + (c - cg)] = Vout[e];
  }
}

// x_out = (float) x
__global__ void srv_cast(int64_t n, const double* __restrict__ x, float* __restrict__ y) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    y[e] = (float)x[e];
}

size_t rup(size_t b) { return (b + 255) / 256 * 256; }

struct Request {
  int64_t id = 0;
  higp_request req{};
  Problem p{};
  int state = HIGP_REQ_QUEUED;
  size_t footprint = 0;   // state bytes + Nyström factor bytes (admission budget)
  size_t state_bytes = 0; // the part allocated as r.mem
  void* mem = nullptr;
  // device state
  float* Xp = nullptr;
  float* Vin = nullptr;
  float* Vout = nullptr;
  float* cg_p = nullptr;
  float* cg_q = nullptr;
  float* QW = nullptr;
  float* WW = nullptr;
  double* zn2 = nullptr;
  double* bb = nullptr;
  double* rr0 = nullptr;
  double* work2 = nullptr;
  unsigned* counter2 = nullptr;
  PcgState S{};
  PcgScalars ps{};
  NysPrec np{};           // Nyström preconditioner (precond_rank > 0)
  double* z = nullptr;    // M⁻¹r (Nyström)
  double* rz = nullptr;   // rᵀM⁻¹r
  LzState L{};
  int N = 0, m = 0;
  int slot = -1;          // index into the pinned status array
  bool cg_active = false;
  bool lz_active = false;
  int lz_step = 0;
  int rounds = 0;
  higp_request_status out{};
};

size_t request_footprint(int64_t n, int d, int N, int m, int rank) {
  const int kmax = 1 + N;
  const size_t nk_pad = ((size_t)n * kmax + 3) / 4 * 4;
  const RedGrid g = red_grid(n);
  size_t b = rup(prepared_points_bytes(n, d)) + 2 * rup(nk_pad * 4);   // Xp, Vin, Vout
  b += 2 * rup((size_t)n * 8) + 2 * rup((size_t)n * 4);               // x, r, p, q
  b += rup(8 * 64 * 8) + rup(4 * 64 * 4) + 2 * rup((size_t)g.blocks * 64 * 8) + rup(16);
  if (N > 0) {
    b += lz_state_bytes(n, N, m) + 2 * rup((size_t)n * N * 4) + rup(64 * 8);  // Lanczos, QW, WW, zn2
  }
  b += (size_t)batch_splits(n) * n * kmax * 4;                         // batch partials
  if (rank > 0) b += nys_bytes(n, rank, 1, HIGP_FP32) + rup((size_t)n * 8) + rup(64);
  return b;
}

struct Server {
  higp_server_opts opts{};
  hipStream_t st = nullptr;
  int num_cus = 256;
  int64_t next_id = 1;
  size_t used = 0;
  std::deque<std::unique_ptr<Request>> queue;
  std::vector<std::unique_ptr<Request>> active;
  std::vector<std::unique_ptr<Request>> finished;  // retired, kept for status queries
  int* status_d = nullptr;           // device: [slot][0] CG active columns, [slot][1] live probes
  int* status_h = nullptr;           // pinned host copy, refreshed once per round
  std::vector<int> free_slots;
};

int admit(Server& sv, Request& r) {
  const int64_t n = r.p.n;
  const int N = r.N, m = r.m;
  const int kmax = 1 + N;
  const size_t nk_pad = ((size_t)n * kmax + 3) / 4 * 4;
  HIGP_TRY(scratch_alloc(&r.mem, r.state_bytes, sv.st));
  char* base = static_cast<char*>(r.mem);
  size_t off = 0;
  auto take = [&](size_t b) {
    char* q = base + off;
    off += rup(b);
    return q;
  };
  const RedGrid g = red_grid(n);
  r.Xp = (float*)take(prepared_points_bytes(n, r.p.d));
  r.Vin = (float*)take(nk_pad * 4);
  r.Vout = (float*)take(nk_pad * 4);
  r.S.x = (double*)take((size_t)n * 8);
  r.S.r = (double*)take((size_t)n * 8);
  r.cg_p = (float*)take((size_t)n * 4);
  r.cg_q = (float*)take((size_t)n * 4);
  if (r.req.precond_rank > 0) {
    r.z = (double*)take((size_t)n * 8);
    r.rz = (double*)take(64);
  }
  double* sc = (double*)take(8 * 64 * 8);
  r.S.rho = sc;
  r.S.pq = sc + 64;
  r.S.beta = sc + 128;
  r.S.bnorm = sc + 192;
  r.S.relres = sc + 256;
  r.bb = sc + 320;
  r.rr0 = sc + 384;
  int* in = (int*)take(4 * 64 * 4);
  r.S.active = in;
  r.S.iters = in + 64;
  r.S.work = (double*)take((size_t)g.blocks * 64 * 8);
  r.work2 = (double*)take((size_t)g.blocks * 64 * 8);
  unsigned* cnt = (unsigned*)take(16);
  r.S.counter = cnt;
  r.counter2 = cnt + 1;
  if (N > 0) {
    const size_t lb = lz_state_bytes(n, N, m);
    r.L = lz_carve((char*)take(lb), n, N, m);
    r.QW = (float*)take((size_t)n * N * 4);
    r.WW = (float*)take((size_t)n * N * 4);
    r.zn2 = (double*)take(64 * 8);
  }
  if (off > r.state_bytes) return set_error(HIGP_ERR_HIP, "internal: footprint underestimated");

  r.slot = sv.free_slots.back();
  sv.free_slots.pop_back();
  r.S.nactive = sv.status_d + 2 * r.slot;
  r.S.nactive_host = nullptr;
  if (N > 0) {
    r.L.nlive = sv.status_d + 2 * r.slot + 1;
    r.L.nlive_host = nullptr;
  }

  hipStream_t st = sv.st;
  HIGP_TRY(prepare_points_f32(r.p, r.Xp, st));
  if (hipMemsetAsync(cnt, 0, 16, st) != hipSuccess ||
      (N > 0 && hipMemsetAsync(r.L.counter, 0, 8, st) != hipSuccess))
    return set_error(HIGP_ERR_HIP, "initialisation failed");
  // CG start: x = 0, r = y, ‖y‖, p = M⁻¹r.
  r.ps.tol = r.req.tol;
  r.ps.max_iter = r.req.max_iter;
  r.ps.minv = 1.0 / (r.p.f * r.p.f + r.p.s);
  hipLaunchKernelGGL((pcg_start_norms<float>), dim3(g.blocks), dim3(kRedThreads), 0, st, n, 1,
                     g.chunk, (const float*)r.req.y, (const float*)nullptr,
                     (const float*)nullptr, r.S, r.bb, r.work2, r.counter2);
  HIGP_TRY(launch_coldot(n, 1, r.S.r, 0, r.S.r, 0, r.rr0, r.S.work, r.S.counter, st));
  hipLaunchKernelGGL(pcg_start_finish, dim3(1), dim3(64), 0, st, 1, r.S, r.ps, (const double*)r.bb,
                     (const double*)r.rr0);
  hipLaunchKernelGGL((pcg_pinit<float>), dim3(elem_blocks(n)), dim3(256), 0, st, n, 1, r.cg_p,
                     (const double*)r.S.r, r.ps.minv);
  if (r.req.precond_rank > 0) {
    // Nyström: z₀ = M⁻¹r₀, ρ = r₀ᵀz₀, p = z₀ (replaces p = M⁻¹r₀ with Jacobi).
    HIGP_TRY(nys_build(r.p, r.req.precond_rank, 1, &r.np, st));
    r.ps.general_m = 1;
    HIGP_TRY(nys_apply(r.np, 1, r.S.r, r.z, st));
    HIGP_TRY(launch_coldot(n, 1, r.S.r, 0, r.z, 0, r.rz, r.S.work, r.S.counter, st));
    hipLaunchKernelGGL(pcg_rho_beta, dim3(1), dim3(64), 0, st, 1, r.S, (const double*)r.rz, 1);
    HIGP_TRY(launch_cast_scale(n, r.z, 0, r.cg_p, 1, 1.0, st));
  }
  r.cg_active = true;
  // Lanczos start: q₀ = z/‖z‖ on K̂/(f²+s).
  if (N > 0) {
    const double isq = 1.0 / std::sqrt(r.p.f * r.p.f + r.p.s);
    HIGP_TRY(launch_coldot(n, N, r.req.Z, 1, r.req.Z, 1, r.zn2, r.L.work, r.L.counter, st));
    hipLaunchKernelGGL((lz_first<float>), dim3(lz_blocks((int64_t)n * N)), dim3(256), 0, st,
                       (int64_t)n * N, N, (const float*)r.req.Z, (const double*)r.zn2, r.QW, isq,
                       r.L);
    r.lz_active = true;
  }
  if (hipGetLastError() != hipSuccess) return set_error(HIGP_ERR_HIP, "admission launch failed");
  r.state = HIGP_REQ_ACTIVE;
  return HIGP_OK;
}

int retire(Server& sv, Request& r) {
  hipStream_t st = sv.st;
  const int64_t n = r.p.n;
  const int N = r.N, m = r.m;
  hipLaunchKernelGGL(srv_cast, dim3(elem_blocks(n)), dim3(256), 0, st, n, (const double*)r.S.x,
                     static_cast<float*>(r.req.x_out));
  int it = 0;
  double rel = 0.0;
  std::vector<double> ah((size_t)m * N), bh((size_t)m * N), zh(N);
  std::vector<int> steps(N);
  int rc = HIGP_OK;
  if (hipMemcpyAsync(&it, r.S.iters, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(&rel, r.S.relres, 8, hipMemcpyDeviceToHost, st) != hipSuccess)
    rc = set_error(HIGP_ERR_HIP, "result copy failed");
  if (rc == HIGP_OK && N > 0 &&
      (hipMemcpyAsync(ah.data(), r.L.ahist, ah.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
       hipMemcpyAsync(bh.data(), r.L.bhist, bh.size() * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
       hipMemcpyAsync(steps.data(), r.L.steps, N * 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
       hipMemcpyAsync(zh.data(), r.zn2, N * 8, hipMemcpyDeviceToHost, st) != hipSuccess))
    rc = set_error(HIGP_ERR_HIP, "result copy failed");
  if (hipStreamSynchronize(st) != hipSuccess && rc == HIGP_OK)
    rc = set_error(HIGP_ERR_HIP, "synchronisation failed");
  r.out.iters = it;
  r.out.relres = rel;
  r.out.converged = rel <= r.req.tol ? 1 : 0;
  r.out.logdet = NAN;
  r.out.lanczos_steps = 0;
  if (rc == HIGP_OK && N > 0) {
    const double m_ = r.p.f * r.p.f + r.p.s;
    const double logm = (double)n * std::log(m_);
    double total = 0.0;
    int minsteps = m;
    std::vector<double> a, b, th, tau;
    for (int c = 0; c < N && rc == HIGP_OK; ++c) {
      const int mc = steps[c];
      minsteps = std::min(minsteps, mc);
      if (mc < 1) {
        rc = set_error(HIGP_ERR_INVALID_ARG, "request %lld: probe %d is zero", (long long)r.id, c);
        break;
      }
      a.resize(mc);
      b.resize(mc > 1 ? mc - 1 : 1);
      for (int i = 0; i < mc; ++i) a[i] = ah[(size_t)i * N + c];
      for (int i = 0; i + 1 < mc; ++i) b[i] = bh[(size_t)i * N + c];
      th.assign(mc, 0.0);
      tau.assign(mc, 0.0);
      rc = higp_tridiag_eig(mc, a.data(), b.data(), th.data(), tau.data());
      double q = 0.0;
      for (int i = 0; i < mc; ++i) q += tau[i] * tau[i] * std::log(th[i]);
      total += logm + zh[c] * q;
    }
    r.out.logdet = total / N;
    r.out.lanczos_steps = minsteps;
  }
  r.out.rounds = r.rounds;
  r.out.state = rc == HIGP_OK ? HIGP_REQ_DONE : HIGP_REQ_FAILED;
  r.state = r.out.state;
  nys_free(r.np, st);
  scratch_free(r.mem, st);
  r.mem = nullptr;
  sv.used -= r.footprint;
  sv.free_slots.push_back(r.slot);
  r.slot = -1;
  return rc;
}

int run_round(Server& sv) {
  hipStream_t st = sv.st;
  // 1. Admission (FIFO) while a slot is free and the state fits.
  while (!sv.queue.empty() && !sv.free_slots.empty() &&
         sv.used + sv.queue.front()->footprint <= sv.opts.hbm_budget) {
    std::unique_ptr<Request> r = std::move(sv.queue.front());
    sv.queue.pop_front();
    sv.used += r->footprint;
    const int rc = admit(sv, *r);
    if (rc != HIGP_OK) {
      r->state = r->out.state = HIGP_REQ_FAILED;
      nys_free(r->np, st);
      if (r->mem) scratch_free(r->mem, st);
      r->mem = nullptr;
      sv.used -= r->footprint;
      if (r->slot >= 0) sv.free_slots.push_back(r->slot);
      sv.finished.push_back(std::move(r));
      return rc;
    }
    sv.active.push_back(std::move(r));
  }
  if (sv.active.empty()) return HIGP_OK;

  // 2. One batched MatVec for every active request (one persistent launch
  //    per column kind; large single-column requests take the symmetric
  //    block-pair kind).
  std::vector<BatchMatvec> jobs;
  std::vector<Request*> owners;
  for (auto& up : sv.active) {
    Request& r = *up;
    const int cg = r.cg_active ? 1 : 0;
    const int lz = r.lz_active ? 1 : 0;
    const int kr = cg + lz * r.N;
    if (kr == 0) continue;
    const int64_t count_pad = (r.p.n * kr + 3) / 4 * 4;
    hipLaunchKernelGGL(srv_pack, dim3(elem_blocks(count_pad)), dim3(256), 0, st, r.p.n, kr, cg,
                       r.N > 0 ? r.N : 1, (const float*)r.cg_p, (const float*)r.QW, r.Vin,
                       count_pad);
    BatchMatvec j{};
    j.Xp = r.Xp;
    j.V = r.Vin;
    j.Y = r.Vout;
    j.n = r.p.n;
    j.k = kr;
    j.d = r.p.d;
    j.kernel = r.p.kernel;
    j.flags = r.p.flags;
    j.f = r.p.f;
    j.s = r.p.s;
    jobs.push_back(j);
    owners.push_back(&r);
  }
  HIGP_TRY(launch_kmatvec_f32_batch(jobs.data(), (int)jobs.size(), st, sv.num_cus));

  // 3. Per-request CG and Lanczos updates.
  for (size_t q = 0; q < owners.size(); ++q) {
    Request& r = *owners[q];
    const int cg = r.cg_active ? 1 : 0;
    const int lz = r.lz_active ? 1 : 0;
    const int kr = jobs[q].k;
    const int64_t n = r.p.n;
    hipLaunchKernelGGL(srv_unpack, dim3(elem_blocks(n * kr)), dim3(256), 0, st, n, kr, cg,
                       r.N > 0 ? r.N : 1, lz, (const float*)r.Vout, r.cg_q, r.WW);
    if (cg) {
      const RedGrid g = red_grid(n);
      HIGP_TRY(launch_coldot(n, 1, r.cg_p, 1, r.cg_q, 1, r.S.pq, r.S.work, r.S.counter, st));
      hipLaunchKernelGGL((pcg_update<float>), dim3(g.blocks), dim3(kRedThreads), 0, st, n, 1,
                         g.chunk, (const float*)r.cg_p, (const float*)r.cg_q, r.S, r.ps, 1,
                         (const double*)nullptr);
      if (r.np.mem) {
        HIGP_TRY(nys_apply(r.np, 1, r.S.r, r.z, st));
        HIGP_TRY(launch_coldot(n, 1, r.S.r, 0, r.z, 0, r.rz, r.S.work, r.S.counter, st));
        hipLaunchKernelGGL(pcg_rho_beta, dim3(1), dim3(64), 0, st, 1, r.S, (const double*)r.rz, 0);
        hipLaunchKernelGGL((pcg_pupdate_z<float>), dim3(elem_blocks(n)), dim3(256), 0, st, n, 1,
                           r.cg_p, (const double*)r.z, r.S);
      } else {
        hipLaunchKernelGGL((pcg_pupdate<float>), dim3(elem_blocks(n)), dim3(256), 0, st, n, 1,
                           r.cg_p, r.S, r.ps.minv);
      }
    }
    if (lz) {
      const double isq = 1.0 / std::sqrt(r.p.f * r.p.f + r.p.s);
      lz_launch_step<float>(n, r.N, r.lz_step, r.m, true, isq, r.WW, r.QW, r.L, st);
      r.lz_step++;
    }
    r.rounds++;
  }
  if (hipGetLastError() != hipSuccess) return set_error(HIGP_ERR_HIP, "update launch failed");
  if (hipMemcpyAsync(sv.status_h, sv.status_d, (size_t)sv.opts.max_active * 2 * sizeof(int),
                     hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return set_error(HIGP_ERR_HIP, "synchronisation failed");

  // 4. Status and retirement.
  int rc = HIGP_OK;
  for (size_t q = 0; q < sv.active.size();) {
    Request& r = *sv.active[q];
    const int* stat = sv.status_h + 2 * r.slot;
    r.cg_active = stat[0] > 0;
    r.lz_active = r.N > 0 && r.lz_step < r.m && stat[1] > 0;
    if (!r.cg_active && !r.lz_active) {
      const int rr = retire(sv, r);
      if (rr != HIGP_OK && rc == HIGP_OK) rc = rr;
      sv.finished.push_back(std::move(sv.active[q]));
      sv.active.erase(sv.active.begin() + q);
    } else {
      ++q;
    }
  }
  return rc;
}

Request* find(Server& sv, int64_t id) {
  for (auto& r : sv.active)
    if (r->id == id) return r.get();
  for (auto& r : sv.queue)
    if (r->id == id) return r.get();
  for (auto& r : sv.finished)
    if (r->id == id) return r.get();
  return nullptr;
}

}  // namespace
}  // namespace higp

using namespace higp;

extern "C" {

uint64_t higp_request_footprint(int64_t n, int32_t d, int32_t nprobe, int32_t nsteps,
                                int32_t precond_rank) {
  if (n < 1 || d < 1 || d > HIGP_MAX_D || nprobe < 0 || nprobe > 31 || nsteps < 0 ||
      precond_rank < 0 || precond_rank > 2048)
    return 0;
  const int m = nprobe > 0 ? nsteps : 0;
  return (uint64_t)(request_footprint(n, d, nprobe, m, 0) +
                    (precond_rank > 0 ? request_footprint(n, d, nprobe, m, precond_rank) -
                                            request_footprint(n, d, nprobe, m, 0) : 0));
}

int higp_server_create(const higp_server_opts* o, higp_server** out) {
  clear_error();
  if (!o || !out) return set_error(HIGP_ERR_INVALID_ARG, "opts and out must be non-NULL");
  if (o->hbm_budget == 0 || o->max_active < 1 || o->max_active > 4096 || o->reserved != 0)
    return set_error(HIGP_ERR_INVALID_ARG, "bad server options");
  auto sv = std::make_unique<Server>();
  sv->opts = *o;
  sv->st = static_cast<hipStream_t>(o->stream);
  sv->num_cus = device_num_cus();
  void* h = nullptr;
  void* d = nullptr;
  const size_t sb = (size_t)o->max_active * 2 * sizeof(int);
  if (hipHostMalloc(&h, sb, hipHostMallocDefault) != hipSuccess)
    return set_error(HIGP_ERR_HIP, "pinned status allocation failed");
  if (hipMalloc(&d, sb) != hipSuccess) {
    (void)hipHostFree(h);
    return set_error(HIGP_ERR_HIP, "status allocation failed");
  }
  sv->status_h = static_cast<int*>(h);
  sv->status_d = static_cast<int*>(d);
  for (int s = o->max_active - 1; s >= 0; --s) sv->free_slots.push_back(s);
  *out = reinterpret_cast<higp_server*>(sv.release());
  return HIGP_OK;
}

int higp_server_submit(higp_server* h, const higp_request* rq, int64_t* id) {
  clear_error();
  if (!h || !rq || !id) return set_error(HIGP_ERR_INVALID_ARG, "NULL argument");
  Server& sv = *reinterpret_cast<Server*>(h);
  Problem p;
  HIGP_TRY(validate_problem(&rq->p, &p));
  if (p.prec != HIGP_FP32)
    return set_error(HIGP_ERR_UNSUPPORTED, "the server runs the FP32 form");
  if (p.d > 8) return set_error(HIGP_ERR_UNSUPPORTED, "the server takes d <= 8");
  if (!rq->y || !rq->x_out) return set_error(HIGP_ERR_INVALID_ARG, "y and x_out must be non-NULL");
  if (rq->nprobe < 0 || rq->nprobe > 31 || (rq->nprobe > 0 && (!rq->Z || rq->nsteps < 1 ||
                                                               rq->nsteps > 1024)))
    return set_error(HIGP_ERR_INVALID_ARG, "bad probe settings (0 <= nprobe <= 31)");
  if (!(rq->tol > 0.0) || rq->max_iter < 1)
    return set_error(HIGP_ERR_INVALID_ARG, "bad CG settings");
  if (rq->precond_rank < 0 || rq->precond_rank > 2048 || (rq->precond_rank > 0 && !(p.s > 0.0)))
    return set_error(HIGP_ERR_INVALID_ARG, "precond_rank must be in [0, 2048] (and s > 0 for > 0)");
  auto r = std::make_unique<Request>();
  r->id = sv.next_id++;
  r->req = *rq;
  r->p = p;
  r->N = rq->nprobe;
  r->m = rq->nprobe > 0 ? rq->nsteps : 0;
  const int rank = rq->precond_rank;
  // State (one allocation) and, with Nyström, the factor nys_build allocates.
  r->state_bytes = request_footprint(p.n, p.d, r->N, r->m, 0) +
                   (rank > 0 ? ((size_t)p.n * 8 + 255) / 256 * 256 + 256 : 0);
  r->footprint = request_footprint(p.n, p.d, r->N, r->m, rank);
  r->out.state = HIGP_REQ_QUEUED;
  if (r->footprint > sv.opts.hbm_budget)
    return set_error(HIGP_ERR_OOM, "request needs %zu bytes, more than the server budget",
                     r->footprint);
  *id = r->id;
  sv.queue.push_back(std::move(r));
  return HIGP_OK;
}

int higp_server_step(higp_server* h, int32_t* n_active, int32_t* n_queued) {
  clear_error();
  if (!h) return set_error(HIGP_ERR_INVALID_ARG, "NULL server");
  Server& sv = *reinterpret_cast<Server*>(h);
  const int rc = run_round(sv);
  if (n_active) *n_active = (int32_t)sv.active.size();
  if (n_queued) *n_queued = (int32_t)sv.queue.size();
  return rc;
}

int higp_server_status(higp_server* h, int64_t id, higp_request_status* out) {
  clear_error();
  if (!h || !out) return set_error(HIGP_ERR_INVALID_ARG, "NULL argument");
  Server& sv = *reinterpret_cast<Server*>(h);
  Request* r = find(sv, id);
  if (!r) return set_error(HIGP_ERR_INVALID_ARG, "unknown request id %lld", (long long)id);
  *out = r->out;
  out->state = r->state;
  out->rounds = r->rounds;
  return HIGP_OK;
}

int higp_server_destroy(higp_server* h) {
  clear_error();
  if (!h) return HIGP_OK;
  Server* sv = reinterpret_cast<Server*>(h);
  for (auto& r : sv->active) {
    nys_free(r->np, sv->st);
    if (r->mem) scratch_free(r->mem, sv->st);
  }
  (void)hipStreamSynchronize(sv->st);
  if (sv->status_h) (void)hipHostFree(sv->status_h);
  if (sv->status_d) (void)hipFree(sv->status_d);
  delete sv;
  return HIGP_OK;
}

}  // extern "C"
