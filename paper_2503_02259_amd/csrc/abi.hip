// C ABI entry points: argument validation, error reporting, scratch memory.
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "common.h"
#include "nystrom.h"

namespace higp {

int run_slq(const Problem& p, int N, int m, const void* Z, int reorth, int precond,
            double* logdet, double* per_probe, hipStream_t st);
int run_nlml(const Problem& p, const void* y, int N, const void* Z, const higp_nlml_opts& o,
             double* loss, double* grad, double* logdet, int32_t* iters, hipStream_t st);
int run_predict(const Problem& p, const void* y, int64_t m, const void* Xq,
                const higp_predict_opts& o, void* mean, void* var, int32_t* pcg_iters,
                hipStream_t st);
int host_coldot(int64_t n, int k, const void* A, int ta, const void* B, int tb, double* out,
                hipStream_t st);

namespace {
thread_local char g_msg[512] = "";
std::atomic<bool> g_pool_ready[64];  // per device: release threshold raised
std::atomic<int> g_fail_allocs{0};   // scratch allocations the test hook makes fail
}  // namespace

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(g_msg, sizeof(g_msg), fmt, ap);
  va_end(ap);
  return code;
}

void clear_error() { g_msg[0] = '\0'; }

int validate_problem(const higp_problem* p, Problem* out) {
  if (!p) return set_error(HIGP_ERR_INVALID_ARG, "problem is NULL");
  if (p->kernel != HIGP_GAUSSIAN && p->kernel != HIGP_MATERN32)
    return set_error(HIGP_ERR_INVALID_ARG, "unknown kernel %d", p->kernel);
  if (p->prec != HIGP_FP64 && p->prec != HIGP_FP32 && p->prec != HIGP_BF16 &&
      p->prec != HIGP_BF16X3)
    return set_error(HIGP_ERR_INVALID_ARG, "unknown precision %d", p->prec);
  if (p->n < 1 || p->n > (int64_t(1) << 30))
    return set_error(HIGP_ERR_INVALID_ARG, "n = %lld out of range [1, 2^30]", (long long)p->n);
  if (p->d < 1 || p->d > HIGP_MAX_D)
    return set_error(HIGP_ERR_INVALID_ARG, "d = %d out of range [1, %d]", p->d, HIGP_MAX_D);
  if ((p->flags & ~HIGP_FLAG_NO_SYMMETRIC) != 0)
    return set_error(HIGP_ERR_INVALID_ARG, "unknown flag bits 0x%x", p->flags);
  if (!p->X) return set_error(HIGP_ERR_INVALID_ARG, "X is NULL");
  if (!(p->l > 0.0) || !std::isfinite(p->l))
    return set_error(HIGP_ERR_INVALID_ARG, "l must be finite and > 0");
  if (!(p->s >= 0.0) || !std::isfinite(p->s))
    return set_error(HIGP_ERR_INVALID_ARG, "s must be finite and >= 0");
  if (!std::isfinite(p->f)) return set_error(HIGP_ERR_INVALID_ARG, "f must be finite");
  out->kernel = p->kernel;
  out->prec = p->prec;
  out->n = p->n;
  out->d = p->d;
  out->flags = p->flags;
  out->X = p->X;
  out->l = p->l;
  out->f = p->f;
  out->s = p->s;
  return HIGP_OK;
}

int scratch_alloc(void** ptr, size_t bytes, hipStream_t st) {
  int dev = 0;
  HIGP_HIP_TRY(hipGetDevice(&dev));
  if (dev >= 0 && dev < 64 && !g_pool_ready[dev].load(std::memory_order_acquire)) {
    // Keep freed stream-ordered memory in the pool between calls instead of
    // returning it to the driver at every synchronisation.
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
      uint64_t thr = UINT64_MAX;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
    }
    g_pool_ready[dev].store(true, std::memory_order_release);
  }
  // Allocations the test hook makes fail (higp_debug_fail_allocs).
  for (int c = g_fail_allocs.load(); c > 0;)
    if (g_fail_allocs.compare_exchange_weak(c, c - 1)) {
      *ptr = nullptr;
      return set_error(HIGP_ERR_OOM, "scratch allocation of %zu bytes failed (injected)", bytes);
    }
  hipError_t e = hipMallocAsync(ptr, bytes ? bytes : 256, st);
  if (e != hipSuccess) {
    *ptr = nullptr;
    (void)hipGetLastError();
    return set_error(e == hipErrorOutOfMemory ? HIGP_ERR_OOM : HIGP_ERR_HIP,
                     "scratch allocation of %zu bytes failed: %s", bytes, hipGetErrorString(e));
  }
  return HIGP_OK;
}

void scratch_free(void* ptr, hipStream_t st) {
  if (ptr) (void)hipFreeAsync(ptr, st);
}

namespace {

size_t elem_size(int prec) { return prec == HIGP_FP64 ? 8 : 4; }

// [a, a + abytes) ∩ [b, b + bbytes) ≠ ∅
bool overlaps(const void* a, size_t abytes, const void* b, size_t bbytes) {
  if (!a || !b) return false;
  const char* pa = static_cast<const char*>(a);
  const char* pb = static_cast<const char*>(b);
  return pa < pb + bbytes && pb < pa + abytes;
}

bool overlaps(const void* a, const void* b, size_t bytes) { return overlaps(a, bytes, b, bytes); }

}  // namespace
}  // namespace higp

using namespace higp;

extern "C" {

int higp_version(void) { return 200; }

int higp_debug_fail_allocs(int32_t count) {
  if (count < 0) return set_error(HIGP_ERR_INVALID_ARG, "count must be >= 0");
  g_fail_allocs.store(count);
  return HIGP_OK;
}

const char* higp_error_string(int code) {
  switch (code) {
    case HIGP_OK: return "ok";
    case HIGP_ERR_INVALID_ARG: return "invalid argument";
    case HIGP_ERR_UNSUPPORTED: return "unsupported";
    case HIGP_ERR_OOM: return "out of device memory";
    case HIGP_ERR_HIP: return "HIP runtime error";
    default: return "unknown error code";
  }
}

const char* higp_last_error(void) { return g_msg; }

int higp_kmatvec(const higp_problem* hp, int32_t k, const void* V, void* Y, void* stream) {
  clear_error();
  Problem p;
  HIGP_TRY(validate_problem(hp, &p));
  if (k < 1 || k > HIGP_MAX_K)
    return set_error(HIGP_ERR_INVALID_ARG, "k = %d out of range [1, %d]", k, HIGP_MAX_K);
  if (!V || !Y) return set_error(HIGP_ERR_INVALID_ARG, "V and Y must be non-NULL");
  const size_t bytes = (size_t)p.n * k * elem_size(p.prec);
  if (overlaps(V, Y, bytes)) return set_error(HIGP_ERR_INVALID_ARG, "Y overlaps V");
  MatvecOut o;
  o.kv = Y;
  return launch_kmatvec(p, k, V, o, static_cast<hipStream_t>(stream));
}

int higp_kmatvec_grad(const higp_problem* hp, int32_t k, const void* V, void* KV, void* dL,
                      void* dF, void* dS, void* stream) {
  clear_error();
  Problem p;
  HIGP_TRY(validate_problem(hp, &p));
  if (k < 1 || k > HIGP_MAX_K)
    return set_error(HIGP_ERR_INVALID_ARG, "k = %d out of range [1, %d]", k, HIGP_MAX_K);
  if (!V) return set_error(HIGP_ERR_INVALID_ARG, "V must be non-NULL");
  if (!KV && !dL && !dF && !dS)
    return set_error(HIGP_ERR_INVALID_ARG, "at least one output must be non-NULL");
  const size_t bytes = (size_t)p.n * k * elem_size(p.prec);
  void* outs[4] = {KV, dL, dF, dS};
  for (int i = 0; i < 4; ++i) {
    if (overlaps(V, outs[i], bytes)) return set_error(HIGP_ERR_INVALID_ARG, "an output overlaps V");
    for (int j = i + 1; j < 4; ++j)
      if (overlaps(outs[i], outs[j], bytes))
        return set_error(HIGP_ERR_INVALID_ARG, "two outputs overlap");
  }
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dS) HIGP_HIP_TRY(hipMemcpyAsync(dS, V, bytes, hipMemcpyDeviceToDevice, st));
  if (!KV && !dL && !dF) return HIGP_OK;
  MatvecOut o;
  o.kv = KV;
  o.dl = dL;
  o.df = dF;
  if (!dL && !dF) return launch_kmatvec(p, k, V, o, st);
  return launch_kmatvec(p, k, V, o, st);
}

int higp_pcg(const higp_problem* hp, int32_t k, const void* B, void* X, const higp_pcg_opts* o,
             higp_pcg_info* info, void* stream) {
  clear_error();
  Problem p;
  HIGP_TRY(validate_problem(hp, &p));
  if (k < 1 || k > HIGP_MAX_K)
    return set_error(HIGP_ERR_INVALID_ARG, "k = %d out of range [1, %d]", k, HIGP_MAX_K);
  if (!B || !X || !o) return set_error(HIGP_ERR_INVALID_ARG, "B, X and opts must be non-NULL");
  if (!(o->tol > 0.0)) return set_error(HIGP_ERR_INVALID_ARG, "tol must be > 0");
  if (o->max_iter < 1) return set_error(HIGP_ERR_INVALID_ARG, "max_iter must be >= 1");
  if (o->precond < 0 || o->precond > 2)
    return set_error(HIGP_ERR_INVALID_ARG, "precond must be 0, 1 or 2");
  if (o->rank < 0 || o->rank > 2048)
    return set_error(HIGP_ERR_INVALID_ARG, "rank must be in [0, 2048]");
  if (o->precond == 2 && !(p.s > 0.0))
    return set_error(HIGP_ERR_INVALID_ARG, "the Nyström preconditioner needs s > 0");
  if (o->refine_every < 0 || o->check_every < 0 || (o->use_x0 != 0 && o->use_x0 != 1))
    return set_error(HIGP_ERR_INVALID_ARG, "bad option value");
  if (o->refine_prec != HIGP_FP64 && o->refine_prec != HIGP_FP32)
    return set_error(HIGP_ERR_INVALID_ARG, "refine_prec must be HIGP_FP64 or HIGP_FP32");
  const size_t bytes = (size_t)p.n * k * elem_size(p.prec);
  if (overlaps(B, X, bytes)) return set_error(HIGP_ERR_INVALID_ARG, "X overlaps B");
  if (o->x_fp64 && (overlaps(o->x_fp64, (size_t)p.n * k * 8, B, bytes) ||
                    overlaps(o->x_fp64, (size_t)p.n * k * 8, X, bytes)))
    return set_error(HIGP_ERR_INVALID_ARG, "x_fp64 overlaps B or Xsol");
  return run_pcg(p, k, B, X, *o, info, static_cast<hipStream_t>(stream));
}

int higp_slq_logdet(const higp_problem* hp, int32_t nprobe, int32_t nsteps, const void* Z,
                    uint64_t seed, int32_t reorth, int32_t precond, double* logdet,
                    double* per_probe, void* stream) {
  (void)seed;
  clear_error();
  Problem p;
  HIGP_TRY(validate_problem(hp, &p));
  if (nprobe < 1 || nprobe > HIGP_MAX_K)
    return set_error(HIGP_ERR_INVALID_ARG, "nprobe = %d out of range [1, %d]", nprobe, HIGP_MAX_K);
  if (nsteps < 1 || nsteps > 1024)
    return set_error(HIGP_ERR_INVALID_ARG, "nsteps = %d out of range [1, 1024]", nsteps);
  if ((reorth != 0 && reorth != 1) || (precond != 0 && precond != 1))
    return set_error(HIGP_ERR_INVALID_ARG, "reorth and precond must be 0 or 1");
  if (!logdet) return set_error(HIGP_ERR_INVALID_ARG, "logdet must be non-NULL");
  if (!Z) return set_error(HIGP_ERR_UNSUPPORTED, "Z = NULL (device-generated probes) is not supported");
  return run_slq(p, nprobe, nsteps, Z, reorth, precond, logdet, per_probe,
                 static_cast<hipStream_t>(stream));
}

int higp_coldot(int64_t n, int32_t k, int32_t prec_a, const void* A, int32_t prec_b,
                const void* B, double* out, void* stream) {
  clear_error();
  if (n < 1 || n > (int64_t(1) << 30))
    return set_error(HIGP_ERR_INVALID_ARG, "n = %lld out of range", (long long)n);
  if (k < 1 || k > HIGP_MAX_K)
    return set_error(HIGP_ERR_INVALID_ARG, "k = %d out of range [1, %d]", k, HIGP_MAX_K);
  for (int pr : {prec_a, prec_b})
    if (pr != HIGP_FP64 && pr != HIGP_FP32 && pr != HIGP_BF16 && pr != HIGP_BF16X3)
      return set_error(HIGP_ERR_INVALID_ARG, "unknown precision %d", pr);
  if (!A || !B || !out) return set_error(HIGP_ERR_INVALID_ARG, "A, B and out must be non-NULL");
  return host_coldot(n, k, A, prec_a == HIGP_FP64 ? 0 : 1, B, prec_b == HIGP_FP64 ? 0 : 1, out,
                     static_cast<hipStream_t>(stream));
}

int higp_nlml(const higp_problem* hp, const void* y, int32_t nprobe, const void* Z,
              const higp_nlml_opts* o, double* loss, double* grad, double* logdet,
              int32_t* pcg_iters, void* stream) {
  clear_error();
  Problem p;
  HIGP_TRY(validate_problem(hp, &p));
  if (nprobe < 1 || nprobe > HIGP_MAX_K - 1)
    return set_error(HIGP_ERR_INVALID_ARG, "nprobe = %d out of range [1, %d]", nprobe,
                     HIGP_MAX_K - 1);
  if (!y || !Z || !o || !loss || !grad)
    return set_error(HIGP_ERR_INVALID_ARG, "y, Z, opts, loss and grad must be non-NULL");
  if (!(o->tol > 0.0) || o->max_iter < 1 || (o->precond != 0 && o->precond != 1) ||
      o->refine_every < 0 || o->nsteps < 1 || o->nsteps > 1024 ||
      (o->reorth != 0 && o->reorth != 1) || o->logdet_mode < 0 || o->logdet_mode > 1 ||
      o->trace_mode < 0 || o->trace_mode > 1 || o->reserved != 0)
    return set_error(HIGP_ERR_INVALID_ARG, "bad option value");
  if (o->logdet_mode == 1 && o->refine_every != 0)
    return set_error(HIGP_ERR_INVALID_ARG,
                     "logdet_mode 1 reads the PCG coefficients and needs refine_every = 0");
  if (o->logdet_mode == 1 && o->max_iter > 100000)
    return set_error(HIGP_ERR_INVALID_ARG, "logdet_mode 1 takes max_iter ≤ 100000");
  if (o->trace_mode == 1 && (nprobe < 2 || nprobe > 42 || o->logdet_mode != 0))
    return set_error(HIGP_ERR_INVALID_ARG,
                     "trace_mode 1 (Hutch++) needs 2 ≤ nprobe ≤ 42 and logdet_mode 0");
  return run_nlml(p, y, nprobe, Z, *o, loss, grad, logdet, pcg_iters,
                  static_cast<hipStream_t>(stream));
}

int higp_fps_landmarks(const higp_problem* hp, int32_t rank, int32_t* idx, void* stream) {
  clear_error();
  Problem p;
  HIGP_TRY(validate_problem(hp, &p));
  if (p.prec != HIGP_FP64 && p.prec != HIGP_FP32 && p.prec != HIGP_BF16 && p.prec != HIGP_BF16X3)
    return set_error(HIGP_ERR_INVALID_ARG, "unknown precision");
  if (rank < 1 || rank > 2048) return set_error(HIGP_ERR_INVALID_ARG, "rank must be in [1, 2048]");
  if (!idx) return set_error(HIGP_ERR_INVALID_ARG, "idx must be non-NULL");
  return fps_landmarks(p, rank, idx, static_cast<hipStream_t>(stream));
}

int higp_kmatvec_cross(const higp_problem* hp, int64_t m, const void* Xq, int32_t k,
                       const void* V, void* Y, void* stream) {
  clear_error();
  Problem p;
  HIGP_TRY(validate_problem(hp, &p));
  if (p.prec != HIGP_FP64 && p.prec != HIGP_FP32)
    return set_error(HIGP_ERR_UNSUPPORTED, "the rectangular MatVec runs in FP64 or FP32");
  if (m < 1 || m > (int64_t(1) << 31))
    return set_error(HIGP_ERR_INVALID_ARG, "m = %lld out of range", (long long)m);
  if (k < 1 || k > HIGP_MAX_K)
    return set_error(HIGP_ERR_INVALID_ARG, "k = %d out of range [1, %d]", k, HIGP_MAX_K);
  if (!Xq || !V || !Y) return set_error(HIGP_ERR_INVALID_ARG, "Xq, V and Y must be non-NULL");
  const size_t es = elem_size(p.prec);
  const size_t ybytes = (size_t)m * k * es;
  if (overlaps(Y, ybytes, V, (size_t)p.n * k * es) || overlaps(Y, ybytes, Xq, (size_t)m * p.d * es))
    return set_error(HIGP_ERR_INVALID_ARG, "Y overlaps V or Xq");
  return launch_kmatvec_cross(p, m, Xq, k, V, Y, static_cast<hipStream_t>(stream));
}

int higp_gpr_predict(const higp_problem* hp, const void* y, int64_t m, const void* Xq,
                     const higp_predict_opts* o, void* mean, void* var, int32_t* pcg_iters,
                     void* stream) {
  clear_error();
  Problem p;
  HIGP_TRY(validate_problem(hp, &p));
  if (p.prec != HIGP_FP64 && p.prec != HIGP_FP32)
    return set_error(HIGP_ERR_UNSUPPORTED, "prediction runs in FP64 or FP32");
  if (m < 1 || m > (int64_t(1) << 31))
    return set_error(HIGP_ERR_INVALID_ARG, "m = %lld out of range", (long long)m);
  if (!y || !Xq || !o || !mean)
    return set_error(HIGP_ERR_INVALID_ARG, "y, Xq, opts and mean must be non-NULL");
  if (!(o->tol > 0.0) || o->max_iter < 1 || o->precond < 0 || o->precond > 2 ||
      (o->precond == 2 && !(p.s > 0.0)) || (o->want_var != 0 && o->want_var != 1) ||
      o->rank < 0 || o->rank > 2048 || (o->rank != 0 && o->precond != 2))
    return set_error(HIGP_ERR_INVALID_ARG, "bad option value");
  if ((o->want_var != 0) != (var != nullptr))
    return set_error(HIGP_ERR_INVALID_ARG, "var must be non-NULL exactly when want_var is 1");
  const size_t es = elem_size(p.prec);
  const size_t mbytes = (size_t)m * es;
  if (overlaps(mean, mbytes, y, (size_t)p.n * es) || overlaps(mean, mbytes, Xq, mbytes * p.d) ||
      (var && (overlaps(var, mbytes, mean, mbytes) || overlaps(var, mbytes, y, (size_t)p.n * es) ||
               overlaps(var, mbytes, Xq, mbytes * p.d))))
    return set_error(HIGP_ERR_INVALID_ARG, "an output overlaps an input or the other output");
  return run_predict(p, y, m, Xq, *o, mean, var, pcg_iters, static_cast<hipStream_t>(stream));
}

}  // extern "C"
