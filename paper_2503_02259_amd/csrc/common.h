// Internal declarations shared by the translation units of libhigp.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "higp.h"

namespace higp {

// ---------------------------------------------------------------------------
// Errors: a thread-local message beside the returned code.
int set_error(int code, const char* fmt, ...);
void clear_error();

#define HIGP_HIP_TRY(expr)                                                        \
  do {                                                                            \
    hipError_t e_ = (expr);                                                       \
    if (e_ != hipSuccess)                                                         \
      return ::higp::set_error(e_ == hipErrorOutOfMemory ? HIGP_ERR_OOM : HIGP_ERR_HIP, \
                               "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                               __FILE__, __LINE__);                               \
  } while (0)

#define HIGP_TRY(expr)          \
  do {                          \
    int rc_ = (expr);           \
    if (rc_ != HIGP_OK) return rc_; \
  } while (0)

// ---------------------------------------------------------------------------
// Vector types for MFMA operands.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Validated problem description used inside the library.
struct Problem {
  int kernel;  // HIGP_GAUSSIAN / HIGP_MATERN32
  int prec;    // HIGP_FP64 / HIGP_FP32 / HIGP_BF16 / HIGP_BF16X3
  int64_t n;
  int d;
  int flags = 0;  // HIGP_FLAG_* bits
  const void* X;
  double l, f, s;
};

int validate_problem(const higp_problem* p, Problem* out);

// Scratch memory, stream-ordered.  Freed with scratch_free on the same stream.
int scratch_alloc(void** ptr, size_t bytes, hipStream_t st);
void scratch_free(void* ptr, hipStream_t st);

// ---------------------------------------------------------------------------
// MatVec launchers (kmatvec.hip).  All asynchronous on `st`.
//
// Outputs: out[0] = K̂V, out[1] = ∂K̂/∂l·V, out[2] = ∂K̂/∂f·V (each may be
// null).  V/out element type follows p.prec (double for FP64, float otherwise).
// `prec_override` >= 0 runs the MatVec in that precision instead of p.prec
// (used for the FP32 true-residual recompute of the BF16 form).
struct MatvecOut {
  void* kv = nullptr;
  void* dl = nullptr;
  void* df = nullptr;
};
int launch_kmatvec(const Problem& p, int k, const void* V, MatvecOut out, hipStream_t st,
                   int prec_override = -1);
// Rectangular Y = f²·k(Xq, X)·V: m rows (query points Xq, element type of X),
// n = p.n J points; FP64 and FP32 only.
int launch_kmatvec_cross(const Problem& p, int64_t m, const void* Xq, int k, const void* V,
                         void* Y, hipStream_t st);

// One problem of a batched FP32 MatVec (serving): prepared points (see
// prepare_points_f32), V n×k (16-byte aligned, zero up to n·k rounded up to a
// multiple of 4), output Y n×k; 1 ≤ k ≤ 32.
struct BatchMatvec {
  const float* Xp;
  const float* V;
  float* Y;
  int64_t n;
  int k, d, kernel;
  int flags;  // HIGP_FLAG_* of the problem
  double f, s;
};
size_t prepared_points_bytes(int64_t n, int d);
int prepare_points_f32(const Problem& p, float* Xp, hipStream_t st);
int launch_kmatvec_f32_batch(const BatchMatvec* jobs, int count, hipStream_t st, int num_cus);
// Symmetric-tiled FP32 square MatVec Y = K̂V (k ≤ 2 with d ≤ 4 or k = 1 with
// d ≤ 8, large n; see kmatvec_f32_sym.hip) and the test of whether it applies
// to (p, k).
bool kmatvec_f32_sym_applies(const Problem& p, int k);
int launch_kmatvec_f32_sym(const Problem& p, int k, const void* V, void* Y, hipStream_t st);
int batch_splits(int64_t n);
int device_num_cus();

// ---------------------------------------------------------------------------
// Vector kernels (blas.hip).
// Column-wise dot products of two n×k row-major blocks, accumulated in FP64
// with a fixed reduction order (deterministic).  `ta`, `tb`: 0 = double,
// 1 = float.  out: device double[k].  `work` must hold
// dot_work_doubles(n, k) doubles and `counter` one zero-initialised uint32
// (left zero on return).
size_t dot_work_doubles(int64_t n, int k);
int launch_coldot(int64_t n, int k, const void* A, int ta, const void* B, int tb, double* out,
                  double* work, unsigned* counter, hipStream_t st);

// y = cast(x) between double (0) and float (1), optional scale: y = a·x.
int launch_cast_scale(int64_t count, const void* x, int tx, void* y, int ty, double a,
                      hipStream_t st);

// PCG of higp_pcg.  With `ahist` and `bhist` (device, max_iter×k doubles,
// row j = iteration j) the step lengths α_j and direction coefficients β_j of
// every column are recorded as they are taken (β_j only for iterations that
// are followed by another); only meaningful without residual replacement.
int run_pcg(const Problem& p, int k, const void* B, void* X, const higp_pcg_opts& o,
            higp_pcg_info* info, hipStream_t st, double* ahist = nullptr,
            double* bhist = nullptr);

}  // namespace higp
