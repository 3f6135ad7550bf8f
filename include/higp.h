/*
 * higp.h — C ABI of the MI355X (gfx950) on-the-fly kernel MatVec engine.
 *
 * The operations follow the statement of the Gaussian-process problem in
 * HiGP (Huang, Xu, Xi, Chow; arXiv 2503.02259), section "Gaussian
 * Processes": training points X ∈ R^{n×d}, parameters Θ = (s, f, l) (noise
 * level s, scale f, kernel parameter l) and the regularised kernel matrix
 *
 *        K̂ = f² · k(X, X; l) + s · I.
 *
 * The kernels k are the Gaussian (RBF) and Matérn-3/2 kernels named in the
 * paper's Listing 1 and Tables 1-2, in their textbook form with a scalar,
 * isotropic length-scale l and r = ‖x_i − x_j‖₂:
 *
 *        Gaussian     k(r) = exp(−r² / (2 l²))
 *        Matérn-3/2   k(r) = (1 + √3 r / l) · exp(−√3 r / l)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Pointers documented as "device" are HIP device memory owned by the
 *    caller; the library never frees or keeps them after the call returns.
 *    Pointers documented as "host" are ordinary host memory.
 *  - Matrices are row-major: X is n×d, and every block of vectors (V, Y, B,
 *    Xsol, Z) is n×k with element (i, c) at offset i·k + c.
 *  - Element type: double for HIGP_FP64; float for HIGP_FP32, HIGP_BF16 and
 *    HIGP_BF16X3 (in the BF16 forms only the kernel tile and V are rounded to
 *    bfloat16, inside the kernel, and products are accumulated in FP32).
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is ordered
 *    on that stream.  higp_kmatvec and higp_kmatvec_grad only enqueue work and
 *    return; higp_pcg and higp_slq_logdet synchronise the stream before they
 *    fill their host outputs.
 *  - Calls are stateless and reentrant (the paper's Python interfaces are
 *    stateless, "Design and Implementation"); any scratch memory is
 *    allocated stream-ordered and released before the call returns.
 *  - Return value: HIGP_OK (0) on success, a negative HIGP_ERR_* code
 *    otherwise; higp_last_error() then returns a message for the calling
 *    thread.  Invalid arguments are detected before any work is enqueued.
 */
#ifndef HIGP_H
#define HIGP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HIGP_OK 0
#define HIGP_ERR_INVALID_ARG (-1) /* a size, pointer or parameter is out of range */
#define HIGP_ERR_UNSUPPORTED (-2) /* a valid combination the library does not implement */
#define HIGP_ERR_OOM (-3)         /* device scratch allocation failed */
#define HIGP_ERR_HIP (-4)         /* a HIP runtime call failed (message has the detail) */

#define HIGP_MAX_D 32 /* largest point dimension d (the BF16 forms and the
                         server take d ≤ 8; the paper's on-the-fly runs use 20) */
#define HIGP_MAX_K 64 /* largest number of vectors k per call */

typedef enum { HIGP_GAUSSIAN = 0, HIGP_MATERN32 = 1 } higp_kernel;

typedef enum {
  HIGP_FP64 = 0, /* everything in double */
  HIGP_FP32 = 1, /* distances, kernel values and the K-tile×V product in float */
  HIGP_BF16 = 2, /* kernel tile and V rounded to bfloat16, FP32 accumulation */
  HIGP_BF16X3 = 3 /* split BF16: kernel tile and V each as hi + lo bfloat16 pairs
                     (hi = RNE(x), lo = RNE(x − hi)); the product keeps the three
                     terms K_hi·V_hi + K_hi·V_lo + K_lo·V_hi, FP32 accumulation;
                     relative error of order 2⁻¹⁶ instead of 2⁻⁸ */
} higp_precision;

/* Problem flags.
 * HIGP_FLAG_NO_SYMMETRIC: the FP32 square MatVec with k ≤ 2 vectors and
 *   d ≤ 4 (or k = 1 and d ≤ 8) at 32768 ≤ n (up to about 4·10⁵ for k = 2,
 *   5.6·10⁵ for k = 1, where its per-block-pair slots reach 2 GiB)
 *   normally evaluates each
 *   kernel value of a pair of
 *   point blocks once and uses it for both output blocks (K̂ is symmetric:
 *   about n²/2 kernel values instead of n²).  This flag selects the
 *   full-block form instead, whose summation order is that of the wider
 *   MatVecs (both forms are deterministic).                                */
#define HIGP_FLAG_NO_SYMMETRIC 1

/* One GP problem: K̂ = f²·k(X, X; l) + s·I.
 * X: device, n×d row-major (double for HIGP_FP64, float otherwise).
 * Valid: n ≥ 1, 1 ≤ d ≤ HIGP_MAX_D, l > 0, s ≥ 0, f finite.               */
typedef struct {
  int32_t kernel; /* higp_kernel */
  int32_t prec;   /* higp_precision */
  int64_t n;
  int32_t d;
  int32_t flags;  /* 0 or HIGP_FLAG_* bits */
  const void* X;
  double l, f, s;
} higp_problem;

/* Y = K̂·V — the on-the-fly kernel MatVec ("Statement of Need": small kernel
 * matrix blocks are formed, used in the MatVec and discarded).
 * V: device n×k, Y: device n×k (must not overlap V); 1 ≤ k ≤ HIGP_MAX_K.
 * K̂ is never stored.  Asynchronous on `stream`.                            */
int higp_kmatvec(const higp_problem* p, int32_t k, const void* V, void* Y,
                 void* stream);

/* Derivative MatVecs ∂K̂/∂θ·V for θ ∈ {l, f, s} (the quantities inside the
 * gradient of the negative log marginal likelihood, "Gaussian Processes"),
 * with ∂K̂/∂l = f²·∂k/∂l, ∂K̂/∂f = 2f·k(X, X; l), ∂K̂/∂s = I.
 * Each output is device n×k and may be NULL (not computed); KV receives
 * K̂·V from the same kernel tiles.  At least one output must be non-NULL and
 * none may overlap V.  Asynchronous on `stream`.                           */
int higp_kmatvec_grad(const higp_problem* p, int32_t k, const void* V,
                      void* KV, void* dL_V, void* dF_V, void* dS_V,
                      void* stream);

/* Rectangular on-the-fly MatVec Y = f²·k(Xq, X; l)·V, the product prediction
 * needs (`gpr_prediction` in Listing 1), formed block by block like K̂·V.
 * p: the training problem — X device n×d; its s is not used; prec HIGP_FP64
 *    or HIGP_FP32 (the BF16 forms return HIGP_ERR_UNSUPPORTED).
 * m: number of query points (1 ≤ m ≤ 2^31); Xq: device m×d, same element
 *    type as X.  V: device n×k; Y: device m×k, must not overlap V or Xq;
 *    1 ≤ k ≤ HIGP_MAX_K.  Asynchronous on `stream`.                         */
int higp_kmatvec_cross(const higp_problem* p, int64_t m, const void* Xq,
                       int32_t k, const void* V, void* Y, void* stream);

/* Options of higp_pcg.                                                     */
typedef struct {
  double tol;           /* stop column c when ‖r_c‖₂ ≤ tol·‖b_c‖₂ (recursive r); > 0 */
  int32_t max_iter;     /* cap on iterations per column; ≥ 1 */
  int32_t precond;      /* 0 = none, 1 = Jacobi (M = diag K̂), 2 = Nyström: the
                           low-rank approximation the paper's AFN preconditioner
                           is built on ("Statement of Need"), in its generic
                           form M = s·I + f²·K_nr·K_rr⁻¹·K_rn on `rank` landmarks
                           chosen by farthest-point sampling, applied by the
                           Woodbury identity (needs s > 0) */
  int32_t refine_every; /* R > 0: after every R-th iteration replace the recursive
                           residual by b − K̂x computed with the iterate x (FP64)
                           and a MatVec in precision refine_prec; with
                           HIGP_FP64 a column then stops on tol only at such an
                           iteration, so the tolerance holds for the recomputed
                           residual (at most R − 1 extra iterations); 0 = off */
  int32_t use_x0;       /* 1: Xsol holds the initial guess on entry; 0: x0 = 0 */
  int32_t check_every;  /* host convergence poll period (≥ 1; 0 = library default).
                           Converged columns are frozen on the device, so this
                           changes only when the call returns, never the result. */
  int32_t refine_prec;  /* precision of the replacement MatVec: HIGP_FP64 (x and
                           the points widened to double; the residual is then
                           accurate to FP64, so the tolerance holds for the true
                           residual) or HIGP_FP32 (x rounded to float: cheaper,
                           accurate only to the FP32 floor u·‖|K̂||x|‖/‖b‖; a
                           column takes no further replacements once one fails
                           to lower its residual, and then converges on the
                           recursive residual like the unrefined form).
                           Any column whose residual becomes non-finite or
                           exceeds 1e8·‖b‖ stops as diverged (converged = 0). */
  void* x_fp64;         /* optional (NULL = unused): device n×k double buffer that
                           receives the FP64 iterate, which is more accurate than
                           Xsol when the problem is FP32/BF16; must not overlap B
                           or Xsol */
  int32_t rank;         /* Nyström landmarks (precond 2): 0 = min(n, 1024), else
                           1 … 2048 (clamped to n); ignored otherwise.  Building
                           costs n·rank² flops on the GPU and rank³/2 on the host;
                           each application 4·n·rank·k flops */
} higp_pcg_opts;

/* Per-column results of higp_pcg (host arrays of length k, caller-owned). */
typedef struct {
  int32_t* iters;     /* iterations taken */
  double* relres;     /* final recursive relative residual ‖r‖/‖b‖ */
  int32_t* converged; /* 1 if relres ≤ tol, else 0 */
} higp_pcg_info;

/* Solve K̂·Xsol = B by preconditioned CG (the paper approximates K̂⁻¹y with
 * PCG, Saad 2003, "Gaussian Processes"), for k right-hand sides at once:
 * k independent CG recurrences sharing one k-column MatVec per iteration.
 * CG scalars are FP64; the iterate x and residual r are kept in FP64 on the
 * device; the search direction enters the MatVec in the problem's precision.
 * B: device n×k; Xsol: device n×k (initial guess on entry if use_x0).
 * Not converging within max_iter is not an error (converged[c] = 0).
 * Synchronises `stream` before returning.                                  */
int higp_pcg(const higp_problem* p, int32_t k, const void* B, void* Xsol,
             const higp_pcg_opts* opts, higp_pcg_info* info, void* stream);

/* log|K̂| by eq. (1) with M = I (precond 0) or M = diag(K̂) (precond 1), its
 * second term estimated by stochastic Lanczos quadrature (Ubaru et al. 2017,
 * cited in "Gaussian Processes"): for each probe z, nsteps Lanczos steps on
 * M^{-1/2}K̂M^{-1/2} from z/‖z‖ (full reorthogonalisation when reorth = 1),
 * T = SΘSᵀ in FP64 on the host, and ‖z‖²·Σ_k S_{1k}²·log θ_k.
 * A probe stops early (shorter T) when β_j ≤ 1e-12·max_{i≤j}|α_i|.
 * Z: device n×nprobe probe block in the problem's precision (normally ±1).
 *    Z = NULL is not supported (HIGP_ERR_UNSUPPORTED); pass
 *    the probes explicitly.  `seed` is reserved and ignored.
 * logdet: host, receives log|M| + mean of the probes' quadratures.
 * per_probe: host array of nprobe (may be NULL): log|M| + each probe's value.
 * 1 ≤ nprobe ≤ HIGP_MAX_K, 1 ≤ nsteps ≤ 1024.  Synchronises `stream`.      */
int higp_slq_logdet(const higp_problem* p, int32_t nprobe, int32_t nsteps,
                    const void* Z, uint64_t seed, int32_t reorth,
                    int32_t precond, double* logdet, double* per_probe,
                    void* stream);

/* Column dot products out[c] = Σ_i A[i,c]·B[i,c] of two device n×k blocks,
 * accumulated in FP64 in a fixed order (bitwise reproducible).  prec_a and
 * prec_b give each block's element type (HIGP_FP64 = double, otherwise
 * float).  out: host array of k doubles.  1 ≤ k ≤ HIGP_MAX_K, n ≥ 1.
 * Synchronises `stream`.  (The inner products of the gradient of the
 * negative log marginal likelihood, "Gaussian Processes".)               */
int higp_coldot(int64_t n, int32_t k, int32_t prec_a, const void* A, int32_t prec_b,
                const void* B, double* out, void* stream);

/* Options of higp_nlml.                                                    */
typedef struct {
  double tol;           /* PCG tolerance on [y | Z] (tracked residual) */
  int32_t max_iter;     /* PCG iteration cap */
  int32_t precond;      /* 0 = none, 1 = Jacobi (also used for eq. (1) and (2)) */
  int32_t refine_every; /* PCG residual replacement period (0 = off), FP64 MatVec */
  int32_t nsteps;       /* Lanczos steps of SLQ (logdet_mode 0) */
  int32_t reorth;       /* 1 = full reorthogonalisation in SLQ (logdet_mode 0) */
  int32_t logdet_mode;  /* 0 = SLQ: a Lanczos pass over Z after the solve;
                           1 = the tridiagonals PCG builds on the Z columns
                           (CG–Lanczos correspondence, Saad 2003 §6.7.3, as
                           GPyTorch's mBCG): no Lanczos pass, no
                           reorthogonalisation; needs refine_every = 0 */
  int32_t trace_mode;   /* 0 = Hutchinson over all of Z; 1 = Hutch++ (Meyer et
                           al. 2021, cited with eq. (2)): sketch S = the first
                           ⌊N/2⌋ columns of Z, Hutchinson probes G = the rest;
                           needs 2 ≤ N ≤ 42 and logdet_mode 0 */
  int32_t reserved;     /* must be 0 */
} higp_nlml_opts;

/* Negative log marginal likelihood L(Θ) = ½(yᵀK̂⁻¹y + log|K̂| + n·log 2π) and
 * its gradient ∂L/∂θ = ½(−yᵀK̂⁻¹(∂K̂/∂θ)K̂⁻¹y + tr(K̂⁻¹ ∂K̂/∂θ)) for
 * θ = (l, f, s) ("Gaussian Processes"), estimated as in the paper:
 *   K̂⁻¹y and K̂⁻¹Z by PCG on [y | Z] (one MatVec of 1 + nprobe columns per
 *   iteration); log|K̂| by eq. (1) with SLQ over the probes Z; the trace by
 *   eq. (2) with M = diag(K̂) and the Hutchinson estimator
 *   (1/N) Σ_i [(K̂⁻¹z_i)ᵀ(∂K̂/∂θ z_i) − z_iᵀM⁻¹(∂M/∂θ)z_i]; the products
 *   ∂K̂/∂θ·[K̂⁻¹y | Z] by one fused derivative MatVec.
 * y: device n; Z: device n×nprobe (both in the problem's element type);
 * 1 ≤ nprobe ≤ HIGP_MAX_K − 1.  loss: host double; grad: host double[3]
 * (∂L/∂l, ∂L/∂f, ∂L/∂s); logdet: host double or NULL (the SLQ estimate);
 * pcg_iters: host int32 or NULL (largest PCG iteration count).
 * Synchronises `stream`.                                                  */
int higp_nlml(const higp_problem* p, const void* y, int32_t nprobe, const void* Z,
              const higp_nlml_opts* opts, double* loss, double* grad, double* logdet,
              int32_t* pcg_iters, void* stream);

/* ------------------------------------------------------------------------
 * Continuous-batching serving of independent GP solves (FP32 form).
 *
 * A request is one problem K̂ = f²·k(X,X;l) + s·I with targets y and probes
 * Z; the server computes x = K̂⁻¹y by Jacobi-preconditioned CG (tolerance on
 * the recursive residual, as higp_pcg) and log|K̂| by eq. (1) with SLQ over
 * the probes (full reorthogonalisation, as higp_slq_logdet) — the two terms of
 * L(Θ) ("Gaussian Processes").  Requests wait in a FIFO queue and are admitted
 * while a slot is free and their device state fits in hbm_budget; admitted
 * requests keep their state resident.  Each higp_server_step runs one round:
 * admissions, ONE batched MatVec launch for every active request (the CG
 * column and the live Lanczos columns of a request, k ≤ 32), every request's
 * CG and Lanczos updates, and retirement of finished requests.  A request's
 * arithmetic depends only on the request, so its results are bitwise equal
 * alone and in any mix.  All work is ordered on opts.stream; higp_server_step
 * synchronises it.  A server is not thread-safe.
 * ------------------------------------------------------------------------ */
/* Landmark points of the Nyström preconditioner (precond 2 of higp_pcg):
 * min(rank, n) indices into X chosen by farthest-point sampling — the first
 * is 0, each next one is the point whose smallest squared distance (FP64,
 * coordinates summed in order) to the landmarks so far is largest, lowest
 * index on ties.  AFN, the paper's preconditioner, builds its Nyström part
 * on such selected points ("Statement of Need").
 * p: X device n×d (FP64 or FP32 coordinates; l, f, s unused).
 * idx: host array of min(rank, n) int32.  1 ≤ rank ≤ 2048.  Synchronises. */
int higp_fps_landmarks(const higp_problem* p, int32_t rank, int32_t* idx, void* stream);

/* Options of higp_gpr_predict.                                             */
typedef struct {
  double tol;        /* PCG tolerance of the solves with K̂ (> 0) */
  int32_t max_iter;  /* PCG cap per solve (≥ 1; the paper's prediction runs use 50) */
  int32_t precond;   /* 0 = none, 1 = Jacobi, 2 = Nyström */
  int32_t want_var;  /* 1: also the latent predictive variance; 0: mean only */
  int32_t rank;      /* Nyström landmarks, 0..2048 (0: min(n, 1024)); must be 0 unless
                        precond is 2 (the paper's prediction runs use rank 100) */
} higp_predict_opts;

/* GP regression prediction (`gpr_prediction` in Listing 1), the textbook GP
 * posterior with the trained Θ = (l, f, s) of p:
 *   mean_q = f²·k(x_q, X)·α,  α = K̂⁻¹y (PCG),
 *   var_q  = f² − k*_qᵀK̂⁻¹k*_q with k*_q = f²·k(X, x_q) — the variance of the
 *            latent function (add s for a noisy observation); a value the
 *            solver tolerance leaves below 0 is reported as 0.
 * p: prec HIGP_FP64 or HIGP_FP32.  y: device n; Xq: device m×d (element type
 * of X); mean: device m; var: device m, non-NULL iff want_var (one PCG solve
 * with up to 64 right-hand sides per 64 query points).  pcg_iters (host,
 * nullable): iterations of the α solve.  Scratch is allocated and released
 * inside; synchronises `stream` before returning.                          */
int higp_gpr_predict(const higp_problem* p, const void* y, int64_t m,
                     const void* Xq, const higp_predict_opts* opts, void* mean,
                     void* var, int32_t* pcg_iters, void* stream);

typedef struct higp_server higp_server;  /* opaque */

typedef struct {
  uint64_t hbm_budget; /* bytes of device memory the server may hold for request state */
  int32_t max_active;  /* concurrently active requests, 1..4096 */
  int32_t reserved;    /* must be 0 */
  void* stream;        /* hipStream_t (NULL = default stream) */
} higp_server_opts;

typedef struct {
  higp_problem p;      /* prec must be HIGP_FP32; X device n×d float */
  const void* y;       /* device n float */
  const void* Z;       /* device n×nprobe float (±1 probes), NULL if nprobe = 0 */
  int32_t nprobe;      /* 0..31 */
  int32_t nsteps;      /* Lanczos steps (1..1024) when nprobe > 0 */
  double tol;          /* CG tolerance (> 0) */
  int32_t max_iter;    /* CG iteration cap (≥ 1) */
  int32_t precond_rank; /* 0: Jacobi; 1 … 2048: the Nyström preconditioner of
                           higp_pcg (precond 2) with that many landmarks (clamped
                           to n; needs s > 0), built when the request is admitted */
  void* x_out;         /* device n float: receives x = K̂⁻¹y when the request is done */
} higp_request;

#define HIGP_REQ_QUEUED 0
#define HIGP_REQ_ACTIVE 1
#define HIGP_REQ_DONE 2
#define HIGP_REQ_FAILED 3

typedef struct {
  int32_t state;         /* HIGP_REQ_* */
  int32_t iters;         /* CG iterations */
  double relres;         /* final recursive relative residual */
  int32_t converged;     /* relres ≤ tol */
  int32_t lanczos_steps; /* shortest Lanczos run over the probes */
  double logdet;         /* SLQ estimate of log|K̂| (NaN if nprobe = 0) */
  int32_t rounds;        /* server rounds the request took part in */
  int32_t reserved;
} higp_request_status;

/* Device bytes the server reserves for a request (state, vectors, Lanczos
 * basis, batch partials, and the Nyström factor when precond_rank > 0).
 * Host only; 0 for invalid sizes.                                          */
uint64_t higp_request_footprint(int64_t n, int32_t d, int32_t nprobe, int32_t nsteps,
                                int32_t precond_rank);

int higp_server_create(const higp_server_opts* opts, higp_server** server);
/* Queue a request; the caller's buffers (X, y, Z, x_out) must stay valid until
 * the request is done.  HIGP_ERR_OOM if it can never fit in the budget.      */
int higp_server_submit(higp_server* server, const higp_request* req, int64_t* id);
/* One round (see above); returns the numbers of active and queued requests. */
int higp_server_step(higp_server* server, int32_t* n_active, int32_t* n_queued);
int higp_server_status(higp_server* server, int64_t id, higp_request_status* status);
/* Frees all server memory (active requests are abandoned).                  */
int higp_server_destroy(higp_server* server);

/* Host utility: eigenvalues θ[0..m-1] and first eigenvector components
 * τ[0..m-1] of the symmetric tridiagonal T with diagonal a[0..m-1] and
 * off-diagonal b[0..m-2] — the FP64 eigen-solve inside higp_slq_logdet
 * (implicit symmetric QR with Wilkinson shifts).  All pointers are host
 * memory; b may be NULL when m = 1.  The eigenvalues are not sorted.
 * Returns HIGP_ERR_INVALID_ARG for m < 1 or a NULL pointer and
 * HIGP_ERR_UNSUPPORTED if the iteration fails to converge.  No GPU needed. */
int higp_tridiag_eig(int32_t m, const double* a, const double* b, double* theta,
                     double* tau);

/* Static description of an error code (never NULL).                        */
const char* higp_error_string(int code);

/* Message of the last failing call on the calling thread ("" if none).      */
const char* higp_last_error(void);

/* ABI version: major·10000 + minor·100 + patch.                            */
int higp_version(void);

/* Test hook for failure handling (not part of any computation): the next
 * `count` scratch allocations made by the library in this process (any
 * thread, any call) fail as if the device were out of memory, so that the
 * calls making them return HIGP_ERR_OOM having launched nothing that
 * depends on the missing memory and leaving no state behind.  count = 0
 * disarms the hook.  Returns HIGP_ERR_INVALID_ARG for count < 0.  No GPU
 * needed.                                                                   */
int higp_debug_fail_allocs(int32_t count);

#ifdef __cplusplus
}
#endif

#endif /* HIGP_H */
