"""Python API over the C ABI: torch device tensors in, torch tensors out.

Every function only marshals arguments (shapes, dtypes, device pointers and
the current HIP stream) and calls the library; all arithmetic of the path
runs in the HIP kernels.  Tensors must be contiguous and on a ROCm device;
float64 selects the FP64 form, float32 the FP32 form (or a BF16 form with
``precision="bf16"`` or the split ``precision="bf16x3"``).
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import GAUSSIAN, MATERN32, FP64, FP32, BF16, BF16X3, HigpError  # noqa: F401

_KERNELS = {"gaussian": GAUSSIAN, "rbf": GAUSSIAN, "matern32": MATERN32, GAUSSIAN: GAUSSIAN,
            MATERN32: MATERN32}


def _kernel_id(kernel):
    try:
        return _KERNELS[kernel.lower() if isinstance(kernel, str) else kernel]
    except KeyError:
        raise ValueError("unknown kernel %r" % (kernel,))


def _prec(X, precision):
    if precision is None:
        if X.dtype == torch.float64:
            return FP64
        if X.dtype == torch.float32:
            return FP32
        raise TypeError("X must be float64 or float32")
    p = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "bf16x3": BF16X3}.get(precision, precision)
    want = torch.float64 if p == FP64 else torch.float32
    if X.dtype != want:
        raise TypeError("precision %r needs %s tensors" % (precision, want))
    return p


def _dev(t, name, dtype, shape=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream, device):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


def problem(X, kernel, l, f, s, precision=None, symmetric=True):
    """The ABI problem struct for points X (n×d device tensor).
    symmetric=False selects the full-block FP32 MatVec where the symmetric
    one would apply (n ≥ 32768 and k ≤ 2 with d ≤ 4, or k = 1 with d ≤ 8)."""
    if X.dim() != 2:
        raise ValueError("X must be n×d")
    p = _lib.Problem()
    p.kernel = _kernel_id(kernel)
    p.prec = _prec(X, precision)
    p.n, p.d = X.shape
    p.flags = 0 if symmetric else _lib.HIGP_FLAG_NO_SYMMETRIC
    p.X = _dev(X, "X", X.dtype)
    p.l, p.f, p.s = float(l), float(f), float(s)
    return p


def _as2d(V):
    return (V.unsqueeze(1), True) if V.dim() == 1 else (V, False)


def kmatvec(X, V, kernel, l, f, s, precision=None, out=None, stream=None, symmetric=True):
    """Y = K̂·V with K̂ = f²·k(X, X; l) + s·I (on-the-fly; K̂ is never stored).
    symmetric=False: see ``problem``."""
    p = problem(X, kernel, l, f, s, precision, symmetric)
    V2, squeeze = _as2d(V)
    n, k = V2.shape
    vp = _dev(V2, "V", X.dtype, (p.n, k))
    Y = torch.empty_like(V2) if out is None else out.view(n, k)
    yp = _dev(Y, "out", X.dtype, (p.n, k))
    _lib.check(_lib.lib().higp_kmatvec(ctypes.byref(p), k, vp, yp, _stream(stream, X.device)))
    return Y[:, 0] if squeeze else Y


def kmatvec_grad(X, V, kernel, l, f, s, precision=None, want=("kv", "dl", "df", "ds"),
                 stream=None):
    """(K̂V, ∂K̂/∂l·V, ∂K̂/∂f·V, ∂K̂/∂s·V); entries not in `want` are None."""
    p = problem(X, kernel, l, f, s, precision)
    V2, squeeze = _as2d(V)
    n, k = V2.shape
    vp = _dev(V2, "V", X.dtype, (p.n, k))
    outs = [torch.empty_like(V2) if w in want else None for w in ("kv", "dl", "df", "ds")]
    ptrs = [ctypes.c_void_p(o.data_ptr()) if o is not None else None for o in outs]
    _lib.check(_lib.lib().higp_kmatvec_grad(ctypes.byref(p), k, vp, *ptrs,
                                           _stream(stream, X.device)))
    if squeeze:
        outs = [o[:, 0] if o is not None else None for o in outs]
    return tuple(outs)


_PRECOND = {"jacobi": 1, "none": 0, "nystrom": 2, None: 0, 0: 0, 1: 1, 2: 2}


def pcg(X, B, kernel, l, f, s, tol=1e-6, max_iter=1000, precond="jacobi", refine_every=0,
        x0=None, check_every=0, precision=None, refine_prec="fp64", return_fp64=False,
        rank=0, stream=None):
    """Solve K̂·x = b for each column of B.  Returns (x, info) with info a dict
    of per-column numpy arrays: iters, relres (tracked residual), converged.
    With refine_every = R > 0 the tracked residual is replaced by b − K̂x every
    R iterations, the MatVec then running in `refine_prec` ("fp64"/"fp32").
    With return_fp64 the FP64 iterate is returned as well: (x, x64, info).
    precond: "none", "jacobi" or "nystrom" (``rank`` landmarks, 0 = default)."""
    p = problem(X, kernel, l, f, s, precision)
    B2, squeeze = _as2d(B)
    n, k = B2.shape
    bp = _dev(B2, "B", X.dtype, (p.n, k))
    if x0 is not None:
        Xs = (x0.unsqueeze(1) if x0.dim() == 1 else x0).clone()
    else:
        Xs = torch.empty_like(B2)
    xp = _dev(Xs, "x0", X.dtype, (p.n, k))
    o = _lib.PcgOpts(tol=float(tol), max_iter=int(max_iter),
                     precond=_PRECOND[precond], rank=int(rank),
                     refine_every=int(refine_every), use_x0=1 if x0 is not None else 0,
                     check_every=int(check_every),
                     refine_prec={"fp64": FP64, "fp32": FP32, FP64: FP64, FP32: FP32}[refine_prec])
    x64 = None
    if return_fp64:
        x64 = torch.empty(B2.shape, dtype=torch.float64, device=B2.device)
        o.x_fp64 = x64.data_ptr()
    iters = np.zeros(k, dtype=np.int32)
    relres = np.zeros(k, dtype=np.float64)
    conv = np.zeros(k, dtype=np.int32)
    info = _lib.PcgInfo(iters.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                        relres.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                        conv.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    _lib.check(_lib.lib().higp_pcg(ctypes.byref(p), k, bp, xp, ctypes.byref(o), ctypes.byref(info),
                                  _stream(stream, X.device)))
    res = dict(iters=iters, relres=relres, converged=conv.astype(bool))
    if squeeze:
        res = {key: v[0] for key, v in res.items()}
        Xs = Xs[:, 0]
        x64 = x64[:, 0] if x64 is not None else None
    return (Xs, x64, res) if return_fp64 else (Xs, res)


def slq_logdet(X, Z, kernel, l, f, s, nsteps, reorth=True, precond="jacobi", precision=None,
               stream=None):
    """log|K̂| by eq. (1) and stochastic Lanczos quadrature over the probe
    columns of Z.  Returns (logdet, per_probe numpy array)."""
    p = problem(X, kernel, l, f, s, precision)
    n, N = Z.shape
    zp = _dev(Z, "Z", X.dtype, (p.n, N))
    logdet = ctypes.c_double(0.0)
    per = np.zeros(N, dtype=np.float64)
    _lib.check(_lib.lib().higp_slq_logdet(
        ctypes.byref(p), N, int(nsteps), zp, 0, 1 if reorth else 0,
        {"jacobi": 1, "none": 0, None: 0, 0: 0, 1: 1}[precond], ctypes.byref(logdet),
        per.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _stream(stream, X.device)))
    return logdet.value, per


def tridiag_eig(a, b):
    """Host FP64 eigen-solve used by SLQ: (θ, τ) of the tridiagonal (a, b)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    m = a.size
    th = np.zeros(m)
    tau = np.zeros(m)
    dp = ctypes.POINTER(ctypes.c_double)
    _lib.check(_lib.lib().higp_tridiag_eig(m, a.ctypes.data_as(dp),
                                          b.ctypes.data_as(dp) if b.size else None,
                                          th.ctypes.data_as(dp), tau.ctypes.data_as(dp)))
    return th, tau


def coldot(A, B, stream=None):
    """Column dot products Σ_i A[i,c]·B[i,c] (FP64, deterministic) of two
    device n×k blocks (float32 or float64 each).  Returns a numpy array."""
    A2 = A.unsqueeze(1) if A.dim() == 1 else A
    B2 = B.unsqueeze(1) if B.dim() == 1 else B
    if A2.shape != B2.shape:
        raise ValueError("shape mismatch %s vs %s" % (tuple(A2.shape), tuple(B2.shape)))
    n, k = A2.shape
    pa = FP64 if A2.dtype == torch.float64 else FP32
    pb = FP64 if B2.dtype == torch.float64 else FP32
    ap = _dev(A2, "A", A2.dtype)
    bp = _dev(B2, "B", B2.dtype)
    out = np.zeros(k, dtype=np.float64)
    _lib.check(_lib.lib().higp_coldot(n, k, pa, ap, pb, bp,
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     _stream(stream, A2.device)))
    return out


def nlml(X, y, Z, kernel, l, f, s, tol=1e-6, max_iter=2000, precond="jacobi", refine_every=0,
         nsteps=50, reorth=True, precision=None, stream=None, logdet="slq", trace="hutchinson"):
    """L(Θ) and (∂L/∂l, ∂L/∂f, ∂L/∂s) by PCG on [y | Z], SLQ over Z and the
    Hutchinson estimator (eq. (1) and (2)).  Returns (loss, grad, info).
    logdet: "slq" (a Lanczos pass over Z) or "cg" (the tridiagonals of the
    PCG run on the Z columns); trace: "hutchinson" or "hutchpp"."""
    p = problem(X, kernel, l, f, s, precision)
    n, N = Z.shape
    yp = _dev(y, "y", X.dtype, (p.n,))
    zp = _dev(Z, "Z", X.dtype, (p.n, N))
    o = _lib.NlmlOpts(tol=float(tol), max_iter=int(max_iter),
                      precond={"jacobi": 1, "none": 0, None: 0, 0: 0, 1: 1}[precond],
                      refine_every=int(refine_every), nsteps=int(nsteps),
                      reorth=1 if reorth else 0, logdet_mode={"slq": 0, "cg": 1}[logdet],
                      trace_mode={"hutchinson": 0, "hutchpp": 1}[trace], reserved=0)
    loss = ctypes.c_double()
    logdet = ctypes.c_double()
    its = ctypes.c_int32()
    grad = np.zeros(3, dtype=np.float64)
    _lib.check(_lib.lib().higp_nlml(ctypes.byref(p), yp, N, zp, ctypes.byref(o),
                                   ctypes.byref(loss),
                                   grad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   ctypes.byref(logdet), ctypes.byref(its),
                                   _stream(stream, X.device)))
    return loss.value, grad, dict(logdet=logdet.value, pcg_iters=its.value)


def kmatvec_cross(Xq, X, V, kernel, l, f, precision=None, out=None, stream=None):
    """Y = f²·k(Xq, X; l)·V (rectangular; the product prediction needs).
    X: n×d training points, Xq: m×d query points, V: n×k (or n)."""
    p = problem(X, kernel, l, f, 0.0, precision)
    V2, squeeze = _as2d(V)
    k = V2.shape[1]
    m = Xq.shape[0]
    if Xq.dim() != 2 or Xq.shape[1] != p.d:
        raise ValueError("Xq must be m×%d" % p.d)
    xq = _dev(Xq, "Xq", X.dtype)
    vp = _dev(V2, "V", X.dtype, (p.n, k))
    Y = out if out is not None else torch.empty((m, k), dtype=X.dtype, device=X.device)
    yp = _dev(Y, "Y", X.dtype, (m, k))
    _lib.check(_lib.lib().higp_kmatvec_cross(ctypes.byref(p), m, xq, k, vp, yp,
                                            _stream(stream, X.device)))
    return Y[:, 0] if squeeze else Y


def gpr_predict(X, y, Xq, kernel, l, f, s, tol=1e-6, max_iter=1000, precond="jacobi",
                want_var=False, precision=None, stream=None, rank=0):
    """GP regression prediction at the query points Xq with the trained
    (l, f, s): returns (mean, var, info) — var is the latent predictive
    variance (None unless want_var) and info holds the iterations of the
    α = K̂⁻¹y solve.  rank: Nyström landmarks when precond is "nystrom"
    (0: min(n, 1024))."""
    p = problem(X, kernel, l, f, s, precision)
    m = Xq.shape[0]
    if Xq.dim() != 2 or Xq.shape[1] != p.d:
        raise ValueError("Xq must be m×%d" % p.d)
    yp = _dev(y, "y", X.dtype, (p.n,))
    xq = _dev(Xq, "Xq", X.dtype)
    mean = torch.empty(m, dtype=X.dtype, device=X.device)
    var = torch.empty(m, dtype=X.dtype, device=X.device) if want_var else None
    o = _lib.PredictOpts(tol=float(tol), max_iter=int(max_iter), precond=_PRECOND[precond],
                         want_var=1 if want_var else 0, rank=int(rank))
    its = ctypes.c_int32()
    _lib.check(_lib.lib().higp_gpr_predict(
        ctypes.byref(p), yp, m, xq, ctypes.byref(o), ctypes.c_void_p(mean.data_ptr()),
        ctypes.c_void_p(var.data_ptr()) if var is not None else None, ctypes.byref(its),
        _stream(stream, X.device)))
    return mean, var, dict(pcg_iters=its.value)


def fps_landmarks(X, rank, stream=None):
    """Indices (numpy int32) of the min(rank, n) farthest-point landmarks of
    the Nyström preconditioner."""
    p = problem(X, 0, 1.0, 1.0, 0.0)
    r = min(int(rank), p.n)
    idx = np.zeros(r, dtype=np.int32)
    _lib.check(_lib.lib().higp_fps_landmarks(ctypes.byref(p), int(rank),
                                            idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            _stream(stream, X.device)))
    return idx


def debug_fail_allocs(count):
    """Test hook: the library's next ``count`` scratch allocations fail with
    HIGP_ERR_OOM (0 disarms it)."""
    _lib.check(_lib.lib().higp_debug_fail_allocs(int(count)))
