"""Dense, row-blocked MatVecs with K̂ and its derivatives (oracle, FP64).

Test infrastructure only (see ``oracle/__init__``).

The paper's on-the-fly MatVec forms small kernel-matrix blocks, multiplies
them into the vectors and discards them ("Statement of Need", MatVec
paragraph).  This oracle does the same thing in the plainest possible form:
each block of ``block`` rows of K̂ is formed densely in float64 (direct
coordinate differences, ``np.exp``) and multiplied with BLAS.  The rows of a
block never depend on another block, so blocks may run on a thread pool
(NumPy ufuncs and BLAS release the GIL); the result does not depend on the
number of workers.
"""
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .kernels import sqdist, kernel_value, kernel_dl


def _row_blocks(n, block):
    return [slice(i, min(i + block, n)) for i in range(0, n, block)]


def _run_blocks(fn, n, block, workers):
    blocks = _row_blocks(n, block)
    if workers is None or workers <= 1:
        for b in blocks:
            fn(b)
    else:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(fn, blocks))


def _out_rows(n, rows):
    """The output rows (a slice of range(n)) and their offset in the result."""
    sel = slice(0, n) if rows is None else slice(*rows.indices(n)[:2])
    return sel, sel.start


def kmatvec(X, V, kernel, l, f, s, block=512, workers=1, rows=None):
    """Y = K̂·V with K̂ = f²·k(X, X; l) + s·I.  X is n×d, V is n×k (or n).
    ``rows`` (a slice, default all) restricts the output to those rows."""
    X = np.asarray(X, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    vec = V.ndim == 1
    V2 = V[:, None] if vec else V
    sel, off = _out_rows(X.shape[0], rows)
    Y = np.empty((sel.stop - sel.start, V2.shape[1]))

    def one(b):
        r = slice(b.start + off, b.stop + off)
        K = kernel_value(sqdist(X[r], X), kernel, l)
        Y[b] = (f * f) * (K @ V2) + s * V2[r]

    _run_blocks(one, sel.stop - sel.start, block, workers)
    return Y[:, 0] if vec else Y


def kmatvec_grad(X, V, kernel, l, f, s, block=512, workers=1):
    """Derivative MatVecs ∂K̂/∂θ·V for θ = l, f, s, plus K̂·V.

    ∂K̂/∂l = f²·∂k/∂l, ∂K̂/∂f = 2f·k, ∂K̂/∂s = I (K̂ = f²k + sI).
    Returns (KV, dL_V, dF_V, dS_V).
    """
    X = np.asarray(X, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    n = X.shape[0]
    KV = np.empty_like(V)
    DL = np.empty_like(V)
    DF = np.empty_like(V)

    def one(rows):
        r2 = sqdist(X[rows], X)
        KVb = kernel_value(r2, kernel, l) @ V
        KV[rows] = (f * f) * KVb + s * V[rows]
        DL[rows] = (f * f) * (kernel_dl(r2, kernel, l) @ V)
        DF[rows] = (2.0 * f) * KVb

    _run_blocks(one, n, block, workers)
    return KV, DL, DF, V.copy()


def round_bf16(a):
    """Round float64 values to the nearest bfloat16 (8 significant bits),
    ties to even, returned as float64.  Normal range only (|a| ≥ 2⁻¹²⁶ or 0)."""
    a = np.asarray(a, dtype=np.float64)
    m, e = np.frexp(a)               # a = m·2^e, 0.5 ≤ |m| < 1
    return np.ldexp(np.round(m * 256.0), e - 8)   # np.round: half to even


def kmatvec_bf16_emulated(X, V, kernel, l, f, s, block=512, workers=1, rows=None):
    """The BF16 form of the MatVec, emulated: the kernel tile k(X, X; l) and
    V are each rounded to bfloat16 (round to nearest even), their products
    are exact and summed in float64; then Y = f²·acc + s·V with V unrounded.
    ``rows`` (a slice, default all) restricts the output to those rows.

    This predicts the behaviour of a K-tile×V product done in BF16 with wide
    accumulation; it is not a pin of the FP64 result.
    """
    X = np.asarray(X, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    sel, off = _out_rows(X.shape[0], rows)
    Vb = round_bf16(V)
    Y = np.empty((sel.stop - sel.start,) + V.shape[1:])

    def one(b):
        r = slice(b.start + off, b.stop + off)
        Kb = round_bf16(kernel_value(sqdist(X[r], X), kernel, l))
        Y[b] = (f * f) * (Kb @ Vb) + s * V[r]

    _run_blocks(one, sel.stop - sel.start, block, workers)
    return Y


def split_bf16(a):
    """Two-term bfloat16 split: hi = RNE(a), lo = RNE(a − hi).  With the
    bfloat16 unit roundoff u = 2⁻⁸, |a − hi| ≤ u·|a| and
    |a − hi − lo| ≤ u²·|a| = 2⁻¹⁶·|a|."""
    hi = round_bf16(a)
    return hi, round_bf16(np.asarray(a, dtype=np.float64) - hi)


def kmatvec_bf16x3_emulated(X, V, kernel, l, f, s, block=512, workers=1, rows=None):
    """The split-BF16 form of the MatVec, emulated: the kernel tile K and V
    are each split into hi + lo bfloat16 pairs (``split_bf16``) and the
    product is formed from the three leading terms
    K_hi·V_hi + K_hi·V_lo + K_lo·V_hi (the K_lo·V_lo term, of relative size
    at most about 2⁻¹⁶, is dropped), with exact products summed in float64; then
    Y = f²·acc + s·V with V unsplit.

    Like ``kmatvec_bf16_emulated`` this predicts a kernel's arithmetic; it is
    pinned by the split's error bound against the FP64 product, not by a value
    the paper prints.  ``rows`` (a slice, default all) restricts the output to
    those rows.
    """
    X = np.asarray(X, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    sel, off = _out_rows(X.shape[0], rows)
    Vh, Vl = split_bf16(V)
    Y = np.empty((sel.stop - sel.start,) + V.shape[1:])

    def one(b):
        r = slice(b.start + off, b.stop + off)
        Kh, Kl = split_bf16(kernel_value(sqdist(X[r], X), kernel, l))
        Y[b] = (f * f) * (Kh @ Vh + Kh @ Vl + Kl @ Vh) + s * V[r]

    _run_blocks(one, sel.stop - sel.start, block, workers)
    return Y
