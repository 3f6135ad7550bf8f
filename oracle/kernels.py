"""Kernel functions and the regularised kernel matrix (oracle, FP64).

Test infrastructure only (see ``oracle/__init__``).

The paper defines ``K̂`` as the regularised kernel matrix with scale ``f``,
noise level ``s`` and kernel parameter ``l`` ("Gaussian Processes" section),
and names the Gaussian (RBF) and Matérn-3/2 kernels (Listing 1, Tables 1-2)
without printing their formulas.  The reading used here is the textbook one of
Rasmussen & Williams (2005), which the paper cites:

* Gaussian:    k(r) = exp(-r² / (2 l²))
* Matérn-3/2:  k(r) = (1 + √3 r / l) · exp(-√3 r / l)

with a scalar, isotropic length-scale ``l`` and ``K̂ = f²·K + s·I``.
"""
import numpy as np

GAUSSIAN = 0
MATERN32 = 1


def sqdist(Xa, Xb):
    """Squared Euclidean distances ``r²_ij = Σ_c (Xa_ic − Xb_jc)²``.

    Direct coordinate differences, accumulated over c in increasing order, so
    that ``sqdist(X, X)`` is bitwise symmetric and its diagonal is exactly 0.
    """
    Xa = np.asarray(Xa, dtype=np.float64)
    Xb = np.asarray(Xb, dtype=np.float64)
    D = np.zeros((Xa.shape[0], Xb.shape[0]))
    for c in range(Xa.shape[1]):
        diff = Xa[:, c][:, None] - Xb[:, c][None, :]
        D += diff * diff
    return D


def kernel_value(r2, kernel, l):
    """k(r; l) as a function of r² (see module docstring for the reading)."""
    if kernel == GAUSSIAN:
        return np.exp(-r2 / (2.0 * l * l))
    if kernel == MATERN32:
        a = np.sqrt(3.0 * r2) / l
        return (1.0 + a) * np.exp(-a)
    raise ValueError("unknown kernel")


def kernel_dl(r2, kernel, l):
    """∂k/∂l as a function of r².

    Gaussian: k · r² / l³.  Matérn-3/2: (3 r² / l³) · exp(−√3 r / l), which is
    what differentiating (1 + a)e^{−a} with a = √3 r / l in l gives
    (d/da[(1+a)e^{−a}] = −a e^{−a}, da/dl = −a / l).
    """
    if kernel == GAUSSIAN:
        return np.exp(-r2 / (2.0 * l * l)) * r2 / (l ** 3)
    if kernel == MATERN32:
        a = np.sqrt(3.0 * r2) / l
        return (3.0 * r2 / (l ** 3)) * np.exp(-a)
    raise ValueError("unknown kernel")


def khat_block(X, rows, kernel, l, f, s):
    """Rows ``rows`` (a slice) of K̂ = f²·k(X, X; l) + s·I, as a dense block."""
    X = np.asarray(X, dtype=np.float64)
    K = f * f * kernel_value(sqdist(X[rows], X), kernel, l)
    start = rows.start or 0
    idx = np.arange(K.shape[0])
    K[idx, start + idx] += s
    return K


def khat_dense(X, kernel, l, f, s):
    """The whole K̂ (only for small n)."""
    X = np.asarray(X, dtype=np.float64)
    return khat_block(X, slice(0, X.shape[0]), kernel, l, f, s)
