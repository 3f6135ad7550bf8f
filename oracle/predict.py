"""GP regression prediction (oracle, FP64, dense).

Test infrastructure only (see ``oracle/__init__``).

Prediction with the trained Θ (the `gpr_prediction` call of Listing 1) is
the textbook GP posterior (Rasmussen & Williams, Algorithm 2.1): with the
Cholesky factor L of K̂, α = K̂⁻¹y, the predictive mean at x_q is
f²·k(x_q, X)·α and the latent predictive variance is f² − ‖L⁻¹k*_q‖² with
k*_q = f²·k(X, x_q).  The rectangular product f²·k(Xq, X)·V is formed in row
blocks like the square MatVec.
"""
import numpy as np
import scipy.linalg

from .kernels import sqdist, kernel_value, khat_dense
from .matvec import _run_blocks


def kmatvec_cross(Xq, X, V, kernel, l, f, block=512, workers=1):
    """Y = f²·k(Xq, X; l)·V: Xq is m×d, X is n×d, V is n×k (or n)."""
    Xq = np.asarray(Xq, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    vec = V.ndim == 1
    V2 = V[:, None] if vec else V
    Y = np.empty((Xq.shape[0], V2.shape[1]))

    def one(rows):
        Y[rows] = (f * f) * (kernel_value(sqdist(Xq[rows], X), kernel, l) @ V2)

    _run_blocks(one, Xq.shape[0], block, workers)
    return Y[:, 0] if vec else Y


def gpr_predict(X, y, Xq, kernel, l, f, s):
    """(mean, latent variance) at the m query points, by Cholesky."""
    X = np.asarray(X, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    L = scipy.linalg.cholesky(khat_dense(X, kernel, l, f, s), lower=True)
    alpha = scipy.linalg.cho_solve((L, True), y)
    Ks = (f * f) * kernel_value(sqdist(X, np.asarray(Xq, dtype=np.float64)), kernel, l)  # n×m
    mean = Ks.T @ alpha
    W = scipy.linalg.solve_triangular(L, Ks, lower=True)
    var = f * f - np.sum(W * W, axis=0)
    return mean, var
