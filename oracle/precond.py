"""Low-rank (Nyström) preconditioner for K̂ (oracle, FP64, dense).

Test infrastructure only (see ``oracle/__init__``).

The paper's preconditioner (AFN, Zhao et al. 2024) builds a Nyström
approximation of the kernel matrix on selected points; its full algorithm is
not in the paper.  The generic form built here:
  * r landmark points chosen by farthest-point sampling: the first is point
    0, each next one is the point whose smallest squared distance to the
    landmarks chosen so far is largest (lowest index on ties);
  * M = s·I + f²·K_nr (K_rr + εI)⁻¹ K_rn with K_nr = k(X, X_landmarks; l)
    and ε = 1e-8: the jitter keeps K_rr invertible when landmarks sit much
    closer than the length-scale (K_rr's spectrum then falls below the
    rounding level); M stays symmetric positive definite;
  * M⁻¹ by the Woodbury identity with W = K_nr:
      M⁻¹R = (R − W C⁻¹ WᵀR)/s,   C = (s/f²)·(K_rr + εI) + WᵀW.
"""
JITTER = 1e-8
import numpy as np

from .kernels import sqdist, kernel_value


def fps_landmarks(X, r):
    """Indices of r landmarks by farthest-point sampling (squared Euclidean
    distances summed over the coordinates in order)."""
    X = np.asarray(X, dtype=np.float64)
    n, d = X.shape
    r = min(r, n)
    sel = [0]
    dmin = np.full(n, np.inf)
    for _ in range(r - 1):
        p = sel[-1]
        dist = np.zeros(n)
        for c in range(d):
            dist = dist + (X[:, c] - X[p, c]) ** 2
        dmin = np.minimum(dmin, dist)
        sel.append(int(np.argmax(dmin)))
    return np.array(sel, dtype=np.int64)


def nystrom_parts(X, kernel, l, f, s, r):
    """(W, C, landmarks) of the preconditioner."""
    X = np.asarray(X, dtype=np.float64)
    idx = fps_landmarks(X, r)
    W = kernel_value(sqdist(X, X[idx]), kernel, l)
    C = (s / (f * f)) * (W[idx] + JITTER * np.eye(len(idx))) + W.T @ W
    return W, C, idx


def nystrom_apply_inv(W, C, s, R):
    """M⁻¹R by the Woodbury identity."""
    R = np.asarray(R, dtype=np.float64)
    return (R - W @ np.linalg.solve(C, W.T @ R)) / s


def nystrom_dense(W, idx, f, s):
    """M itself (small n only): s·I + f²·W (K_rr + εI)⁻¹ Wᵀ."""
    Krr = W[idx] + JITTER * np.eye(len(idx))
    return s * np.eye(W.shape[0]) + (f * f) * W @ np.linalg.solve(Krr, W.T)
