"""Negative log marginal likelihood, its gradient and exact log-determinant
(oracle, FP64, dense).

Test infrastructure only (see ``oracle/__init__``).

L(Θ) = ½(yᵀK̂⁻¹y + log|K̂| + n log 2π) and
∂L/∂θ = ½(−yᵀK̂⁻¹(∂K̂/∂θ)K̂⁻¹y + tr(K̂⁻¹ ∂K̂/∂θ)) ("Gaussian Processes"
section).  The exact forms use a Cholesky factorisation of the dense K̂ and
are meant for n up to a few thousand.  The stochastic form evaluates the
trace term by eq. (2) with the Hutchinson estimator over given probes.
"""
import numpy as np
import scipy.linalg

from .kernels import sqdist, kernel_value, kernel_dl, khat_dense
from .matvec import kmatvec_grad


def logdet_exact(X, kernel, l, f, s):
    """log|K̂| from the Cholesky factor: 2 Σ log diag(C)."""
    C = scipy.linalg.cholesky(khat_dense(X, kernel, l, f, s), lower=True)
    return 2.0 * float(np.sum(np.log(np.diag(C))))


def nlml_exact(X, y, kernel, l, f, s):
    """L(Θ) with a dense Cholesky solve and log-determinant."""
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    cf = scipy.linalg.cho_factor(khat_dense(X, kernel, l, f, s), lower=True)
    alpha = scipy.linalg.cho_solve(cf, y)
    logdet = 2.0 * float(np.sum(np.log(np.diag(cf[0]))))
    return 0.5 * (float(y @ alpha) + logdet + n * np.log(2.0 * np.pi))


def _dkhat(X, kernel, l, f, s):
    r2 = sqdist(X, X)
    return {
        "l": f * f * kernel_dl(r2, kernel, l),
        "f": 2.0 * f * kernel_value(r2, kernel, l),
        "s": np.eye(X.shape[0]),
    }


def nlml_grad_exact(X, y, kernel, l, f, s):
    """(∂L/∂l, ∂L/∂f, ∂L/∂s) with the trace taken exactly from the dense K̂⁻¹."""
    y = np.asarray(y, dtype=np.float64)
    n = y.shape[0]
    cf = scipy.linalg.cho_factor(khat_dense(X, kernel, l, f, s), lower=True)
    alpha = scipy.linalg.cho_solve(cf, y)
    Kinv = scipy.linalg.cho_solve(cf, np.eye(n))
    G = _dkhat(X, kernel, l, f, s)
    out = []
    for t in ("l", "f", "s"):
        out.append(0.5 * (-float(alpha @ (G[t] @ alpha)) + float(np.sum(Kinv * G[t]))))
    return np.array(out)


def nlml_grad_hutchinson(X, y, Z, kernel, l, f, s, jacobi=True):
    """(∂L/∂l, ∂L/∂f, ∂L/∂s) with tr(K̂⁻¹∂K̂/∂θ) split by eq. (2) with the
    Jacobi preconditioner M = diag(K̂) and its second term estimated by the
    Hutchinson estimator over the probe columns of Z:
        (1/N) Σ_i [ (K̂⁻¹z_i)ᵀ(∂K̂/∂θ z_i) − z_iᵀ M⁻¹(∂M/∂θ) z_i ].
    K̂⁻¹y and K̂⁻¹Z are taken exactly (Cholesky), so this is the estimator's
    value for the given probes, free of solver error.
    """
    y = np.asarray(y, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    n, N = Z.shape
    cf = scipy.linalg.cho_factor(khat_dense(X, kernel, l, f, s), lower=True)
    alpha = scipy.linalg.cho_solve(cf, y)
    W = scipy.linalg.cho_solve(cf, Z)
    A = np.concatenate([alpha[:, None], Z], axis=1)
    _, DL, DF, DS = kmatvec_grad(X, A, kernel, l, f, s)
    mdiag = np.full(n, f * f + s)            # stationary kernel: k(0) = 1
    dm = {"l": np.zeros(n), "f": np.full(n, 2.0 * f), "s": np.ones(n)}
    out = []
    for t, GA in (("l", DL), ("f", DF), ("s", DS)):
        quad = float(alpha @ GA[:, 0])
        if jacobi:
            tr_m = float(np.sum(dm[t] / mdiag))
            corr = np.sum(Z * Z * (dm[t] / mdiag)[:, None], axis=0)
        else:
            tr_m = 0.0
            corr = np.zeros(N)
        hutch = float(np.mean(np.sum(W * GA[:, 1:], axis=0) - corr))
        out.append(0.5 * (-quad + tr_m + hutch))
    return np.array(out)


def orth_range(Y, rcond=1e-7):
    """Orthonormal basis of the range of Y (n×s): the left singular vectors
    whose singular values exceed rcond·σ_max (a rank-revealing orth, as
    Hutch++ needs when AS is rank-deficient)."""
    U, sv, _ = np.linalg.svd(np.asarray(Y, dtype=np.float64), full_matrices=False)
    if sv.size == 0 or sv[0] == 0.0:
        return U[:, :0]
    return U[:, sv > rcond * sv[0]]


def hutchpp_trace(apply_a, S, G, rcond=1e-7):
    """Hutch++ (Meyer, Musco, Musco & Woodruff 2021, the estimator the paper
    cites next to Hutchinson's for eq. (2)): with sketch probes S and
    Hutchinson probes G, Q = orth(A·S) and
        tr(A) ≈ tr(QᵀAQ) + (1/|G|)·tr(Gᵀ(I − QQᵀ)A(I − QQᵀ)G).
    apply_a(V) -> A·V for an n×k block."""
    S = np.asarray(S, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    Q = orth_range(apply_a(S), rcond)
    top = float(np.trace(Q.T @ apply_a(Q))) if Q.shape[1] else 0.0
    Gp = G - Q @ (Q.T @ G)
    rest = float(np.trace(Gp.T @ apply_a(Gp))) / G.shape[1]
    return top + rest


def nlml_grad_hutchpp(X, y, Z, kernel, l, f, s, jacobi=True, rcond=1e-7):
    """(∂L/∂l, ∂L/∂f, ∂L/∂s) with the second term of eq. (2),
    tr(K̂⁻¹∂K̂/∂θ − M⁻¹∂M/∂θ), estimated by Hutch++ per θ (``hutchpp_trace``)
    instead of Hutchinson's estimator.  The probe block Z (n×N) is split into
    the sketch S = Z[:, :N//2] and the Hutchinson probes G = Z[:, N//2:]
    (Meyer et al. give the sketch and the remainder equal shares).  M is
    diag(K̂) = (f²+s)·I with ``jacobi``, else I.  Solves are exact (dense
    Cholesky), so this is the estimator's value for the given probes."""
    y = np.asarray(y, dtype=np.float64)
    Z = np.asarray(Z, dtype=np.float64)
    n, N = Z.shape
    ns = N // 2
    S, G = Z[:, :ns], Z[:, ns:]
    cf = scipy.linalg.cho_factor(khat_dense(X, kernel, l, f, s), lower=True)
    alpha = scipy.linalg.cho_solve(cf, y)
    D = _dkhat(X, kernel, l, f, s)
    m = f * f + s
    cm = {"l": 0.0, "f": 2.0 * f / m, "s": 1.0 / m} if jacobi else {"l": 0.0, "f": 0.0, "s": 0.0}
    out = []
    for t in ("l", "f", "s"):
        c = cm[t]

        def apply_a(V, Dt=D[t], c=c):
            return scipy.linalg.cho_solve(cf, Dt @ V) - c * V
        est = hutchpp_trace(apply_a, S, G, rcond)
        out.append(0.5 * (-float(alpha @ (D[t] @ alpha)) + c * n + est))
    return np.array(out)
