"""PCG, Lanczos and stochastic Lanczos quadrature (oracle, FP64).

Test infrastructure only (see ``oracle/__init__``).

* PCG follows the preconditioned conjugate gradient method the paper cites
  (Saad 2003, Alg. 9.1) for ``K̂⁻¹y`` with ``M ≈ K̂`` ("Gaussian Processes"
  section).  Several right-hand sides are k independent recurrences that share
  one k-column MatVec; each column stops on its own when its recursively
  updated residual satisfies ‖r‖₂/‖b‖₂ ≤ tol (checked after every iteration)
  and is then frozen.
* SLQ estimates the second term of eq. (1), log|M^{-1/2} K̂ M^{-1/2}|, with
  the stochastic Lanczos quadrature of Ubaru et al. (2017): Lanczos from
  z/‖z‖, eigen-decomposition T = S Θ Sᵀ, and ‖z‖² Σ_k S_{1k}² log θ_k per
  probe, averaged over probes.
* The same quadrature can take its tridiagonal from the coefficients of a
  PCG run on the probe (the CG–Lanczos correspondence, Saad 2003 §6.7.3;
  GPyTorch's mBCG, Gardner et al. 2018): no separate Lanczos pass.
"""
import numpy as np
import scipy.linalg


def pcg(matvec, B, tol, max_iter, mdiag=None, x0=None, refine_every=0,
        true_matvec=None, apply_minv=None, coeffs=None):
    """Solve A X = B column by column with (Jacobi-)preconditioned CG.

    matvec(P) -> A·P for an n×k block.  mdiag: diagonal of M (None = no
    preconditioner); apply_minv(R) -> M⁻¹R for a general SPD M instead.
    refine_every = R > 0 replaces the recursive residual by the true residual
    b − A·x (computed with ``true_matvec``, default ``matvec``) after every
    R-th iteration of a column.  coeffs: a dict that receives, per column,
    the step lengths α_j ("alpha") and the direction coefficients β_j
    ("beta", one per iteration that is followed by another) as lists.

    Returns (X, iters, relres, converged) with per-column arrays; relres is the
    recursive relative residual at exit.
    """
    B = np.asarray(B, dtype=np.float64)
    vec = B.ndim == 1
    B = B[:, None] if vec else B
    n, k = B.shape
    tmv = true_matvec if true_matvec is not None else matvec
    minv = None if mdiag is None else 1.0 / np.asarray(mdiag, dtype=np.float64)

    def prec(R):
        if apply_minv is not None:
            return apply_minv(R)
        return R.copy() if minv is None else minv[:, None] * R

    X = np.zeros((n, k)) if x0 is None else np.array(x0, dtype=np.float64).reshape(n, k)
    R = B - matvec(X) if x0 is not None else B.copy()
    bnorm = np.linalg.norm(B, axis=0)
    Z = prec(R)
    P = Z.copy()
    rho = np.sum(R * Z, axis=0)
    iters = np.zeros(k, dtype=np.int64)
    relres = np.where(bnorm > 0, np.linalg.norm(R, axis=0) / np.where(bnorm > 0, bnorm, 1.0), 0.0)
    active = relres > tol
    if coeffs is not None:
        coeffs["alpha"] = [[] for _ in range(k)]
        coeffs["beta"] = [[] for _ in range(k)]
    for _ in range(max_iter):
        if not active.any():
            break
        Q = matvec(P)
        a = active
        alpha = rho[a] / np.sum(P[:, a] * Q[:, a], axis=0)
        if coeffs is not None:
            for c, v in zip(np.flatnonzero(a), alpha):
                coeffs["alpha"][c].append(float(v))
        X[:, a] += alpha * P[:, a]
        R[:, a] -= alpha * Q[:, a]
        iters[a] += 1
        if refine_every > 0:
            due = a & (iters % refine_every == 0)
            if due.any():
                R[:, due] = B[:, due] - tmv(X)[:, due]
        relres[a] = np.linalg.norm(R[:, a], axis=0) / bnorm[a]
        done = a & (relres <= tol)
        active = a & ~done
        a = active & (iters < max_iter)
        if not a.any():
            break
        Z = prec(R)
        rho_new = np.sum(R[:, a] * Z[:, a], axis=0)
        beta = rho_new / rho[a]
        if coeffs is not None:
            for c, v in zip(np.flatnonzero(a), beta):
                coeffs["beta"][c].append(float(v))
        rho[a] = rho_new
        P[:, a] = Z[:, a] + beta * P[:, a]
    converged = relres <= tol
    if vec:
        return X[:, 0], iters[0], relres[0], bool(converged[0])
    return X, iters, relres, converged


def lanczos(matvec, Z, m, reorth=True, breakdown=1e-12):
    """Lanczos tridiagonalisation from each column of Z (n×N), independently.

    Step j (0-based) of column c: w = A q_j; α_j = q_jᵀw;
    w ← w − α_j q_j − β_{j−1} q_{j−1}; with ``reorth`` one classical
    Gram–Schmidt pass of w against all of q_0..q_j; β_j = ‖w‖.  The column
    stops after m steps, or early (breakdown) when β_j ≤ breakdown·max|α_0..j|,
    in which case its T has size j+1.  matvec is applied to the n×N block.

    Returns (alphas, betas): lists (one per column) of 1-D arrays of lengths
    m_c and m_c − 1.
    """
    Z = np.asarray(Z, dtype=np.float64)
    if Z.ndim == 1:
        Z = Z[:, None]
    n, N = Z.shape
    q = Z / np.linalg.norm(Z, axis=0)
    Qs = [q.copy()]
    q_prev = np.zeros_like(q)
    beta_prev = np.zeros(N)
    alphas = [[] for _ in range(N)]
    betas = [[] for _ in range(N)]
    live = np.ones(N, dtype=bool)
    amax = np.zeros(N)
    for j in range(m):
        W = matvec(q)
        alpha = np.sum(q * W, axis=0)
        W = W - alpha * q - beta_prev * q_prev
        if reorth:
            Qj = np.stack(Qs, axis=0)                    # (j+1)×n×N
            coef = np.einsum('jnc,nc->jc', Qj, W)
            W = W - np.einsum('jnc,jc->nc', Qj, coef)
        beta = np.linalg.norm(W, axis=0)
        amax = np.maximum(amax, np.abs(alpha))
        for c in range(N):
            if live[c]:
                alphas[c].append(alpha[c])
        if j == m - 1:
            break
        stop = live & (beta <= breakdown * amax)
        for c in range(N):
            if live[c] and not stop[c]:
                betas[c].append(beta[c])
        live = live & ~stop
        if not live.any():
            break
        safe = np.where(live, beta, 1.0)
        q_next = np.where(live, W / safe, 0.0)
        q_prev, q = q, q_next
        beta_prev = np.where(live, beta, 0.0)
        Qs.append(q.copy())
    return ([np.array(a) for a in alphas], [np.array(b) for b in betas])


def tridiag_eig(alpha, beta):
    """Eigenvalues θ and first eigenvector components τ of the symmetric
    tridiagonal T with diagonal alpha and off-diagonal beta (LAPACK via SciPy)."""
    alpha = np.asarray(alpha, dtype=np.float64)
    beta = np.asarray(beta, dtype=np.float64)
    if alpha.size == 1:
        return alpha.copy(), np.ones(1)
    try:
        theta, S = scipy.linalg.eigh_tridiagonal(alpha, beta)
    except np.linalg.LinAlgError:
        # LAPACK's MRRR driver can fail on long tridiagonals with clustered
        # (ghost) eigenvalues; the implicit-QR driver does not.
        theta, S = scipy.linalg.eigh_tridiagonal(alpha, beta, lapack_driver="stev")
    return theta, S[0, :]


def slq_from_tridiag(alpha, beta, znorm2):
    """One probe's quadrature: ‖z‖² Σ_k τ_k² log θ_k."""
    theta, tau = tridiag_eig(alpha, beta)
    return znorm2 * np.sum(tau * tau * np.log(theta))


def slq_logdet(matvec, Z, m, reorth=True, mdiag=None):
    """Estimate log|A| by eq. (1) with M = diag(mdiag) (None: M = I) and SLQ
    on M^{-1/2} A M^{-1/2} with the probe columns of Z.

    Returns (logdet, per_probe) where per_probe[i] = log|M| + the i-th probe's
    quadrature, so that logdet = mean(per_probe).
    """
    Z = np.asarray(Z, dtype=np.float64)
    if Z.ndim == 1:
        Z = Z[:, None]
    if mdiag is None:
        op = matvec
        logm = 0.0
    else:
        d = np.asarray(mdiag, dtype=np.float64)
        isq = 1.0 / np.sqrt(d)
        logm = float(np.sum(np.log(d)))

        def op(Q):
            return isq[:, None] * matvec(isq[:, None] * Q)
    alphas, betas = lanczos(op, Z, m, reorth=reorth)
    zn2 = np.sum(Z * Z, axis=0)
    per = np.array([logm + slq_from_tridiag(a, b, zn2[c])
                    for c, (a, b) in enumerate(zip(alphas, betas))])
    return float(np.mean(per)), per


def tridiag_from_cg(alpha, beta):
    """The Lanczos tridiagonal that m PCG steps implicitly build (Saad 2003,
    §6.7.3), from their step lengths α_0..α_{m−1} and direction
    coefficients β_0..β_{m−2}:
        T_00 = 1/α_0,   T_jj = 1/α_j + β_{j−1}/α_{j−1} (j ≥ 1),
        T_{j,j+1} = T_{j+1,j} = √β_j / α_j.
    It is the Lanczos matrix of M^{-1/2}AM^{-1/2} from M^{-1/2}b/‖M^{-1/2}b‖
    (M = I without preconditioning), up to the signs of its off-diagonal,
    which the quadrature does not see.  Returns (diagonal, off-diagonal)."""
    a = np.asarray(alpha, dtype=np.float64)
    b = np.asarray(beta, dtype=np.float64)
    m = a.size
    diag = 1.0 / a
    diag[1:] += b[:m - 1] / a[:m - 1]
    off = np.sqrt(b[:m - 1]) / a[:m - 1]
    return diag, off


def cg_logdet(matvec, Z, tol, max_iter, mdiag=None):
    """Estimate log|A| by eq. (1) with M = I (mdiag None) or a constant
    M = c·I (the Jacobi preconditioner of a stationary kernel), with the
    stochastic Lanczos quadrature whose tridiagonals come from PCG on the
    probe columns of Z (each column runs until its own stopping test or
    max_iter, see ``pcg``).  PCG with M = c·I takes the steps of CG on A/c,
    so T (``tridiag_from_cg``) is the Lanczos matrix of A/c from z/‖z‖ and
    the probe value is log|M| + ‖z‖²·e₁ᵀlog(T)e₁, as in ``slq_logdet``.
    Returns (logdet, per_probe, iters)."""
    Z = np.asarray(Z, dtype=np.float64)
    if Z.ndim == 1:
        Z = Z[:, None]
    if mdiag is not None:
        md = np.asarray(mdiag, dtype=np.float64)
        assert np.all(md == md[0]), "cg_logdet takes M = I or a constant diagonal"
    coeffs = {}
    _, iters, _, _ = pcg(matvec, Z, tol, max_iter, mdiag=mdiag, coeffs=coeffs)
    logm = 0.0 if mdiag is None else float(np.sum(np.log(np.asarray(mdiag, dtype=np.float64))))
    zn2 = np.sum(Z * Z, axis=0)
    per = []
    for c in range(Z.shape[1]):
        diag, off = tridiag_from_cg(coeffs["alpha"][c], coeffs["beta"][c])
        per.append(logm + slq_from_tridiag(diag, off, zn2[c]))
    per = np.array(per)
    return float(np.mean(per)), per, iters
