"""Pins of the oracle's PCG, Lanczos and SLQ (CPU only): Cholesky solves,
Sherman–Morrison closed forms, dense eigen-decompositions and exact
log-determinants, and statistical bounds."""
import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2503_02259_amd import workloads as W


def _setup(n=200, d=3, seed=0, l=0.3, f=1.0, s=0.05, kern=0):
    X = W.rng(900 + seed, 0).random((n, d))
    mv = lambda P: oracle.kmatvec(X, P, kern, l, f, s)
    return X, mv, oracle.khat_dense(X, kern, l, f, s)


def test_pcg_matches_cholesky():
    X, mv, K = _setup()
    B = W.rng(1, 4).standard_normal((200, 3))
    Xs, it, rr, conv = oracle.pcg(mv, B, 1e-10, 500)
    ref = scipy.linalg.cho_solve(scipy.linalg.cho_factor(K), B)
    assert conv.all()
    cond = np.linalg.cond(K)
    for c in range(3):
        assert np.linalg.norm(Xs[:, c] - ref[:, c]) / np.linalg.norm(ref[:, c]) < 10 * cond * 1e-10
        true_rel = np.linalg.norm(B[:, c] - K @ Xs[:, c]) / np.linalg.norm(B[:, c])
        assert true_rel < 1.1e-10


def test_pcg_jacobi_equals_cg_for_stationary_kernel():
    X, mv, K = _setup(seed=1)
    b = W.rng(2, 4).standard_normal(200)
    x1, it1, _, _ = oracle.pcg(mv, b, 1e-9, 500)
    x2, it2, _, _ = oracle.pcg(mv, b, 1e-9, 500, mdiag=np.diag(K))
    assert abs(int(it1) - int(it2)) <= 1
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) < 1e-8


def test_pcg_large_l_sherman_morrison():
    n, f, s = 300, 1.3, 0.02
    X, mv, _ = _setup(n=n, l=1e8, f=f, s=s, seed=2)
    b = W.rng(3, 4).standard_normal(n)
    x, it, _, conv = oracle.pcg(mv, b, 1e-12, 50)
    ref = (b - f * f * b.sum() / (s + n * f * f)) / s
    assert conv and it <= 2
    np.testing.assert_allclose(x, ref, rtol=1e-9)


def test_pcg_small_l_one_iteration():
    G = np.stack(np.meshgrid(np.arange(5), np.arange(5), np.arange(4), indexing="ij"), -1).reshape(-1, 3) * 0.1
    f, s = 1.0, 0.1
    mv = lambda P: oracle.kmatvec(G, P, 0, 1e-3, f, s)
    b = W.rng(4, 4).standard_normal(G.shape[0])
    x, it, _, conv = oracle.pcg(mv, b, 1e-12, 10)
    assert conv and it == 1
    np.testing.assert_allclose(x, b / (f * f + s), rtol=1e-14)


def test_pcg_warm_start_and_frozen_columns_and_zero_rhs():
    X, mv, K = _setup(seed=3)
    B = W.rng(5, 4).standard_normal((200, 3))
    B[:, 1] = 0.0
    ref = scipy.linalg.cho_solve(scipy.linalg.cho_factor(K), B)
    Xs, it, rr, conv = oracle.pcg(mv, B, 1e-8, 500, x0=ref)
    assert conv.all() and it.max() == 0
    Xs, it, rr, conv = oracle.pcg(mv, B, 1e-8, 500)
    assert it[1] == 0 and np.all(Xs[:, 1] == 0.0) and conv.all()
    Xs2, it2, _, conv2 = oracle.pcg(mv, B, 1e-8, 3)
    assert not conv2[0] and it2[0] == 3           # max_iter is a cap, not an error


def test_pcg_residual_replacement_keeps_convergence_in_fp64():
    # CG iterates are sensitive to any perturbation, so the two runs need not
    # agree step by step; both must converge, with true residuals at the
    # tolerance and close iteration counts.
    X, mv, K = _setup(seed=4)
    b = W.rng(6, 4).standard_normal(200)
    for R in (0, 10):
        x, it, rr, conv = oracle.pcg(mv, b, 1e-10, 500, refine_every=R)
        assert conv
        assert np.linalg.norm(b - K @ x) / np.linalg.norm(b) < 1.1e-10
        assert 90 <= it <= 140


def test_tridiag_eig_matches_dense():
    a = W.rng(7, 4).standard_normal(12) + 5
    b = W.rng(8, 4).random(11)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    th, tau = oracle.tridiag_eig(a, b)
    lam, S = np.linalg.eigh(T)
    np.testing.assert_allclose(th, lam, rtol=1e-13)
    np.testing.assert_allclose(np.abs(tau), np.abs(S[0]), atol=1e-12)


def test_lanczos_full_length_reproduces_spectrum_and_quadratic_form():
    # m = n: T is similar to A, and the quadrature is zᵀ log(A) z exactly.
    n = 40
    X, mv, K = _setup(n=n, seed=5, l=0.2)
    z = W.rademacher(n, 1, 11)[:, 0]
    al, be = oracle.lanczos(mv, z, n)
    m = al[0].size
    th, tau = oracle.tridiag_eig(al[0], be[0])
    lam, S = np.linalg.eigh(K)
    quad_ref = float(z @ (S @ (np.log(lam) * (S.T @ z))))
    quad = oracle.slq_from_tridiag(al[0], be[0], float(z @ z))
    assert abs(quad - quad_ref) < 1e-11 * abs(quad_ref)
    if m == n:
        np.testing.assert_allclose(np.sort(th), lam, rtol=1e-10)


def test_slq_large_l_closed_form():
    n, f, s = 250, 1.0, 0.01
    X, mv, K = _setup(n=n, l=1e8, f=f, s=s, seed=6)
    Z = W.rademacher(n, 6, 12)
    logdet, per = oracle.slq_logdet(mv, Z, 30)
    one_z = Z.sum(0)
    ref = np.log(s) * (n - one_z ** 2 / n) + np.log(s + n * f * f) * one_z ** 2 / n
    np.testing.assert_allclose(per, ref, rtol=1e-10)
    exact = (n - 1) * np.log(s) + np.log(s + n * f * f)
    assert abs(np.linalg.slogdet(K)[1] - exact) < 1e-9 * abs(exact)


def test_slq_small_l_exact():
    G = np.stack(np.meshgrid(np.arange(5), np.arange(5), np.arange(4), indexing="ij"), -1).reshape(-1, 3) * 0.1
    n, f, s = G.shape[0], 1.2, 0.1
    mv = lambda P: oracle.kmatvec(G, P, 0, 1e-3, f, s)
    logdet, per = oracle.slq_logdet(mv, W.rademacher(n, 4, 13), 10)
    np.testing.assert_allclose(per, n * np.log(f * f + s), rtol=1e-13)


def test_slq_jacobi_equals_plain_and_statistical_accuracy():
    n = 400
    X, mv, K = _setup(n=n, seed=7, l=0.5, s=0.01)
    Z = W.rademacher(n, 24, 14)
    ld1, per1 = oracle.slq_logdet(mv, Z, 30)
    ld2, per2 = oracle.slq_logdet(mv, Z, 30, mdiag=np.diag(K))
    np.testing.assert_allclose(per1, per2, rtol=1e-9, atol=1e-9)
    exact = np.linalg.slogdet(K)[1]
    se = per1.std(ddof=1) / np.sqrt(per1.size)
    assert abs(ld1 - exact) <= 3 * se + 1e-6 * abs(exact)


def test_lanczos_reorth_agreement_between_orders():
    # With full reorthogonalisation the tridiagonal is insensitive to the
    # summation order of the MatVec (here: different row-block sizes).
    n = 300
    X = W.rng(901, 0).random((n, 3))
    z = W.rademacher(n, 2, 15)
    mv1 = lambda P: oracle.kmatvec(X, P, 0, 0.5, 1.0, 0.01, block=512)
    mv2 = lambda P: oracle.kmatvec(X, P, 0, 0.5, 1.0, 0.01, block=13)
    a1, b1 = oracle.lanczos(mv1, z, 25)
    a2, b2 = oracle.lanczos(mv2, z, 25)
    for c in range(2):
        np.testing.assert_allclose(a1[c], a2[c], rtol=1e-10)
        np.testing.assert_allclose(b1[c], b2[c], rtol=1e-9)


# ---- log-determinant from the PCG coefficients (CG–Lanczos correspondence)

def test_cg_tridiagonal_equals_lanczos_in_early_steps():
    # Before orthogonality is lost, the T that PCG implicitly builds is the
    # Lanczos T from the same start vector (Lanczos with full
    # reorthogonalisation, pinned above against dense spectra).
    n = 300
    X, mv, K = _setup(n=n, seed=3, l=0.3, s=0.1)
    Z = W.rademacher(n, 3, 21)
    co = {}
    oracle.pcg(mv, Z, 1e-15, 10, coeffs=co)
    la, lb = oracle.lanczos(mv, Z, 10)
    for c in range(3):
        d, o = oracle.tridiag_from_cg(co["alpha"][c], co["beta"][c])
        np.testing.assert_allclose(d, la[c], rtol=1e-11)
        np.testing.assert_allclose(np.abs(o), lb[c], rtol=1e-10)
    # with the constant Jacobi M the coefficients are those of CG on K̂/(f²+s)
    co2 = {}
    oracle.pcg(mv, Z, 1e-15, 10, mdiag=np.diag(K), coeffs=co2)
    la2, _ = oracle.lanczos(lambda P: mv(P) / K[0, 0], Z, 10)
    d2, _ = oracle.tridiag_from_cg(co2["alpha"][0], co2["beta"][0])
    np.testing.assert_allclose(d2, la2[0], rtol=1e-11)


def test_cg_logdet_to_convergence_is_the_quadratic_form():
    # Run to convergence the quadrature is exact: ‖z‖²e₁ᵀlog(T)e₁ = zᵀlog(K̂)z.
    n = 200
    X, mv, K = _setup(n=n, seed=4, l=0.3, s=0.1)
    Z = W.rademacher(n, 4, 22)
    w, V = np.linalg.eigh(K)
    exact = np.array([z @ (V @ (np.log(w) * (V.T @ z))) for z in Z.T])
    for md in (None, np.diag(K)):
        ld, per, it = oracle.cg_logdet(mv, Z, 1e-13, 500, mdiag=md)
        assert np.all(it < 500)
        np.testing.assert_allclose(per, exact, rtol=1e-11)
        assert abs(ld - exact.mean()) <= 1e-11 * abs(exact.mean())


def test_cg_logdet_large_l_closed_form():
    # l → ∞: K̂ = f²11ᵀ + sI; CG ends after two steps and the probe value is
    # log s·(n − (1ᵀz)²/n) + log(s + nf²)·(1ᵀz)²/n.
    n, f, s = 64, 1.3, 0.2
    X = W.rng(905, 0).random((n, 3))
    mv = lambda P: oracle.kmatvec(X, P, 0, 1e8, f, s)
    Z = W.rademacher(n, 5, 23)
    ld, per, it = oracle.cg_logdet(mv, Z, 1e-12, 50)
    one = Z.sum(axis=0) ** 2 / n
    ref = np.log(s) * (n - one) + np.log(s + n * f * f) * one
    assert np.all(it <= 2)
    np.testing.assert_allclose(per, ref, rtol=1e-12)


def test_cg_logdet_statistical_accuracy():
    n = 400
    X, mv, K = _setup(n=n, seed=7, l=0.5, s=0.01)
    Z = W.rademacher(n, 24, 14)
    ld, per, it = oracle.cg_logdet(mv, Z, 1e-8, 60, mdiag=np.diag(K))
    exact = np.linalg.slogdet(K)[1]
    se = per.std(ddof=1) / np.sqrt(per.size)
    assert abs(ld - exact) <= 3 * se + 1e-6 * abs(exact)
