"""Pins of the oracle's NLML, gradient and log-determinant (CPU only):
SciPy's multivariate normal density, central finite differences, the
exactness of Hutchinson's estimator on a complete basis, and
Sherman–Morrison closed forms."""
import numpy as np
import pytest
from scipy.stats import multivariate_normal

import oracle
from paper_2503_02259_amd import workloads as W


def _data(n=60, d=3, seed=0):
    X = W.rng(1100 + seed, 0).random((n, d))
    y = np.sin(2 * np.pi * X[:, 0]) + 0.1 * W.rng(1100 + seed, 1).standard_normal(n)
    return X, y


@pytest.mark.parametrize("kern", [oracle.GAUSSIAN, oracle.MATERN32])
def test_nlml_matches_scipy_logpdf(kern):
    X, y = _data(seed=kern)
    l, f, s = 0.3, 1.2, 0.05
    K = oracle.khat_dense(X, kern, l, f, s)
    ref = -multivariate_normal(mean=np.zeros(len(y)), cov=K).logpdf(y)
    assert abs(oracle.nlml_exact(X, y, kern, l, f, s) - ref) < 1e-10 * abs(ref)
    assert abs(oracle.logdet_exact(X, kern, l, f, s) - np.linalg.slogdet(K)[1]) < 1e-10


@pytest.mark.parametrize("kern", [oracle.GAUSSIAN, oracle.MATERN32])
def test_exact_gradient_central_fd(kern):
    X, y = _data(80, 3, 2 + kern)
    p = dict(l=0.25, f=1.1, s=0.04)
    g = oracle.nlml_grad_exact(X, y, kern, p["l"], p["f"], p["s"])
    h = 1e-4
    for i, t in enumerate(("l", "f", "s")):
        pp, pm = dict(p), dict(p)
        pp[t] += h
        pm[t] -= h
        fd = (oracle.nlml_exact(X, y, kern, **pp) - oracle.nlml_exact(X, y, kern, **pm)) / (2 * h)
        assert abs(g[i] - fd) <= 1e-6 * max(1.0, abs(fd))


@pytest.mark.parametrize("jacobi", [True, False])
def test_hutchinson_on_complete_basis_is_exact(jacobi):
    # Probes √n·e_i (i = 1..n) satisfy (1/N) Σ z zᵀ = I exactly, so the
    # estimator equals the trace.
    n = 50
    X, y = _data(n, 2, 4)
    Z = np.sqrt(n) * np.eye(n)
    args = (oracle.GAUSSIAN, 0.3, 0.9, 0.03)
    np.testing.assert_allclose(oracle.nlml_grad_hutchinson(X, y, Z, *args, jacobi=jacobi),
                               oracle.nlml_grad_exact(X, y, *args), rtol=1e-9, atol=1e-9)


def test_hutchinson_statistical():
    n = 300
    X, y = _data(n, 3, 5)
    args = (oracle.GAUSSIAN, 0.3, 1.0, 0.05)
    exact = oracle.nlml_grad_exact(X, y, *args)
    ests = np.array([oracle.nlml_grad_hutchinson(X, y, W.rademacher(n, 8, 50 + r), *args)
                     for r in range(12)])
    se = ests.std(axis=0, ddof=1) / np.sqrt(ests.shape[0])
    assert np.all(np.abs(ests.mean(0) - exact) <= 4 * se + 1e-9)


def test_large_l_gradient_in_s_closed_form():
    n, f, s = 70, 1.1, 0.07
    X, y = _data(n, 3, 6)
    g = oracle.nlml_grad_exact(X, y, oracle.GAUSSIAN, 1e8, f, s)
    c = s + n * f * f
    alpha = (y - f * f * y.sum() / c) / s
    tr = (n - 1) / s + 1.0 / c
    assert abs(g[2] - 0.5 * (-(alpha @ alpha) + tr)) < 1e-8 * abs(tr)
    # ∂L/∂f: K̂ = f²11ᵀ + sI, ∂K̂/∂f = 2f11ᵀ
    gf = 0.5 * (-2 * f * alpha.sum() ** 2 + 2 * f * n / c)
    assert abs(g[1] - gf) < 1e-7 * max(1.0, abs(gf))


# ---- Hutch++ for the second term of eq. (2)

def test_hutchpp_trace_of_explicit_matrices():
    # Exact when A has rank ≤ |S| (Q captures the range, the rest is zero);
    # exact when the sketch spans the whole space.
    rng = W.rng(950, 0)
    n = 30
    U = rng.standard_normal((n, 3))
    A = U @ np.diag([5.0, -2.0, 0.5]) @ U.T
    S = W.rademacher(n, 4, 951)
    G = W.rademacher(n, 4, 952)
    assert abs(oracle.hutchpp_trace(lambda V: A @ V, S, G) - np.trace(A)) <= 1e-12 * np.abs(A).sum()
    B = rng.standard_normal((8, 8))
    Sg = rng.standard_normal((8, 8))
    Gg = rng.standard_normal((8, 3))
    assert abs(oracle.hutchpp_trace(lambda V: B @ V, Sg, Gg) - np.trace(B)) <= 1e-12 * np.abs(B).sum()


@pytest.mark.parametrize("jacobi", [True, False])
def test_hutchpp_gradient_with_full_sketch_is_exact(jacobi):
    n = 10
    X = W.rng(953, 0).random((n, 3))
    y = W.rng(953, 1).standard_normal(n)
    Z = W.rng(953, 2).standard_normal((n, 24))     # sketch of 12 Gaussian columns spans R^10
    g = oracle.nlml_grad_hutchpp(X, y, Z, 0, 0.3, 1.1, 0.05, jacobi=jacobi)
    e = oracle.nlml_grad_exact(X, y, 0, 0.3, 1.1, 0.05)
    np.testing.assert_allclose(g, e, rtol=1e-9)


def test_hutchpp_gradient_exact_for_low_rank_terms():
    # Points at 3 distinct locations: ∂K̂/∂l and ∂K̂/∂f = 2f·K have rank 3, so
    # without the Jacobi shift K̂⁻¹∂K̂/∂θ has rank ≤ 3 and a 4-column sketch
    # makes Hutch++ exact for l and f (s keeps its stochastic remainder).
    base = W.rng(954, 0).random((3, 3))
    X = base[np.arange(40) % 3]
    y = W.rng(954, 1).standard_normal(40)
    Z = W.rademacher(40, 9, 955)
    g = oracle.nlml_grad_hutchpp(X, y, Z, 0, 0.3, 1.1, 0.05, jacobi=False)
    e = oracle.nlml_grad_exact(X, y, 0, 0.3, 1.1, 0.05)
    np.testing.assert_allclose(g[:2], e[:2], rtol=1e-10)


def test_hutchpp_unbiased_and_lower_variance_for_decaying_spectrum():
    # Over 60 probe draws the mean is within 3.5 standard errors of the exact
    # gradient; at l = 1 (fast-decaying spectrum of K̂⁻¹∂K̂/∂l) the spread of
    # the l component is well below Hutchinson's with the same probes.
    n = 150
    X = W.rng(956, 0).random((n, 3))
    y = W.rng(956, 1).standard_normal(n)
    for l, s in ((0.5, 0.05), (1.0, 1.0)):
        e = oracle.nlml_grad_exact(X, y, 0, l, 1.0, s)
        hp, hu = [], []
        for t in range(60):
            Z = W.rademacher(n, 12, 1000 + t)
            hp.append(oracle.nlml_grad_hutchpp(X, y, Z, 0, l, 1.0, s))
            hu.append(oracle.nlml_grad_hutchinson(X, y, Z, 0, l, 1.0, s))
        hp, hu = np.array(hp), np.array(hu)
        se = hp.std(axis=0, ddof=1) / np.sqrt(60)
        assert np.all(np.abs(hp.mean(axis=0) - e) <= 3.5 * se), (hp.mean(0), e, se)
        if l == 1.0:
            assert hp[:, 0].std() < 0.6 * hu[:, 0].std()


def test_orth_range_rank_and_projection():
    """orth_range returns orthonormal columns spanning exactly range(Y): for
    Y = A·B with A n×3 and B 3×5 (rank 3, with a duplicated and a zero
    column), Q has 3 columns, QᵀQ = I, and the projector QQᵀ reproduces Y;
    a zero matrix has an empty range."""
    g = np.random.default_rng(5)
    A = g.standard_normal((40, 3))
    B = g.standard_normal((3, 5))
    Y = A @ B
    Y[:, 3] = Y[:, 0]
    Y[:, 4] = 0.0
    Q = oracle.orth_range(Y)
    assert Q.shape == (40, 3)
    np.testing.assert_allclose(Q.T @ Q, np.eye(3), atol=1e-12)
    np.testing.assert_allclose(Q @ (Q.T @ Y), Y, atol=1e-12 * np.abs(Y).max())
    # a vector outside range(A) is not reproduced
    w = g.standard_normal(40)
    w -= A @ np.linalg.lstsq(A, w, rcond=None)[0]
    assert np.linalg.norm(Q @ (Q.T @ w)) <= 1e-12 * np.linalg.norm(w)
    assert oracle.orth_range(np.zeros((10, 4))).shape == (10, 0)
