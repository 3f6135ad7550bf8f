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
