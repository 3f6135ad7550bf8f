"""Pins of the oracle's kernel functions and K̂ (CPU only).

Each check is against something other than the oracle's own formula:
scikit-learn's independent kernel implementations, closed-form limits,
textbook constants and spectral bounds.
"""
import math

import numpy as np
import pytest
from scipy.spatial.distance import cdist
from sklearn.gaussian_process.kernels import RBF, Matern

import oracle
from paper_2503_02259_amd import workloads as W


def _X(n=37, d=3, seed=0):
    return W.rng(500 + seed, 0).random((n, d))


def test_sqdist_matches_scipy_cdist():
    Xa, Xb = _X(31, 5, 1), _X(17, 5, 2)
    np.testing.assert_allclose(oracle.sqdist(Xa, Xb), cdist(Xa, Xb, "sqeuclidean"), rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("d", [1, 2, 3, 8])
def test_gaussian_matches_sklearn_rbf(d):
    X = _X(40, d, d)
    l = 0.37
    ref = RBF(length_scale=l)(X)
    got = oracle.kernel_value(oracle.sqdist(X, X), oracle.GAUSSIAN, l)
    np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("d", [1, 2, 3, 8])
def test_matern32_matches_sklearn(d):
    X = _X(40, d, 10 + d)
    l = 0.29
    ref = Matern(length_scale=l, nu=1.5)(X)
    got = oracle.kernel_value(oracle.sqdist(X, X), oracle.MATERN32, l)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-300)


def test_kernel_textbook_constants():
    # Gaussian at r = l is e^{-1/2}; Matérn-3/2 at r = l/√3 is 2/e.
    l = 0.7
    g = oracle.kernel_value(np.array([l * l]), oracle.GAUSSIAN, l)[0]
    assert abs(g - 0.6065306597126334) < 1e-15
    m = oracle.kernel_value(np.array([l * l / 3.0]), oracle.MATERN32, l)[0]
    assert abs(m - 0.7357588823428847) < 1e-15
    for kern in (oracle.GAUSSIAN, oracle.MATERN32):
        assert oracle.kernel_value(np.array([0.0]), kern, l)[0] == 1.0


@pytest.mark.parametrize("kern", [oracle.GAUSSIAN, oracle.MATERN32])
def test_kernel_dl_matches_sklearn_gradient(kern):
    # sklearn returns ∂k/∂(log l) = l·∂k/∂l for its isotropic kernels.
    X = _X(30, 3, 20 + kern)
    l = 0.41
    kobj = RBF(length_scale=l) if kern == oracle.GAUSSIAN else Matern(length_scale=l, nu=1.5)
    _, grad = kobj(X, eval_gradient=True)
    got = l * oracle.kernel_dl(oracle.sqdist(X, X), kern, l)
    np.testing.assert_allclose(got, grad[:, :, 0], rtol=1e-10, atol=1e-14)


@pytest.mark.parametrize("kern", [oracle.GAUSSIAN, oracle.MATERN32])
def test_kernel_dl_central_fd(kern):
    r2 = np.linspace(0.0, 2.0, 41)
    l, h = 0.5, 1e-6
    fd = (oracle.kernel_value(r2, kern, l + h) - oracle.kernel_value(r2, kern, l - h)) / (2 * h)
    np.testing.assert_allclose(oracle.kernel_dl(r2, kern, l), fd, rtol=1e-7, atol=1e-9)


@pytest.mark.parametrize("kern", [oracle.GAUSSIAN, oracle.MATERN32])
def test_khat_symmetric_diag_spd(kern):
    n = 120
    X = _X(n, 3, 30 + kern)
    f, s, l = 1.3, 0.02, 0.3
    K = oracle.khat_dense(X, kern, l, f, s)
    assert np.array_equal(K, K.T)                      # bitwise symmetric
    assert np.all(np.diag(K) == f * f + s)
    np.linalg.cholesky(K)                              # SPD
    lam = np.linalg.eigvalsh(K)
    assert lam[0] >= s * (1 - 1e-10)
    assert lam[-1] <= n * f * f + s + 1e-9             # Gershgorin


@pytest.mark.parametrize("kern", [oracle.GAUSSIAN, oracle.MATERN32])
def test_khat_limits(kern):
    n, f, s = 50, 1.7, 0.03
    X = _X(n, 3, 40)
    big = oracle.khat_dense(X, kern, 1e8, f, s)
    np.testing.assert_allclose(big, f * f * np.ones((n, n)) + s * np.eye(n), rtol=0, atol=1e-12)
    # points at least 0.1 apart and l = 1e-3: every off-diagonal entry vanishes
    G = np.stack(np.meshgrid(np.arange(4), np.arange(4), np.arange(3), indexing="ij"), -1).reshape(-1, 3) * 0.1
    small = oracle.khat_dense(G, kern, 1e-3, f, s)
    np.testing.assert_allclose(small, (f * f + s) * np.eye(G.shape[0]), rtol=0, atol=1e-60)


def test_khat_block_rows_match_dense():
    X = _X(70, 2, 50)
    K = oracle.khat_dense(X, oracle.GAUSSIAN, 0.2, 1.1, 0.01)
    B = oracle.khat_block(X, slice(30, 55), oracle.GAUSSIAN, 0.2, 1.1, 0.01)
    assert np.array_equal(B, K[30:55])


def test_gaussian_is_product_over_dimensions():
    X = _X(25, 3, 60)
    l = 0.33
    full = oracle.kernel_value(oracle.sqdist(X, X), oracle.GAUSSIAN, l)
    prod = np.ones_like(full)
    for c in range(3):
        prod *= oracle.kernel_value(oracle.sqdist(X[:, c:c + 1], X[:, c:c + 1]), oracle.GAUSSIAN, l)
    np.testing.assert_allclose(full, prod, rtol=1e-13)
