"""Pins of the oracle's rectangular MatVec and GP prediction (CPU)."""
import numpy as np
import pytest
from sklearn.gaussian_process import GaussianProcessRegressor
from sklearn.gaussian_process.kernels import RBF, ConstantKernel, Matern

import oracle
from paper_2503_02259_amd import workloads as W


def _data(n, m, d, seed):
    g = W.rng(20 + seed, 0)
    X = g.random((n, d))
    Xq = g.random((m, d))
    y = np.sin(2 * np.pi * X[:, 0]) + 0.1 * g.standard_normal(n)
    return X, Xq, y


@pytest.mark.parametrize("kern", [oracle.GAUSSIAN, oracle.MATERN32])
def test_cross_matvec_matches_sklearn_kernel(kern):
    X, Xq, _ = _data(70, 45, 3, 1)
    V = W.rng(21, 4).standard_normal((70, 4))
    l, f = 0.3, 1.4
    K = (RBF(l) if kern == oracle.GAUSSIAN else Matern(l, nu=1.5))(Xq, X)
    np.testing.assert_allclose(oracle.kmatvec_cross(Xq, X, V, kern, l, f, block=16),
                               f * f * K @ V, rtol=1e-12, atol=1e-12)


def test_cross_matvec_square_case_is_the_matvec_without_noise():
    X, _, _ = _data(60, 1, 2, 2)
    V = W.rng(22, 4).standard_normal((60, 3))
    l, f, s = 0.25, 0.8, 0.03
    got = oracle.kmatvec_cross(X, X, V, oracle.GAUSSIAN, l, f) + s * V
    np.testing.assert_allclose(got, oracle.kmatvec(X, V, oracle.GAUSSIAN, l, f, s), rtol=1e-12)


@pytest.mark.parametrize("kern", [oracle.GAUSSIAN, oracle.MATERN32])
def test_prediction_matches_sklearn_regressor(kern):
    X, Xq, y = _data(150, 40, 3, 3)
    l, f, s = 0.35, 1.2, 0.05
    base = RBF(l, "fixed") if kern == oracle.GAUSSIAN else Matern(l, "fixed", nu=1.5)
    gp = GaussianProcessRegressor(ConstantKernel(f * f, "fixed") * base, alpha=s,
                                  optimizer=None, normalize_y=False).fit(X, y)
    mu, sd = gp.predict(Xq, return_std=True)
    mean, var = oracle.gpr_predict(X, y, Xq, kern, l, f, s)
    np.testing.assert_allclose(mean, mu, rtol=1e-9, atol=1e-10)
    np.testing.assert_allclose(var, sd ** 2, rtol=1e-8, atol=1e-10)


def test_prediction_limits():
    X, _, y = _data(40, 1, 2, 4)
    l, f, s = 0.03, 1.3, 1e-8
    # at the training points with vanishing noise (and K well conditioned:
    # short length-scale): interpolation, zero variance
    mean, var = oracle.gpr_predict(X, y, X[:10], oracle.GAUSSIAN, l, f, s)
    np.testing.assert_allclose(mean, y[:10], atol=1e-5)
    assert np.all(np.abs(var) < 1e-5)
    # far from every training point: the prior (mean 0, variance f²)
    mean, var = oracle.gpr_predict(X, y, X[:5] + 100.0, oracle.GAUSSIAN, 0.2, f, 0.01)
    np.testing.assert_allclose(mean, 0.0, atol=1e-12)
    np.testing.assert_allclose(var, f * f, rtol=1e-12)
