"""The estimator variants of higp_nlml against the oracle: log|K̂| from the
tridiagonals PCG builds on the probe columns (logdet="cg"), and Hutch++ for
the trace term of eq. (2) (trace="hutchpp")."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_02259_amd as hg
from paper_2503_02259_amd import workloads as W
from helpers import as_prec, to_dev

pytestmark = pytest.mark.gpu


def _case(n, N, dtype, l=0.2, f=1.0, s=0.05, seed=4):
    # Gradient workload recipe (uniform [0,1]^3, y = sin(2πx₀) + noise,
    # Rademacher probes) at a size the dense oracle handles.
    X = as_prec(W.uniform_points(n, 3, seed), dtype)
    y = as_prec(W.sine_targets(X, seed), dtype)
    Z = W.rademacher(n, N, seed)
    return X, y, Z, l, f, s


@pytest.mark.parametrize("precond", ["jacobi", "none"])
def test_cg_logdet_fp64_matches_oracle(precond):
    n, N = 3000, 8
    X, y, Z, l, f, s = _case(n, N, torch.float64)
    Xd, yd, Zd = to_dev(X, torch.float64), to_dev(y, torch.float64), to_dev(Z, torch.float64)
    loss_c, grad_c, info_c = hg.nlml(Xd, yd, Zd, 0, l, f, s, tol=1e-10, max_iter=3000,
                                     precond=precond, logdet="cg")
    loss_s, grad_s, info_s = hg.nlml(Xd, yd, Zd, 0, l, f, s, tol=1e-10, max_iter=3000,
                                     precond=precond, nsteps=60)
    K = oracle.khat_dense(X, 0, l, f, s)
    md = np.full(n, f * f + s) if precond == "jacobi" else None
    ref, per, its = oracle.cg_logdet(lambda P: K @ P, Z, 1e-10, 3000, mdiag=md)
    print("CG log-determinant %.12e, oracle %.12e, SLQ %.12e, iterations %s"
          % (info_c["logdet"], ref, info_s["logdet"], its))
    assert abs(info_c["logdet"] - ref) <= 1e-9 * abs(ref)
    # the gradient does not depend on how log|K̂| is estimated; the loss moves
    # by half the change of the log-determinant estimate
    np.testing.assert_array_equal(grad_c, grad_s)
    assert abs((loss_c - loss_s) - 0.5 * (info_c["logdet"] - info_s["logdet"])) <= 1e-9 * abs(loss_s)
    exact = oracle.logdet_exact(X, 0, l, f, s)
    se = per.std(ddof=1) / np.sqrt(N)
    assert abs(info_c["logdet"] - exact) <= 3 * se


def test_cg_logdet_fp32():
    # FP32 MatVecs.  Without reorthogonalisation the CG coefficients follow
    # the exact ones only until the first Ritz values converge; after that the
    # rounding of the MatVec input (2⁻²⁴ relative) is amplified (the oracle
    # shows the same when its MatVec input is rounded to float).  So the
    # parity is tight over the first 12 iterations, and at 60 iterations the
    # estimate is checked against the exact log-determinant statistically.
    n, N = 4000, 16
    X, y, Z, l, f, s = _case(n, N, torch.float32, seed=5)
    args = (to_dev(X, torch.float32), to_dev(y, torch.float32), to_dev(Z, torch.float32), 0, l,
            f, s)
    K = oracle.khat_dense(X, 0, l, f, s)
    md = np.full(n, f * f + s)
    _, _, info = hg.nlml(*args, tol=1e-6, max_iter=12, logdet="cg")
    ref, per, its = oracle.cg_logdet(lambda P: K @ P, Z, 1e-6, 12, mdiag=md)
    assert np.all(its == 12)
    print("FP32 CG log-determinant (12 its) %.9e, oracle %.9e" % (info["logdet"], ref))
    assert abs(info["logdet"] - ref) <= 1e-6 * abs(ref)
    _, _, info = hg.nlml(*args, tol=1e-6, max_iter=60, logdet="cg")
    ref, per, its = oracle.cg_logdet(lambda P: K @ P, Z, 1e-6, 60, mdiag=md)
    exact = np.linalg.slogdet(K)[1]
    se = per.std(ddof=1) / np.sqrt(N)
    print("FP32 CG log-determinant (60 its) %.9e, oracle %.9e, exact %.9e, SE %.2e"
          % (info["logdet"], ref, exact, se))
    assert abs(info["logdet"] - exact) <= 3 * se


@pytest.mark.parametrize("N", [8, 5, 2])
@pytest.mark.parametrize("kernel", [hg.GAUSSIAN, hg.MATERN32])
def test_hutchpp_fp64_matches_oracle(kernel, N):
    n = 2000
    X, y, Z, l, f, s = _case(n, N, torch.float64, seed=6)
    Xd, yd, Zd = to_dev(X, torch.float64), to_dev(y, torch.float64), to_dev(Z, torch.float64)
    loss, grad, info = hg.nlml(Xd, yd, Zd, kernel, l, f, s, tol=1e-12, max_iter=4000,
                               nsteps=40, trace="hutchpp")
    ref = oracle.nlml_grad_hutchpp(X, y, Z, kernel, l, f, s)
    exact = oracle.nlml_grad_exact(X, y, kernel, l, f, s)
    print("Hutch++ N=%d: %s oracle %s exact %s" % (N, grad, ref, exact))
    scale = np.abs(ref) + np.abs(exact)
    assert np.all(np.abs(grad - ref) <= 1e-7 * scale), (grad, ref)
    # the loss is the Hutchinson mode's (same α, same SLQ)
    loss_h, _, _ = hg.nlml(Xd, yd, Zd, kernel, l, f, s, tol=1e-12, max_iter=4000, nsteps=40)
    assert abs(loss - loss_h) <= 1e-9 * abs(loss_h)


def test_hutchpp_two_chunks_and_jacobi_off():
    # N = 42: 21 sketch columns, B2 has up to 126 columns (two PCG chunks).
    n, N = 1200, 42
    X, y, Z, l, f, s = _case(n, N, torch.float64, l=0.3, s=0.1, seed=7)
    loss, grad, info = hg.nlml(to_dev(X, torch.float64), to_dev(y, torch.float64),
                               to_dev(Z, torch.float64), 0, l, f, s, tol=1e-12, max_iter=3000,
                               nsteps=30, precond="none", trace="hutchpp")
    ref = oracle.nlml_grad_hutchpp(X, y, Z, 0, l, f, s, jacobi=False)
    exact = oracle.nlml_grad_exact(X, y, 0, l, f, s)
    scale = np.abs(ref) + np.abs(exact)
    assert np.all(np.abs(grad - ref) <= 1e-7 * scale), (grad, ref)


def test_hutchpp_fp32():
    n, N = 3000, 16
    X, y, Z, l, f, s = _case(n, N, torch.float32, seed=8)
    loss, grad, info = hg.nlml(to_dev(X, torch.float32), to_dev(y, torch.float32),
                               to_dev(Z, torch.float32), 0, l, f, s, tol=1e-7, max_iter=3000,
                               refine_every=10, nsteps=40, trace="hutchpp")
    ref = oracle.nlml_grad_hutchpp(X, y, Z, 0, l, f, s)
    exact = oracle.nlml_grad_exact(X, y, 0, l, f, s)
    scale = np.abs(ref) + np.abs(exact)
    print("FP32 Hutch++: %s oracle %s" % (grad, ref))
    assert np.all(np.abs(grad - ref) <= 2e-4 * scale), (grad, ref)
