"""Pins of the oracle's training loop (CPU): Adam against torch.optim.Adam,
the softplus transform against torch's, and descent of the exact NLML."""
import numpy as np
import torch

import oracle
from paper_2503_02259_amd import workloads as W


def test_adam_matches_torch():
    g = W.rng(30, 0).standard_normal((40, 3)) * np.array([1.0, 1e-3, 50.0])
    x0 = np.array([0.5, -1.0, 2.0])
    opt = oracle.Adam(x0, lr=0.01)
    p = torch.nn.Parameter(torch.tensor(x0, dtype=torch.float64))
    topt = torch.optim.Adam([p], lr=0.01)
    for gi in g:
        opt.step(gi)
        p.grad = torch.tensor(gi, dtype=torch.float64)
        topt.step()
    np.testing.assert_allclose(opt.x, p.detach().numpy(), rtol=1e-14, atol=1e-15)


def test_softplus_and_inverse():
    r = np.linspace(-30, 20, 51)  # torch switches to the identity above 20
    np.testing.assert_allclose(oracle.softplus(r),
                               torch.nn.functional.softplus(torch.tensor(r)).numpy(), rtol=1e-14)
    t = np.array([1e-6, 0.01, 0.5, 3.0, 40.0])
    np.testing.assert_allclose(oracle.softplus(oracle.softplus_inv(t)), t, rtol=1e-12)


def test_training_descends_the_exact_nlml():
    # With all n unit vectors scaled by √n as probes the Hutchinson trace is
    # exact, so the gradient is the exact one and Adam must lower the exact
    # NLML over the run.
    n = 60
    g = W.rng(31, 0)
    X = g.random((n, 2))
    y = np.sin(4 * X[:, 0]) + 0.05 * g.standard_normal(n)
    Z = np.sqrt(n) * np.eye(n)
    theta0 = np.array([0.6, 1.0, 0.2])
    path, theta = oracle.train_gpr(X, y, Z, oracle.GAUSSIAN, theta0, steps=30, lr=0.05,
                                   transform="softplus")
    L0 = oracle.nlml_exact(X, y, oracle.GAUSSIAN, *theta0)
    L1 = oracle.nlml_exact(X, y, oracle.GAUSSIAN, *theta)
    assert L1 < L0 - 1e-3
    exact = oracle.nlml_grad_exact(X, y, oracle.GAUSSIAN, *theta0)
    hutch = oracle.nlml_grad_hutchinson(X, y, Z, oracle.GAUSSIAN, *theta0)
    np.testing.assert_allclose(hutch, exact, rtol=1e-9, atol=1e-12)
