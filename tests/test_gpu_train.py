"""Training loop: Adam on Θ through GPRModel/GPLossFn against the oracle's
Adam with the Hutchinson gradient (same probes, exact solves)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2503_02259_amd import workloads as W
from paper_2503_02259_amd.autograd import GPRModel, train_gpr
from helpers import to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("transform", [None, "softplus"])
def test_training_trajectory_matches_oracle(transform):
    # n = 1,500 uniform in [0,1]^3, y = sin(2πx₀) + noise, 8 Rademacher
    # probes; FP64 with solves to 1e-11, so the GPU gradient equals the
    # estimator's exact value to ~1e-9 and the Adam paths must agree.
    n = 1500
    X = W.uniform_points(n, 3, 40)
    y = W.sine_targets(X, 40)
    Z = W.rademacher(n, 8, 40)
    theta0 = np.array([0.3, 1.0, 0.1])
    model = GPRModel(to_dev(X, torch.float64), to_dev(y, torch.float64), to_dev(Z, torch.float64),
                     kernel=0, l=theta0[0], f=theta0[1], s=theta0[2],
                     opts=dict(tol=1e-11, max_iter=5000, nsteps=20), transform=transform)
    hist = train_gpr(model, steps=15, lr=0.01)
    path, theta = oracle.train_gpr(X, y, Z, 0, theta0, steps=15, lr=0.01, transform=transform)
    got = np.array([[h["l"], h["f"], h["s"]] for h in hist])
    err = np.abs(got - np.array(path)).max()
    fin = np.array(list(model.get_params().values()))
    print("transform %s: max path difference %.2e, final θ %s vs %s" % (transform, err, fin, theta))
    np.testing.assert_allclose(got, np.array(path), rtol=1e-7, atol=1e-9)
    np.testing.assert_allclose(fin, theta, rtol=1e-7)
    assert not np.allclose(fin, theta0)
