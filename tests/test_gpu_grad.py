"""Parity of the fused derivative MatVec (higp_kmatvec_grad) with the oracle."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_02259_amd as hg
from paper_2503_02259_amd import workloads as W
from helpers import TOL, as_prec, colrel, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kernel", [hg.GAUSSIAN, hg.MATERN32])
@pytest.mark.parametrize("n,d,k", [(1, 2, 1), (257, 3, 33), (1200, 3, 17), (800, 8, 64),
                                   (3001, 2, 2), (700, 20, 33), (400, 13, 5)])
def test_grad_matvec_matches_oracle(n, d, k, kernel, dtype):
    l = 0.3 * max(1.0, np.sqrt(d / 3.0))  # keep K away from the identity at high d
    p = W.random_problem(n, d, 40 + n + k, kernel=kernel, l=l, f=1.1, s=0.05, k=k)
    X = as_prec(p.X, dtype)
    V = as_prec(p.extra["V"], dtype)
    outs = hg.kmatvec_grad(to_dev(X, dtype), to_dev(V, dtype), kernel, p.l, p.f, p.s)
    refs = oracle.kmatvec_grad(X, V, kernel, p.l, p.f, p.s)
    for name, got, ref in zip(("kv", "dl", "df", "ds"), outs, refs):
        err = colrel(got.cpu().numpy(), ref)
        assert err.max() <= TOL[dtype], (name, err.max())


def test_grad_partial_outputs():
    p = W.random_problem(900, 3, 3, k=5)
    X = to_dev(p.X, torch.float64)
    V = to_dev(p.extra["V"], torch.float64)
    kv, dl, df, ds = hg.kmatvec_grad(X, V, 0, 0.3, 1.3, 0.05, want=("dl",))
    assert kv is None and df is None and ds is None
    ref = oracle.kmatvec_grad(p.X, p.extra["V"], 0, 0.3, 1.3, 0.05)[1]
    assert colrel(dl.cpu().numpy(), ref).max() <= 1e-10
