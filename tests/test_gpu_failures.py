"""Failure handling forced from the host: an injected scratch-allocation
failure (the library's test hook) makes a call return HIGP_ERR_OOM, and the
next calls run normally and give the same results as before."""
import numpy as np
import pytest
import torch

import paper_2503_02259_amd as hg
from paper_2503_02259_amd import _lib, workloads as W
from helpers import as_prec, to_dev

pytestmark = pytest.mark.gpu


def test_injected_allocation_failure_reports_oom_and_recovers():
    p = W.random_problem(3001, 3, 11, k=5)
    X = to_dev(as_prec(p.X, torch.float32), torch.float32)
    V = to_dev(as_prec(p.extra["V"], torch.float32), torch.float32)
    ref = hg.kmatvec(X, V, 0, 0.2, 1.0, 0.05)
    x_ref, info_ref = hg.pcg(X, V, 0, 0.2, 1.0, 0.05, tol=1e-6, max_iter=500)
    try:
        for call in (lambda: hg.kmatvec(X, V, 0, 0.2, 1.0, 0.05),
                     lambda: hg.pcg(X, V, 0, 0.2, 1.0, 0.05, tol=1e-6, max_iter=500),
                     lambda: hg.slq_logdet(X, V, 0, 0.2, 1.0, 0.05, 10)):
            hg.debug_fail_allocs(1)
            with pytest.raises(hg.HigpError) as e:
                call()
            assert e.value.code == _lib.HIGP_ERR_OOM
    finally:
        hg.debug_fail_allocs(0)
    torch.cuda.synchronize()
    assert torch.equal(hg.kmatvec(X, V, 0, 0.2, 1.0, 0.05), ref)
    x, info = hg.pcg(X, V, 0, 0.2, 1.0, 0.05, tol=1e-6, max_iter=500)
    assert torch.equal(x, x_ref) and np.array_equal(info["iters"], info_ref["iters"])
