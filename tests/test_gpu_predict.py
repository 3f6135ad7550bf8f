"""GP prediction: the rectangular on-the-fly MatVec f²·k(Xq, X)·V and the
predictive mean and latent variance, against the oracle (dense FP64)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_02259_amd as hg
from paper_2503_02259_amd import workloads as W
from helpers import TOL, as_prec, colrel, colrel_cond, to_dev

pytestmark = pytest.mark.gpu


def _pts(n, d, seed, stream=0):
    return W.rng(600 + seed, stream).random((n, d))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kernel", [hg.GAUSSIAN, hg.MATERN32])
@pytest.mark.parametrize("m,n,d,k", [(1, 1, 1, 1), (130, 257, 3, 33), (1000, 700, 8, 5),
                                     (64, 3000, 2, 64), (5000, 100, 3, 1), (333, 2049, 5, 17),
                                     (500, 1200, 20, 3)])
def test_cross_matvec_matches_oracle(m, n, d, k, kernel, dtype):
    seed = m + n + d + k
    X = as_prec(_pts(n, d, seed), dtype)
    Xq = as_prec(_pts(m, d, seed, 1), dtype)
    V = as_prec(W.rng(600 + seed, 4).standard_normal((n, k)), dtype)
    l, f = 0.3 * max(1.0, np.sqrt(d / 3.0)), 1.2
    Y = hg.kmatvec_cross(to_dev(Xq, dtype), to_dev(X, dtype), to_dev(V, dtype), kernel, l, f)
    ref = oracle.kmatvec_cross(Xq, X, V, kernel, l, f, workers=8)
    err = colrel(Y.cpu().numpy(), ref).max()
    print("m=%d n=%d d=%d k=%d %s: %.2e" % (m, n, d, k, dtype, err))
    assert err <= TOL[dtype]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_cross_square_case_is_the_matvec_without_noise(dtype):
    X = as_prec(_pts(1500, 3, 7), dtype)
    V = as_prec(W.rng(607, 4).standard_normal((1500, 6)), dtype)
    l, f, s = 0.2, 0.9, 0.05
    Xd, Vd = to_dev(X, dtype), to_dev(V, dtype)
    Yc = hg.kmatvec_cross(Xd, Xd, Vd, 0, l, f).double().cpu().numpy() + s * V
    Ys = hg.kmatvec(Xd, Vd, 0, l, f, s).double().cpu().numpy()
    assert colrel(Yc, Ys).max() <= TOL[dtype]


@pytest.mark.parametrize("kernel", [hg.GAUSSIAN, hg.MATERN32])
def test_prediction_fp64_matches_oracle(kernel):
    # c1-like training set (n = 2,000 uniform in [0,1]^3, l = 0.5, s = 0.01)
    # and 150 query points; solves to 1e-12 so that the solver error is far
    # below the bar.
    p = W.workload_fp64_small()
    X, y = p.X, p.extra["y"]
    Xq = _pts(150, 3, 11)
    mean, var, info = hg.gpr_predict(to_dev(X, torch.float64), to_dev(y, torch.float64),
                                     to_dev(Xq, torch.float64), kernel, p.l, p.f, p.s, tol=1e-12,
                                     max_iter=5000, want_var=True)
    rm, rv = oracle.gpr_predict(X, y, Xq, kernel, p.l, p.f, p.s)
    em = np.linalg.norm(mean.cpu().numpy() - rm) / np.linalg.norm(rm)
    ev = np.abs(var.cpu().numpy() - rv).max()
    print("FP64 prediction: mean %.2e, var %.2e (abs), α iterations %d" % (em, ev, info["pcg_iters"]))
    assert em <= 1e-8 and ev <= 1e-8


def test_prediction_fp32_matches_oracle():
    # The same in FP32: α is limited by the FP32 MatVec (≈1e-7 relative per
    # product, amplified by the solve), so the bar is 1e-3.
    p = W.workload_fp64_small()
    X = as_prec(p.X, torch.float32)
    y = as_prec(p.extra["y"], torch.float32)
    Xq = as_prec(_pts(150, 3, 11), torch.float32)
    mean, var, _ = hg.gpr_predict(to_dev(X, torch.float32), to_dev(y, torch.float32),
                                  to_dev(Xq, torch.float32), 0, p.l, p.f, p.s, tol=1e-6,
                                  max_iter=3000, want_var=True)
    rm, rv = oracle.gpr_predict(X, y, Xq, 0, p.l, p.f, p.s)
    em = np.linalg.norm(mean.cpu().numpy() - rm) / np.linalg.norm(rm)
    ev = np.abs(var.cpu().numpy() - rv).max()
    print("FP32 prediction: mean %.2e, var %.2e (abs)" % (em, ev))
    assert em <= 1e-3 and ev <= 1e-3


@pytest.mark.parametrize("kernel", [hg.GAUSSIAN, hg.MATERN32])
def test_prediction_nystrom_rank100_d20_matches_oracle(kernel):
    # The paper's prediction setting in small: d = 20 z-scored points, a
    # rank-100 preconditioner; FP64 and solved to 1e-11, so the mean must
    # agree with the dense posterior whatever the preconditioner is.
    Xtr, ytr, Xte, _ = W.workload_paper_shape(n=1500, m=200)
    l, f, s = 3.0, 1.0, 0.05
    mean, var, info = hg.gpr_predict(to_dev(Xtr, torch.float64), to_dev(ytr, torch.float64),
                                     to_dev(Xte, torch.float64), kernel, l, f, s, tol=1e-11,
                                     max_iter=2000, precond="nystrom", rank=100, want_var=True)
    rm, rv = oracle.gpr_predict(Xtr, ytr, Xte, kernel, l, f, s)
    em = np.linalg.norm(mean.cpu().numpy() - rm) / np.linalg.norm(rm)
    ev = np.abs(var.cpu().numpy() - rv).max()
    print("Nyström-100 d=20 prediction: mean %.2e, var %.2e, α iterations %d"
          % (em, ev, info["pcg_iters"]))
    assert em <= 1e-8 and ev <= 1e-8


def test_prediction_far_queries_give_the_prior():
    X = _pts(500, 2, 12)
    y = np.sin(6 * X[:, 0])
    Xq = _pts(70, 2, 13) + 50.0
    f = 1.3
    mean, var, _ = hg.gpr_predict(to_dev(X, torch.float64), to_dev(y, torch.float64),
                                  to_dev(Xq, torch.float64), 0, 0.1, f, 0.01, tol=1e-10,
                                  want_var=True)
    assert np.abs(mean.cpu().numpy()).max() == 0.0
    np.testing.assert_allclose(var.cpu().numpy(), f * f, rtol=1e-14)


def test_prediction_full_size_sampled():
    # Paper-scale prediction: the n = 100,000 FP32 workload, 4,096 query
    # points, mean only.  α comes from the GPU solve; the mean at 64 sampled
    # query points is checked against the oracle's rectangular product with
    # that same α (the path under test is the rectangular MatVec at size).
    prob = W.workload_fp32_matvec()
    X = as_prec(prob.X, torch.float32)
    y = as_prec(prob.extra["y"], torch.float32)
    Xq = as_prec(_pts(4096, 3, 14), torch.float32)
    Xd, Xqd = to_dev(X, torch.float32), to_dev(Xq, torch.float32)
    alpha, info = hg.pcg(Xd, to_dev(y, torch.float32), 0, prob.l, prob.f, prob.s, tol=1e-4,
                         max_iter=400)
    mean = hg.kmatvec_cross(Xqd, Xd, alpha, 0, prob.l, prob.f).cpu().numpy()
    idx = W.rng(614, 3).choice(4096, 64, replace=False)
    a64 = alpha.double().cpu().numpy()
    ref = oracle.kmatvec_cross(Xq[idx], X, a64, 0, prob.l, prob.f, workers=8)
    refabs = oracle.kmatvec_cross(Xq[idx], X, np.abs(a64), 0, prob.l, prob.f, workers=8)
    # α oscillates, so the product cancels (‖K*α‖ ≪ ‖|K*||α|‖): the error is
    # measured against the magnitude of the summands.
    err = colrel_cond(mean[idx], ref, refabs).max()
    print("full-size rectangular MatVec, sampled rows: %.2e (cancellation %.1f)"
          % (err, np.linalg.norm(refabs) / np.linalg.norm(ref)))
    assert err <= 1e-5
    m2, _, inf2 = hg.gpr_predict(Xd, to_dev(y, torch.float32), Xqd, 0, prob.l, prob.f, prob.s,
                                 tol=1e-4, max_iter=400)
    np.testing.assert_array_equal(m2.cpu().numpy(), mean)
