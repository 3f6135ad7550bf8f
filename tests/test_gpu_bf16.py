"""BF16 precision form (kernel tile and V in bfloat16, FP32 accumulation).

The HIP path is compared with the oracle's emulated-BF16 MatVec (K and V
rounded to bfloat16 with RNE, exact products, FP64 sums).  The GPU rounds
FP32 kernel values (from an FP32 norm-expansion distance) while the oracle
rounds FP64 ones, so a small fraction of roundings differ by one bfloat16
ulp: the bar is 1e-3 normwise against the emulation, while the error
against the FP64 product (≈1e-3–1e-2) is reported.  Where every kernel value
is exactly representable (l → ∞: all ones) the two must agree to FP32
accumulation accuracy."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_02259_amd as hg
from paper_2503_02259_amd import workloads as W
from helpers import as_prec, colrel, colrel_cond, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kernel", [hg.GAUSSIAN, hg.MATERN32])
@pytest.mark.parametrize("n,d,k", [(1, 1, 1), (129, 3, 33), (1000, 8, 33), (700, 2, 17),
                                   (2500, 5, 64), (333, 7, 32)])
def test_bf16_matches_emulated_oracle(n, d, k, kernel):
    p = W.random_problem(n, d, 300 + n + d, kernel=kernel, l=0.3, f=1.1, s=1e-3, k=k)
    X = as_prec(p.X, torch.float32)
    V = as_prec(p.extra["V"], torch.float32)
    Y = hg.kmatvec(to_dev(X, torch.float32), to_dev(V, torch.float32), kernel, p.l, p.f, p.s,
                   precision="bf16").cpu().numpy()
    emu = oracle.kmatvec_bf16_emulated(X, V, kernel, p.l, p.f, p.s)
    exact = oracle.kmatvec(X, V, kernel, p.l, p.f, p.s)
    e_emu = colrel(Y, emu).max()
    e_exact = colrel(Y, exact).max()
    print("n=%d d=%d k=%d: vs emulated %.2e, vs FP64 %.2e" % (n, d, k, e_emu, e_exact))
    assert e_emu <= 1e-3
    assert e_exact <= 5e-2


def test_bf16_exactly_representable_limit():
    n, f, s = 3000, 1.0, 1e-3
    X = as_prec(W.uniform_points(n, 8, 91), torch.float32)
    V = as_prec(W.gaussian_vectors(n, 33, 91), torch.float32)
    Y = hg.kmatvec(to_dev(X, torch.float32), to_dev(V, torch.float32), 0, 1e8, f, s,
                   precision="bf16").cpu().numpy()
    Vb = oracle.round_bf16(V)
    ref = f * f * np.ones((n, 1)) * Vb.sum(0) + s * V
    refabs = f * f * np.ones((n, 1)) * np.abs(Vb).sum(0) + s * np.abs(V)
    assert colrel_cond(Y, ref, refabs).max() <= 1e-6


def test_bf16_mixture_subsample():
    # Precision-form workload (16-component Gaussian mixture in [0,1]^8,
    # σ = 0.05, l = 0.3, s = 1e-3, k = 33) on its seeded 20,000-point
    # subsample: BF16 vs emulation, and the FP32 form vs FP64 for contrast.
    prob = W.workload_bf16_mixture(n=60_000, sub=20_000)
    idx = prob.extra["sub"]
    idx = idx[idx < prob.X.shape[0]][:20_000]
    X = as_prec(prob.X[idx], torch.float32)
    V = as_prec(prob.extra["V"][idx], torch.float32)
    Xd, Vd = to_dev(X, torch.float32), to_dev(V, torch.float32)
    Yb = hg.kmatvec(Xd, Vd, 0, prob.l, prob.f, prob.s, precision="bf16").cpu().numpy()
    Yf = hg.kmatvec(Xd, Vd, 0, prob.l, prob.f, prob.s).cpu().numpy()
    rows = slice(0, 400)
    emu = oracle.kmatvec_bf16_emulated(X, V, 0, prob.l, prob.f, prob.s, workers=8)
    exact = oracle.kmatvec(X, V, 0, prob.l, prob.f, prob.s, workers=8)
    e_emu, e_b, e_f = colrel(Yb, emu).max(), colrel(Yb, exact).max(), colrel(Yf, exact).max()
    print("mixture subsample: bf16 vs emulated %.2e, bf16 vs FP64 %.2e, fp32 vs FP64 %.2e"
          % (e_emu, e_b, e_f))
    assert e_emu <= 1e-3 and e_f <= 1e-5


def test_bf16_pcg_with_refinement():
    # Refinement with a BF16 inner MatVec converges when κ(K̂)·u_bf16 < 1
    # (u_bf16 = 2⁻⁸): here n = 4,000 uniform points in [0,1]^3, l = 0.1,
    # s = 0.5, so λ_max ≈ n(2πl²)^{3/2} ≈ 63 and κ ≈ 130.  The residual is
    # replaced every 10 iterations from an FP64 MatVec of the FP64 iterate,
    # which then meets the tolerance in the true residual.
    n = 4000
    X = as_prec(W.uniform_points(n, 3, 92), torch.float32)
    B = as_prec(W.gaussian_vectors(n, 3, 92), torch.float32)
    x, x64, info = hg.pcg(to_dev(X, torch.float32), to_dev(B, torch.float32), 0, 0.1, 1.0, 0.5,
                          tol=1e-6, max_iter=3000, refine_every=10, precision="bf16",
                          return_fp64=True)
    assert info["converged"].all(), info
    r = B - oracle.kmatvec(X, x64.cpu().numpy(), 0, 0.1, 1.0, 0.5, workers=8)
    tr = np.linalg.norm(r, axis=0) / np.linalg.norm(B, axis=0)
    print("bf16 + refinement: iters", info["iters"], "true residual", tr)
    assert np.all(tr <= 1.1e-6)


def test_bf16_pcg_ill_conditioned_reports_non_convergence():
    # κ·u_bf16 ≫ 1 (l = 0.2, s = 0.05, κ ≈ 1e4): the BF16 operator is too far
    # from K̂ for refinement to converge.  The call must still return normally
    # with converged = 0 and the iteration cap, never an error.
    n = 4000
    X = as_prec(W.uniform_points(n, 3, 92), torch.float32)
    B = as_prec(W.gaussian_vectors(n, 2, 92), torch.float32)
    x, info = hg.pcg(to_dev(X, torch.float32), to_dev(B, torch.float32), 0, 0.2, 1.0, 0.05,
                     tol=1e-6, max_iter=300, refine_every=10, precision="bf16")
    assert info["iters"].max() <= 300
    assert np.all(np.isfinite(x.cpu().numpy())) or not info["converged"].all()
