"""Parity of the HIP MatVec (higp_kmatvec) with the FP64 oracle.

Tolerances: ≤ 1e-10 normwise relative per column for the FP64 form and
≤ 1e-5 for the FP32 form, against the oracle evaluated on the same
(float32-rounded) inputs."""
import numpy as np
import pytest
import torch

import oracle
import paper_2503_02259_amd as hg
from paper_2503_02259_amd import workloads as W
from helpers import TOL, as_prec, colrel, colrel_cond, oracle_rows, to_dev

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (2, 3, 2), (127, 3, 33), (1001, 3, 17), (300, 1, 5), (517, 2, 64),
          (700, 8, 31), (640, 5, 32), (333, 4, 63), (999, 3, 34), (260, 7, 10), (2000, 3, 1),
          (777, 3, 49)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kernel", [hg.GAUSSIAN, hg.MATERN32])
@pytest.mark.parametrize("n,d,k", SHAPES)
def test_kmatvec_matches_oracle(n, d, k, kernel, dtype):
    seed = n * 131 + d * 7 + k
    p = W.random_problem(n, d, seed, kernel=kernel, l=0.35, f=1.3, s=0.05, k=k)
    X = as_prec(p.X, dtype)
    V = as_prec(p.extra["V"], dtype)
    Y = hg.kmatvec(to_dev(X, dtype), to_dev(V, dtype), kernel, p.l, p.f, p.s)
    ref = oracle.kmatvec(X, V, kernel, p.l, p.f, p.s)
    err = colrel(Y.cpu().numpy(), ref)
    assert err.max() <= TOL[dtype], (err.max(), n, d, k)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_vector_input_and_repeatability(dtype):
    p = W.random_problem(3000, 3, 5, k=1)
    X = to_dev(as_prec(p.X, dtype), dtype)
    v = to_dev(as_prec(p.extra["V"][:, 0], dtype), dtype)
    y1 = hg.kmatvec(X, v, hg.GAUSSIAN, 0.2, 1.0, 0.01)
    y2 = hg.kmatvec(X, v, hg.GAUSSIAN, 0.2, 1.0, 0.01)
    assert y1.shape == (3000,)
    assert torch.equal(y1, y2)        # deterministic: no atomics, fixed order


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kernel", [hg.GAUSSIAN, hg.MATERN32])
def test_limits(kernel, dtype):
    n, f, s = 1500, 1.2, 0.02
    X = as_prec(W.uniform_points(n, 3, 77), dtype)
    V = as_prec(W.gaussian_vectors(n, 3, 77), dtype)
    Y = hg.kmatvec(to_dev(X, dtype), to_dev(V, dtype), kernel, 1e8, f, s).cpu().numpy()
    ref = f * f * np.ones((n, 1)) * V.sum(0) + s * V
    # Σ_j v_j of N(0,1) entries cancels heavily (|Σv| ≪ Σ|v|), so the error is
    # measured against the size of the summands, f²·Σ|v| + s·|v|.
    refabs = f * f * np.ones((n, 1)) * np.abs(V).sum(0) + s * np.abs(V)
    assert colrel_cond(Y, ref, refabs).max() <= TOL[dtype]
    G = np.stack(np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij"), -1).reshape(-1, 3) * 0.1
    V2 = as_prec(W.gaussian_vectors(G.shape[0], 2, 78), dtype)
    Y2 = hg.kmatvec(to_dev(as_prec(G, dtype), dtype), to_dev(V2, dtype), kernel, 1e-3, f, s).cpu().numpy()
    assert colrel(Y2, (f * f + s) * V2).max() <= TOL[dtype]


@pytest.mark.parametrize("kernel", [hg.GAUSSIAN, hg.MATERN32])
def test_full_size_fp32_sampled_rows(kernel):
    # n = 100,000 uniform points in [0,1]^3, l = 0.1, f = 1, s = 1e-2, k = 33:
    # the benchmark's launch; rows checked against the oracle slice by slice,
    # including the ragged last row tile.
    prob = W.workload_fp32_matvec(kernel=kernel)
    X = as_prec(prob.X, torch.float32)
    V = as_prec(prob.extra["V"], torch.float32)
    Y = hg.kmatvec(to_dev(X, torch.float32), to_dev(V, torch.float32), kernel, prob.l, prob.f,
                   prob.s).cpu().numpy()
    n = X.shape[0]
    for rows in (slice(0, 97), slice(49_950, 50_130), slice(n - 160, n)):
        ref = oracle_rows(X, V, kernel, prob.l, prob.f, prob.s, rows)
        assert colrel(Y[rows], ref).max() <= 1e-5
    # property at any size: ⟨1, K̂V⟩ = ⟨K̂1, V⟩ (symmetry), checked in FP64
    ones = np.ones((n, 1))
    K1 = hg.kmatvec(to_dev(X, torch.float64), to_dev(ones, torch.float64), kernel, prob.l,
                    prob.f, prob.s).cpu().numpy()
    lhs = Y.sum(0)
    rhs = (K1 * V).sum(0)
    assert np.all(np.abs(lhs - rhs) <= 1e-5 * np.abs(K1).sum() * np.abs(V).max(0))


@pytest.mark.parametrize("kernel", [hg.GAUSSIAN, hg.MATERN32])
def test_full_size_fp64_sampled_rows(kernel):
    # The FP64 MatVec at n = 100,000, d = 3, k = 33 (the residual replacement
    # of the refined solves at that size): rows at both ends and in the middle
    # against the oracle, to the FP64 bar.
    prob = W.workload_fp32_matvec(kernel=kernel)
    X, V = prob.X, prob.extra["V"]
    Y = hg.kmatvec(to_dev(X, torch.float64), to_dev(V, torch.float64), kernel, prob.l, prob.f,
                   prob.s).cpu().numpy()
    n = X.shape[0]
    for rows in (slice(0, 64), slice(n // 2 - 40, n // 2 + 40), slice(n - 100, n)):
        ref = oracle_rows(X, V, kernel, prob.l, prob.f, prob.s, rows)
        assert colrel(Y[rows], ref).max() <= 1e-10


HIGH_D = [(700, 9, 33), (513, 12, 5), (1001, 16, 64), (300, 17, 1), (1500, 20, 33),
          (257, 25, 17), (900, 32, 2)]


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("kernel", [hg.GAUSSIAN, hg.MATERN32])
@pytest.mark.parametrize("n,d,k", HIGH_D)
def test_kmatvec_high_dimension_matches_oracle(n, d, k, kernel, dtype):
    # Up to d = 32 (the paper's on-the-fly runs use d = 20).  The length-scale
    # grows with √d so that the kernel matrix stays far from the identity.
    seed = n * 17 + d
    l = 0.35 * np.sqrt(d / 3.0)
    p = W.random_problem(n, d, seed, kernel=kernel, l=l, f=1.3, s=0.05, k=k)
    X = as_prec(p.X, dtype)
    V = as_prec(p.extra["V"], dtype)
    Y = hg.kmatvec(to_dev(X, dtype), to_dev(V, dtype), kernel, p.l, p.f, p.s)
    ref = oracle.kmatvec(X, V, kernel, p.l, p.f, p.s)
    offdiag = oracle.kmatvec(X, V, kernel, p.l, p.f, 0.0) - p.f ** 2 * V
    assert np.linalg.norm(offdiag) > 0.1 * np.linalg.norm(ref)  # not just the diagonal
    err = colrel(Y.cpu().numpy(), ref)
    assert err.max() <= TOL[dtype], (err.max(), n, d, k)


def test_bf16_and_server_reject_high_dimension():
    p = W.random_problem(100, 12, 3, k=4)
    X = to_dev(as_prec(p.X, torch.float32), torch.float32)
    V = to_dev(as_prec(p.extra["V"], torch.float32), torch.float32)
    for prec in ("bf16", "bf16x3"):
        with pytest.raises(hg.HigpError) as e:
            hg.kmatvec(X, V, 0, 0.5, 1.0, 0.1, precision=prec)
        assert e.value.code == -2
    from paper_2503_02259_amd.serve import Server
    srv = Server(hbm_budget=1 << 30, max_active=2)
    with pytest.raises(hg.HigpError) as e:
        srv.submit(X, V[:, 0].contiguous())
    assert e.value.code == -2
    srv.close()


SYM = [(40_000, 3, 1), (40_000, 3, 2), (33_001, 1, 1), (35_000, 2, 2), (32_768, 4, 1),
       (50_000, 4, 2), (40_000, 8, 1), (36_001, 5, 1), (33_000, 7, 1)]


@pytest.mark.parametrize("kernel", [hg.GAUSSIAN, hg.MATERN32])
@pytest.mark.parametrize("n,d,k", SYM)
def test_symmetric_fp32_matvec(n, d, k, kernel):
    # k ≤ 2 (d ≤ 4) or k = 1 (d ≤ 8), n ≥ 32768: each kernel value of a block pair serves both
    # output blocks.  Rows checked against the oracle where super blocks
    # (1024 points) and tiles (128) meet, at both ends and in the ragged last
    # block; every row against the full-block form.
    X = as_prec(W.uniform_points(n, d, 700 + d), torch.float32)
    V = as_prec(W.rng(700 + k, 4).standard_normal((n, k)), torch.float32)
    l, f, s = 0.15, 1.1, 0.02
    Xd, Vd = to_dev(X, torch.float32), to_dev(V, torch.float32)
    Y = hg.kmatvec(Xd, Vd, kernel, l, f, s).cpu().numpy()
    Yf = hg.kmatvec(Xd, Vd, kernel, l, f, s, symmetric=False).cpu().numpy()
    for rows in (slice(0, 130), slice(1000, 1160), slice(n // 2 - 70, n // 2 + 70),
                 slice(n - 200, n)):
        ref = oracle_rows(X, V, kernel, l, f, s, rows)
        err = colrel(Y[rows], ref).max()
        assert err <= 1e-5, (rows, err)
    diff = colrel(Y, Yf).max()
    print("n=%d d=%d k=%d: symmetric vs full-block %.2e" % (n, d, k, diff))
    assert diff <= 2e-6
    # deterministic
    assert np.array_equal(Y, hg.kmatvec(Xd, Vd, kernel, l, f, s).cpu().numpy())
