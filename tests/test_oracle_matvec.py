"""Pins of the oracle's MatVecs (CPU only): closed-form limits, adjointness,
an independent kernel-matrix implementation (scikit-learn), finite
differences for the derivative MatVecs, and torch's bfloat16 rounding."""
import numpy as np
import pytest
import torch
from sklearn.gaussian_process.kernels import RBF, Matern

import oracle
from paper_2503_02259_amd import workloads as W


def _prob(n=90, d=3, k=5, seed=0):
    X = W.rng(700 + seed, 0).random((n, d))
    V = W.rng(700 + seed, 4).standard_normal((n, k))
    return X, V


@pytest.mark.parametrize("kern", [oracle.GAUSSIAN, oracle.MATERN32])
def test_matches_sklearn_dense_product(kern):
    X, V = _prob(64, 3, 7, kern)
    l, f, s = 0.25, 1.4, 0.03
    Kref = (RBF(l) if kern == oracle.GAUSSIAN else Matern(l, nu=1.5))(X)
    ref = f * f * (Kref @ V) + s * V
    np.testing.assert_allclose(oracle.kmatvec(X, V, kern, l, f, s, block=17), ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("kern", [oracle.GAUSSIAN, oracle.MATERN32])
def test_limits(kern):
    X, V = _prob(80, 3, 4, 2)
    f, s = 1.2, 0.05
    Y = oracle.kmatvec(X, V, kern, 1e8, f, s)
    np.testing.assert_allclose(Y, f * f * np.ones((80, 1)) * V.sum(0) + s * V, rtol=1e-12, atol=1e-11)
    G = np.stack(np.meshgrid(np.arange(5), np.arange(5), np.arange(3), indexing="ij"), -1).reshape(-1, 3) * 0.1
    V2 = W.rng(3, 4).standard_normal((G.shape[0], 3))
    np.testing.assert_allclose(oracle.kmatvec(G, V2, kern, 1e-3, f, s), (f * f + s) * V2, rtol=1e-14, atol=1e-60)


def test_adjoint_and_block_independence():
    X, V = _prob(150, 2, 3, 4)
    U = W.rng(5, 4).standard_normal((150, 3))
    args = (oracle.GAUSSIAN, 0.2, 0.9, 0.01)
    KV = oracle.kmatvec(X, V, *args)
    KU = oracle.kmatvec(X, U, *args)
    assert abs(np.sum(U * KV) - np.sum(KU * V)) <= 1e-12 * np.abs(U).sum() * np.abs(KV).max()
    np.testing.assert_array_equal(oracle.kmatvec(X, V, *args, block=512),
                                  oracle.kmatvec(X, V, *args, block=512, workers=4))
    np.testing.assert_allclose(oracle.kmatvec(X, V, *args, block=7), KV, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("kern", [oracle.GAUSSIAN, oracle.MATERN32])
def test_grad_matvec_central_fd(kern):
    X, V = _prob(60, 3, 4, 6)
    l, f, s = 0.3, 1.1, 0.02
    KV, DL, DF, DS = oracle.kmatvec_grad(X, V, kern, l, f, s)
    np.testing.assert_allclose(KV, oracle.kmatvec(X, V, kern, l, f, s), rtol=1e-13, atol=1e-13)
    for name, out, base in (("l", DL, l), ("f", DF, f), ("s", DS, s)):
        h = 1e-5 * base
        p = dict(l=l, f=f, s=s)
        pp, pm = dict(p), dict(p)
        pp[name] += h
        pm[name] -= h
        fd = (oracle.kmatvec(X, V, kern, pp["l"], pp["f"], pp["s"])
              - oracle.kmatvec(X, V, kern, pm["l"], pm["f"], pm["s"])) / (2 * h)
        np.testing.assert_allclose(out, fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())


def test_grad_matvec_large_l_vanishes():
    X, V = _prob(40, 3, 2, 7)
    _, DL, _, _ = oracle.kmatvec_grad(X, V, oracle.GAUSSIAN, 1e6, 1.0, 0.1)
    assert np.abs(DL).max() < 1e-15


def test_round_bf16_known_values_and_torch():
    one = 1.0
    assert oracle.round_bf16(np.array([one + 2.0 ** -8]))[0] == 1.0            # tie -> even
    assert oracle.round_bf16(np.array([one + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6
    assert oracle.round_bf16(np.array([one + 2.0 ** -8 + 2.0 ** -30]))[0] == 1.0 + 2.0 ** -7
    assert oracle.round_bf16(np.array([-(one + 2.0 ** -8)]))[0] == -1.0
    x = W.rng(8, 4).standard_normal(10000).astype(np.float32).astype(np.float64)
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.round_bf16(x), ref)


def test_bf16_emulated_matches_torch_rounding():
    X, V = _prob(70, 3, 3, 9)
    l, f, s = 0.3, 1.0, 0.01
    got = oracle.kmatvec_bf16_emulated(X, V, oracle.GAUSSIAN, l, f, s, block=32)
    K = RBF(l)(X)
    Kb = torch.from_numpy(K.astype(np.float32)).to(torch.bfloat16).double().numpy()
    Vb = torch.from_numpy(V.astype(np.float32)).to(torch.bfloat16).double().numpy()
    # K in float64 vs float32 before the bf16 rounding differs only at near-ties:
    # compare with a bound of one bf16 ulp per kernel value.
    ref = f * f * (Kb @ Vb) + s * V
    bound = f * f * (2.0 ** -8) * (np.abs(K) @ np.abs(Vb))
    assert np.all(np.abs(got - ref) <= bound + 1e-14)
    # and the result is within bf16 accuracy of the FP64 product
    exact = oracle.kmatvec(X, V, oracle.GAUSSIAN, l, f, s)
    assert np.linalg.norm(got - exact) / np.linalg.norm(exact) < 2e-2


def test_split_bf16_exact_for_16_bit_values_and_bounded_otherwise():
    g = W.rng(8, 5)
    # values with at most 16 significant bits are carried exactly by hi + lo
    m = g.integers(2 ** 15, 2 ** 16, size=5000).astype(np.float64)
    a = m * np.ldexp(1.0, g.integers(-40, 10, size=5000)) * g.choice([-1.0, 1.0], 5000)
    hi, lo = oracle.split_bf16(a)
    np.testing.assert_array_equal(hi + lo, a)
    # general values: |a − hi − lo| ≤ 2⁻¹⁶|a|, hi and lo are bfloat16 values
    a = g.standard_normal(20000) * np.exp(g.uniform(-20, 5, 20000))
    hi, lo = oracle.split_bf16(a)
    assert np.all(np.abs(a - hi - lo) <= 2.0 ** -16 * np.abs(a))
    assert np.all(np.abs(a - hi) <= 2.0 ** -8 * np.abs(a))
    for part in (hi, lo):
        bf = torch.from_numpy(part).to(torch.bfloat16).double().numpy()
        np.testing.assert_array_equal(bf, part)
    # hi is torch's bfloat16 rounding of the (float32-representable) input
    a32 = a.astype(np.float32).astype(np.float64)
    hi32, _ = oracle.split_bf16(a32)
    np.testing.assert_array_equal(hi32, torch.from_numpy(a32.astype(np.float32)).to(torch.bfloat16).double().numpy())


@pytest.mark.parametrize("kern", [oracle.GAUSSIAN, oracle.MATERN32])
def test_bf16x3_emulated_within_split_bound(kern):
    """Elementwise bound of the three-term split product against the FP64
    product: |Y − Y*| ≤ 3.1·u²·f²·(|K|·|V|), u = 2⁻⁸.  Dropping either cross
    term, or swapping hi and lo, breaks it by a factor ~2⁸."""
    X, V = _prob(80, 3, 4, 11)
    l, f, s = 0.35, 1.3, 0.02
    got = oracle.kmatvec_bf16x3_emulated(X, V, kern, l, f, s, block=32)
    K = (RBF(l) if kern == oracle.GAUSSIAN else Matern(l, nu=1.5))(X)
    exact = f * f * (K @ V) + s * V
    bound = 3.1 * 2.0 ** -16 * f * f * (np.abs(K) @ np.abs(V))
    assert np.all(np.abs(got - exact) <= bound + 1e-14)
    # the bound is not vacuous: the single-BF16 form exceeds it
    single = oracle.kmatvec_bf16_emulated(X, V, kern, l, f, s, block=32)
    assert np.any(np.abs(single - exact) > 20 * bound)
    # Rademacher vectors are exact in bfloat16 (V_lo = 0): then the result is
    # (K_hi + K_lo)·V, within u²·|K|·|V| of the exact product
    Z = W.rademacher(80, 3, 11)
    gz = oracle.kmatvec_bf16x3_emulated(X, Z, kern, l, f, 0.0, block=32)
    assert np.all(np.abs(gz - f * f * (K @ Z)) <= 1.01 * 2.0 ** -16 * f * f * (np.abs(K) @ np.abs(Z)) + 1e-14)


def test_row_subsets_equal_full_rows():
    """``rows`` only restricts the output: each subset equals the same rows of
    the full result, across block boundaries and at the end, up to the
    rounding of the row-block products (BLAS may round a row differently with
    another number of rows in its block)."""
    X, V = _prob(300, 3, 5, 21)
    for fn in (oracle.kmatvec, oracle.kmatvec_bf16_emulated, oracle.kmatvec_bf16x3_emulated):
        full = fn(X, V, oracle.GAUSSIAN, 0.3, 1.1, 0.01, block=64)
        for rows in (slice(0, 37), slice(100, 190), slice(250, 300), slice(299, None)):
            part = fn(X, V, oracle.GAUSSIAN, 0.3, 1.1, 0.01, block=16, rows=rows)
            np.testing.assert_allclose(part, full[rows], rtol=1e-13, atol=1e-13 * np.abs(full).max())
