"""Pins of the oracle's Nyström preconditioner (CPU)."""
import numpy as np
import pytest
import scipy.spatial.distance

import oracle
from paper_2503_02259_amd import workloads as W


def _pts(n, d, seed):
    return W.rng(40 + seed, 0).random((n, d))


def test_fps_is_the_greedy_farthest_point_choice():
    # brute force with SciPy's distance matrix: every landmark maximises the
    # distance to the nearest landmark chosen before it
    X = _pts(300, 3, 1)
    idx = oracle.fps_landmarks(X, 40)
    D = scipy.spatial.distance.cdist(X, X)
    assert idx[0] == 0 and len(set(idx.tolist())) == 40
    for j in range(1, 40):
        near = D[:, idx[:j]].min(axis=1)
        assert near[idx[j]] == pytest.approx(near.max(), rel=1e-12)
    # a grid has exact distance ties: the lowest index wins
    g = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [1.0, 1.0]])
    assert oracle.fps_landmarks(g, 4).tolist() == [0, 3, 1, 2]
    assert len(oracle.fps_landmarks(g, 10)) == 4


@pytest.mark.parametrize("kern", [oracle.GAUSSIAN, oracle.MATERN32])
def test_woodbury_matches_dense_inverse(kern):
    X = _pts(150, 2, 2)
    l, f, s = 0.25, 1.3, 0.02
    Wm, C, idx = oracle.nystrom_parts(X, kern, l, f, s, 20)
    M = oracle.nystrom_dense(Wm, idx, f, s)
    np.testing.assert_allclose(M, M.T, atol=1e-12)
    assert np.linalg.eigvalsh(M).min() >= s * (1 - 1e-9)             # M ⪰ sI
    R = W.rng(42, 4).standard_normal((150, 3))
    np.testing.assert_allclose(oracle.nystrom_apply_inv(Wm, C, s, R), np.linalg.solve(M, R),
                               rtol=1e-8, atol=1e-10)
    # M agrees with K̂ on the landmark rows (Nyström interpolates there)
    K = oracle.khat_dense(X, kern, l, f, s)
    np.testing.assert_allclose(M[idx][:, idx], K[idx][:, idx], atol=1e-9)


def test_pcg_with_nystrom():
    X = _pts(400, 3, 3)
    l, f, s = 0.2, 1.0, 0.01
    K = oracle.khat_dense(X, oracle.GAUSSIAN, l, f, s)
    mv = lambda P: K @ P
    B = W.rng(43, 5).standard_normal((400, 2))
    _, itj, _, cj = oracle.pcg(mv, B, 1e-10, 3000, mdiag=np.diag(K))
    Wm, C, _ = oracle.nystrom_parts(X, oracle.GAUSSIAN, l, f, s, 60)
    xn, itn, _, cn = oracle.pcg(mv, B, 1e-10, 3000,
                                apply_minv=lambda R: oracle.nystrom_apply_inv(Wm, C, s, R))
    assert cj.all() and cn.all()
    np.testing.assert_allclose(xn, np.linalg.solve(K, B), rtol=1e-7, atol=1e-9)
    assert itn.max() < 0.5 * itj.max()
    # every point a landmark: M = K̂ and PCG ends after one or two steps
    W2, C2, _ = oracle.nystrom_parts(X[:120], oracle.GAUSSIAN, l, f, s, 120)
    K2 = K[:120, :120]
    _, it1, _, c1 = oracle.pcg(lambda P: K2 @ P, B[:120], 1e-8, 50,
                               apply_minv=lambda R: oracle.nystrom_apply_inv(W2, C2, s, R))
    assert c1.all() and it1.max() <= 2
