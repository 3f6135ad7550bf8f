"""Continuous-batching server (higp_server_*): results against the oracle,
bitwise equality of a request alone and in a mix, and admission by HBM
footprint."""
import numpy as np
import pytest
import torch

import oracle
from paper_2503_02259_amd import _lib, workloads as W
from paper_2503_02259_amd.serve import Server, footprint
from helpers import as_prec, dev, to_dev

pytestmark = pytest.mark.gpu


def _req(n, d, seed, nprobe=16):
    X = as_prec(W.rng(2000 + seed, 0).random((n, d)), torch.float32)
    y = as_prec(np.sin(2 * np.pi * X[:, 0]) + 0.1 * W.rng(2000 + seed, 1).standard_normal(n),
                torch.float32)
    Z = W.rademacher(n, nprobe, 2000 + seed) if nprobe else None
    return X, y, Z


def _upload(X, y, Z):
    return (to_dev(X, torch.float32), to_dev(y, torch.float32),
            to_dev(Z, torch.float32) if Z is not None else None)


def _run(server, reqs, l=0.2, precond_rank=0):
    ids = [server.submit(*_upload(*r), l=l, tol=1e-6, max_iter=1000, nsteps=30,
                         precond_rank=precond_rank) for r in reqs]
    for _ in range(100000):
        na, nq = server.step()
        if na == 0 and nq == 0:
            break
    out = []
    for rid in ids:
        x, st = server.result(rid)
        assert st.state == _lib.HIGP_REQ_DONE
        out.append((x.cpu().numpy().copy(), st.logdet, st.iters, st.relres, st.converged))
    return out


def test_single_request_matches_oracle():
    X, y, Z = _req(3000, 3, 1)
    srv = Server(hbm_budget=8 << 30, max_active=8)
    (x, logdet, iters, relres, conv), = _run(srv, [(X, y, Z)])
    srv.close()
    assert conv and relres <= 1e-6
    K = oracle.khat_dense(X, 0, 0.2, 1.0, 1e-2)
    tr = np.linalg.norm(y - K @ x.astype(np.float64)) / np.linalg.norm(y)
    Kabs = np.abs(K) @ np.abs(x.astype(np.float64))
    floor = 6e-8 * np.linalg.norm(Kabs) / np.linalg.norm(y)
    assert tr <= 1e-6 + 50 * floor, (tr, floor)
    ldo, _ = oracle.slq_logdet(lambda P: K @ P, Z, 30, mdiag=np.full(3000, 1.01))
    assert abs(logdet - ldo) <= 1e-5 * abs(ldo), (logdet, ldo)


def test_single_request_nystrom():
    # The same request solved with the Nyström preconditioner (128 landmarks):
    # fewer CG iterations, the same accuracy, and the SLQ log-determinant of
    # the Jacobi run (the Lanczos columns do not depend on the CG column).
    X, y, Z = _req(3000, 3, 1)
    srv = Server(hbm_budget=8 << 30, max_active=8)
    (xj, ldj, itj, _, _), = _run(srv, [(X, y, Z)])
    (x, logdet, iters, relres, conv), = _run(srv, [(X, y, Z)], precond_rank=128)
    srv.close()
    print("serving CG iterations: Jacobi %d, Nyström %d" % (itj, iters))
    assert conv and relres <= 1e-6 and iters < itj / 2
    K = oracle.khat_dense(X, 0, 0.2, 1.0, 1e-2)
    tr = np.linalg.norm(y - K @ x.astype(np.float64)) / np.linalg.norm(y)
    floor = 6e-8 * np.linalg.norm(np.abs(K) @ np.abs(x.astype(np.float64))) / np.linalg.norm(y)
    assert tr <= 1e-6 + 50 * floor, (tr, floor)
    assert logdet == pytest.approx(ldj, rel=1e-12)


@pytest.mark.parametrize("rank", [0, 96])
def test_alone_equals_in_mix_bitwise(rank):
    target = _req(2500, 3, 2)
    others = [_req(n, d, 10 + i) for i, (n, d) in enumerate([(1200, 2), (4000, 8), (900, 3),
                                                            (3300, 2), (1800, 8)])]
    s1 = Server(hbm_budget=8 << 30, max_active=8)
    alone = _run(s1, [target], precond_rank=rank)[0]
    s1.close()
    s2 = Server(hbm_budget=8 << 30, max_active=8)
    mixed = _run(s2, others[:3] + [target] + others[3:], precond_rank=rank)
    s2.close()
    mix = mixed[3]
    assert np.array_equal(alone[0], mix[0])
    assert alone[1] == mix[1] and alone[2] == mix[2] and alone[3] == mix[3]


def test_admission_respects_budget_and_all_finish():
    reqs = [_req(n, 3, 30 + i, nprobe=8) for i, n in enumerate([2000, 2600, 1500, 3000, 2200])]
    fps = [footprint(r[0].shape[0], 3, 8, 30) for r in reqs]
    budget = int(max(fps) * 2.2)          # at most two requests fit at once
    srv = Server(hbm_budget=budget, max_active=16)
    ids = [srv.submit(*_upload(*r), l=0.2, tol=1e-6, max_iter=1000, nsteps=30) for r in reqs]
    max_active = 0
    for _ in range(100000):
        na, nq = srv.step()
        max_active = max(max_active, na)
        assert na <= 2
        active_fp = sum(fps[i] for i, rid in enumerate(ids) if srv.status(rid).state == _lib.HIGP_REQ_ACTIVE)
        assert active_fp <= budget
        if na == 0 and nq == 0:
            break
    assert max_active == 2
    for rid in ids:
        st = srv.status(rid)
        assert st.state == _lib.HIGP_REQ_DONE and st.converged
    srv.close()


def test_request_larger_than_budget_is_rejected():
    X, y, Z = _req(5000, 3, 40)
    srv = Server(hbm_budget=1 << 20, max_active=4)
    with pytest.raises(_lib.HigpError) as e:
        srv.submit(*_upload(X, y, Z), l=0.2)
    assert e.value.code == _lib.HIGP_ERR_OOM
    srv.close()


@pytest.mark.parametrize("d", [3, 8])
def test_large_request_symmetric_matvec(d):
    # n = 40,000 (d = 3, or 8 with two float4s per staged point): once its
    # Lanczos columns are done, the request's single CG column takes the
    # symmetric-tiled MatVec.  Its result is the same alone and in a mix
    # (with a d = 3 and a d = 8 request beside it), agrees with the
    # full-block form to rounding, and its true residual (FP64 MatVec) is
    # within twice the tolerance (the recursive residual drifts from the true
    # one by the FP32 MatVec error).
    import paper_2503_02259_amd as hg
    n = 40_000
    l = 0.1 if d == 3 else 0.4  # kernel values well away from the identity in 8 dimensions
    big = _req(n, d, 50, nprobe=4)
    small = [_req(m, dm, 60 + i, nprobe=4) for i, (m, dm) in enumerate([(1500, 3), (2500, 8)])]

    def run(reqs, symmetric=True):
        srv = Server(hbm_budget=16 << 30, max_active=8)
        ids = [srv.submit(*_upload(*r), l=l, s=0.1, tol=1e-5, max_iter=1000, nsteps=10,
                          symmetric=symmetric) for r in reqs]
        for _ in range(100000):
            na, nq = srv.step()
            if na == 0 and nq == 0:
                break
        out = []
        for rid in ids:
            x, st = srv.result(rid)
            assert st.state == _lib.HIGP_REQ_DONE
            out.append((x.cpu().numpy().copy(), st.logdet, st.iters, st.relres))
        srv.close()
        return out

    alone = run([big])[0]
    mixed = run([small[0], big, small[1]])[1]
    assert np.array_equal(alone[0], mixed[0]) and alone[1:] == mixed[1:]
    full = run([big], symmetric=False)[0]
    print("large request: %d iterations (full-block form %d), relres %.2e"
          % (alone[2], full[2], alone[3]))
    assert alone[3] <= 1e-5 and abs(alone[2] - full[2]) <= max(3, full[2] // 20)
    X, y, _ = big
    x = alone[0].astype(np.float64)
    Kx = hg.kmatvec(to_dev(X, torch.float64), to_dev(x, torch.float64), 0, l, 1.0,
                    0.1).cpu().numpy()
    tr = np.linalg.norm(y - Kx) / np.linalg.norm(y)
    Kabs = hg.kmatvec(to_dev(X, torch.float64), to_dev(np.abs(x), torch.float64), 0, l, 1.0,
                      0.1).cpu().numpy()
    floor = 6e-8 * np.linalg.norm(Kabs) / np.linalg.norm(y)
    print("true relative residual %.2e, FP32 floor %.2e" % (tr, floor))
    assert tr <= 2e-5, (tr, floor)
