"""C-ABI checks that need no GPU: the library loads and exports every symbol
declared in include/higp.h, invalid arguments are rejected before any work is
enqueued, and the host FP64 tridiagonal eigen-solver is right."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.linalg

from paper_2503_02259_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "higp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(higp_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    declared = _declared_symbols()
    assert len(declared) >= 8
    for name in declared:
        assert hasattr(L, name), name
    assert set(declared) == set(_lib.EXPORTS)
    assert L.higp_version() >= 100


def _prob(**kw):
    p = _lib.Problem(kernel=0, prec=1, n=10, d=3, flags=0, X=ctypes.c_void_p(0x1000),
                     l=0.5, f=1.0, s=0.01)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


@pytest.mark.parametrize("field,value", [("n", 0), ("n", -5), ("d", 0), ("d", 33), ("l", 0.0),
                                         ("l", -1.0), ("s", -1e-3), ("kernel", 7), ("prec", 5),
                                         ("flags", 2), ("flags", -1), ("X", None),
                                         ("l", float("nan")),
                                         ("f", float("inf"))])
def test_kmatvec_rejects_bad_problem(field, value):
    L = _lib.lib()
    p = _prob(**{field: value})
    rc = L.higp_kmatvec(ctypes.byref(p), 4, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x9000), None)
    assert rc == _lib.HIGP_ERR_INVALID_ARG
    assert L.higp_last_error().decode()


@pytest.mark.parametrize("k", [0, 65, -1])
def test_kmatvec_rejects_bad_k(k):
    L = _lib.lib()
    p = _prob()
    rc = L.higp_kmatvec(ctypes.byref(p), k, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x9000), None)
    assert rc == _lib.HIGP_ERR_INVALID_ARG


def test_rejects_null_and_overlapping_buffers():
    L = _lib.lib()
    p = _prob()
    assert L.higp_kmatvec(ctypes.byref(p), 4, None, ctypes.c_void_p(0x9000), None) == _lib.HIGP_ERR_INVALID_ARG
    # Y starts inside V (n·k·4 = 160 bytes)
    assert L.higp_kmatvec(ctypes.byref(p), 4, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x2000 + 64),
                          None) == _lib.HIGP_ERR_INVALID_ARG
    assert L.higp_kmatvec_grad(ctypes.byref(p), 4, ctypes.c_void_p(0x2000), None, None, None, None,
                               None) == _lib.HIGP_ERR_INVALID_ARG


def test_pcg_and_slq_reject_bad_options():
    L = _lib.lib()
    p = _prob()
    info = _lib.PcgInfo()
    for kw in (dict(tol=0.0), dict(max_iter=0), dict(precond=3), dict(precond=-1),
               dict(refine_every=-1), dict(use_x0=3), dict(refine_prec=2), dict(check_every=-1),
               dict(precond=2, rank=-1), dict(precond=2, rank=4096)):
        o = _lib.PcgOpts(tol=1e-6, max_iter=10, precond=1, refine_every=0, use_x0=0,
                         check_every=0, refine_prec=0, x_fp64=None)
        for k, v in kw.items():
            setattr(o, k, v)
        rc = L.higp_pcg(ctypes.byref(p), 2, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x9000),
                        ctypes.byref(o), ctypes.byref(info), None)
        assert rc == _lib.HIGP_ERR_INVALID_ARG, kw
    # the Nyström preconditioner needs s > 0
    o = _lib.PcgOpts(tol=1e-6, max_iter=10, precond=2, refine_every=0, use_x0=0, check_every=0,
                     refine_prec=0, x_fp64=None, rank=16)
    p0 = _prob(s=0.0)
    assert L.higp_pcg(ctypes.byref(p0), 2, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x9000),
                      ctypes.byref(o), ctypes.byref(info), None) == _lib.HIGP_ERR_INVALID_ARG
    idx = (ctypes.c_int32 * 4)()
    for rank in (0, -2, 2049):
        assert L.higp_fps_landmarks(ctypes.byref(p), rank, idx, None) == _lib.HIGP_ERR_INVALID_ARG
    assert L.higp_fps_landmarks(ctypes.byref(p), 4, None, None) == _lib.HIGP_ERR_INVALID_ARG
    ld = ctypes.c_double()
    for N, m, reo in ((0, 10, 1), (65, 10, 1), (4, 0, 1), (4, 2000, 1), (4, 10, 2)):
        rc = L.higp_slq_logdet(ctypes.byref(p), N, m, ctypes.c_void_p(0x2000), 0, reo, 1,
                               ctypes.byref(ld), None, None)
        assert rc == _lib.HIGP_ERR_INVALID_ARG
    rc = L.higp_slq_logdet(ctypes.byref(p), 4, 10, None, 0, 1, 1, ctypes.byref(ld), None, None)
    assert rc == _lib.HIGP_ERR_UNSUPPORTED


def test_error_strings():
    L = _lib.lib()
    for code in (0, -1, -2, -3, -4, -99):
        assert L.higp_error_string(code)


@pytest.mark.parametrize("m,seed", [(1, 0), (2, 1), (7, 2), (30, 3), (50, 4), (200, 5)])
def test_tridiag_eig_matches_lapack(m, seed):
    from paper_2503_02259_amd.api import tridiag_eig
    g = np.random.default_rng(seed)
    a = g.standard_normal(m) * 3 + 1
    b = g.random(m - 1) + 0.01
    th, tau = tridiag_eig(a, b)
    if m == 1:
        assert th[0] == a[0] and tau[0] == 1.0
        return
    lam, S = scipy.linalg.eigh_tridiagonal(a, b)
    i = np.argsort(th)
    np.testing.assert_allclose(th[i], lam, rtol=1e-12, atol=1e-12 * np.abs(lam).max())
    np.testing.assert_allclose(np.abs(tau[i]), np.abs(S[0]), atol=1e-10)
    # Σ τ² log θ (the quadrature) for a positive definite shift
    a2 = a + 2 * np.abs(lam).max()
    th2, tau2 = tridiag_eig(a2, b)
    l2, S2 = scipy.linalg.eigh_tridiagonal(a2, b)
    assert abs(np.sum(tau2 ** 2 * np.log(th2)) - np.sum(S2[0] ** 2 * np.log(l2))) < 1e-12 * m


def test_tridiag_eig_clustered_and_split():
    from paper_2503_02259_amd.api import tridiag_eig
    a = np.array([1.0, 1.0, 1.0, 5.0, 5.0, 1e-8])
    b = np.array([1e-20, 0.0, 1e-9, 1e-30, 0.5])
    th, tau = tridiag_eig(a, b)
    lam, S = scipy.linalg.eigh_tridiagonal(a, b)
    np.testing.assert_allclose(np.sort(th), lam, rtol=1e-12, atol=1e-15)
    assert abs(np.sum(tau ** 2) - 1.0) < 1e-14


def test_pcg_overlap_checks_use_each_buffer_size():
    # x_fp64 (double) right after a float B of n·k·4 bytes does not overlap;
    # one starting inside B does.
    L = _lib.lib()
    p = _prob()            # n = 10, float
    info = _lib.PcgInfo()
    o = _lib.PcgOpts(tol=1e-6, max_iter=10, precond=1, refine_every=0, use_x0=0,
                     check_every=0, refine_prec=0, x_fp64=ctypes.c_void_p(0x2000 + 10 * 2 * 4))
    # B at 0x2000 (80 bytes for k=2), Xsol far away, x_fp64 right after B: the
    # call then proceeds past validation, so only the overlapping case is run.
    o.x_fp64 = 0x2000 + 40
    rc = L.higp_pcg(ctypes.byref(p), 2, ctypes.c_void_p(0x2000), ctypes.c_void_p(0x90000),
                    ctypes.byref(o), ctypes.byref(info), None)
    assert rc == _lib.HIGP_ERR_INVALID_ARG
    assert b"x_fp64" in L.higp_last_error()


def test_coldot_and_nlml_reject_bad_arguments():
    L = _lib.lib()
    out = (ctypes.c_double * 4)()
    assert L.higp_coldot(0, 2, 0, ctypes.c_void_p(16), 0, ctypes.c_void_p(32), out, None) == _lib.HIGP_ERR_INVALID_ARG
    assert L.higp_coldot(10, 65, 0, ctypes.c_void_p(16), 0, ctypes.c_void_p(32), out, None) == _lib.HIGP_ERR_INVALID_ARG
    assert L.higp_coldot(10, 2, 7, ctypes.c_void_p(16), 0, ctypes.c_void_p(32), out, None) == _lib.HIGP_ERR_INVALID_ARG
    assert L.higp_coldot(10, 2, 0, None, 0, ctypes.c_void_p(32), out, None) == _lib.HIGP_ERR_INVALID_ARG
    p = _prob()
    loss = ctypes.c_double()
    g = (ctypes.c_double * 3)()
    good = dict(tol=1e-6, max_iter=10, precond=1, refine_every=0, nsteps=10, reorth=1,
                logdet_mode=0, trace_mode=0, reserved=0)
    for bad in (dict(tol=0.0), dict(max_iter=0), dict(precond=3), dict(refine_every=-1),
                dict(nsteps=0), dict(nsteps=5000), dict(reorth=2), dict(reserved=1),
                dict(logdet_mode=2), dict(logdet_mode=-1), dict(trace_mode=2),
                dict(logdet_mode=1, refine_every=10), dict(logdet_mode=1, trace_mode=1)):
        o = _lib.NlmlOpts(**{**good, **bad})
        rc = L.higp_nlml(ctypes.byref(p), ctypes.c_void_p(16), 4, ctypes.c_void_p(64),
                         ctypes.byref(o), ctypes.byref(loss), g, None, None, None)
        assert rc == _lib.HIGP_ERR_INVALID_ARG, bad
    o = _lib.NlmlOpts(**good)
    for N in (0, 64):
        rc = L.higp_nlml(ctypes.byref(p), ctypes.c_void_p(16), N, ctypes.c_void_p(64),
                         ctypes.byref(o), ctypes.byref(loss), g, None, None, None)
        assert rc == _lib.HIGP_ERR_INVALID_ARG
    # Hutch++ needs a sketch and a remainder (N ≥ 2) and 1 + 3⌊N/2⌋ ≤ 64
    o = _lib.NlmlOpts(**dict(good, trace_mode=1))
    for N in (1, 43):
        rc = L.higp_nlml(ctypes.byref(p), ctypes.c_void_p(16), N, ctypes.c_void_p(64),
                         ctypes.byref(o), ctypes.byref(loss), g, None, None, None)
        assert rc == _lib.HIGP_ERR_INVALID_ARG, N


def test_request_footprint_host_logic():
    L = _lib.lib()
    f = lambda n, d, N, m, r=0: int(L.higp_request_footprint(n, d, N, m, r))
    assert f(0, 3, 16, 40) == 0 and f(100, 33, 16, 40) == 0 and f(100, 3, 32, 40) == 0
    a, b = f(10_000, 3, 16, 40), f(20_000, 3, 16, 40)
    assert 0 < a < b
    # the Lanczos basis dominates: (m + 1)·n·N·8 bytes
    assert b >= 41 * 20_000 * 16 * 8
    assert f(10_000, 3, 16, 40) < f(10_000, 3, 16, 80)
    assert f(10_000, 3, 0, 40) < a
    # the Nyström factor adds at least n·rank floats and n doubles for z
    assert f(10_000, 3, 16, 40, 128) >= a + 10_000 * 128 * 4 + 10_000 * 8
    assert f(10_000, 3, 16, 40, 4096) == 0 and f(10_000, 3, 16, 40, -1) == 0


def test_kmatvec_cross_validation():
    L = _lib.lib()
    a, b, c = ctypes.c_void_p(0x2000), ctypes.c_void_p(0x100000), ctypes.c_void_p(0x900000)
    p = _prob()
    for m, k in ((0, 4), (-3, 4), (5, 0), (5, 65)):
        assert L.higp_kmatvec_cross(ctypes.byref(p), m, a, k, b, c, None) == _lib.HIGP_ERR_INVALID_ARG
    assert L.higp_kmatvec_cross(ctypes.byref(p), 5, None, 4, b, c, None) == _lib.HIGP_ERR_INVALID_ARG
    # Y overlapping V
    assert L.higp_kmatvec_cross(ctypes.byref(p), 5, a, 4, b, ctypes.c_void_p(0x100010),
                                None) == _lib.HIGP_ERR_INVALID_ARG
    for prec in (_lib.BF16, _lib.BF16X3):
        pb = _prob(prec=prec)
        assert L.higp_kmatvec_cross(ctypes.byref(pb), 5, a, 4, b, c, None) == _lib.HIGP_ERR_UNSUPPORTED


def test_gpr_predict_validation():
    L = _lib.lib()
    y, xq, mean, var = (ctypes.c_void_p(v) for v in (0x2000, 0x100000, 0x900000, 0xA00000))
    good = dict(tol=1e-6, max_iter=50, precond=1, want_var=0, rank=0)
    p = _prob()
    for bad in (dict(tol=0.0), dict(max_iter=0), dict(precond=3), dict(want_var=2),
                dict(rank=100), dict(precond=2, rank=-1), dict(precond=2, rank=2049)):
        o = _lib.PredictOpts(**dict(good, **bad))
        rc = L.higp_gpr_predict(ctypes.byref(p), y, 5, xq, ctypes.byref(o), mean, None, None, None)
        assert rc == _lib.HIGP_ERR_INVALID_ARG, bad
    o = _lib.PredictOpts(**good)
    # var given without want_var, and want_var without var
    assert L.higp_gpr_predict(ctypes.byref(p), y, 5, xq, ctypes.byref(o), mean, var, None,
                              None) == _lib.HIGP_ERR_INVALID_ARG
    o1 = _lib.PredictOpts(**dict(good, want_var=1))
    assert L.higp_gpr_predict(ctypes.byref(p), y, 5, xq, ctypes.byref(o1), mean, None, None,
                              None) == _lib.HIGP_ERR_INVALID_ARG
    assert L.higp_gpr_predict(ctypes.byref(p), y, 0, xq, ctypes.byref(o), mean, None, None,
                              None) == _lib.HIGP_ERR_INVALID_ARG
    # mean overlapping y
    assert L.higp_gpr_predict(ctypes.byref(p), y, 5, xq, ctypes.byref(o), ctypes.c_void_p(0x2004),
                              None, None, None) == _lib.HIGP_ERR_INVALID_ARG
    pb = _prob(prec=_lib.BF16)
    assert L.higp_gpr_predict(ctypes.byref(pb), y, 5, xq, ctypes.byref(o), mean, None, None,
                              None) == _lib.HIGP_ERR_UNSUPPORTED


def test_debug_fail_allocs_rejects_negative_count():
    L = _lib.lib()
    assert L.higp_debug_fail_allocs(-1) == _lib.HIGP_ERR_INVALID_ARG
    assert L.higp_debug_fail_allocs(0) == _lib.HIGP_OK
