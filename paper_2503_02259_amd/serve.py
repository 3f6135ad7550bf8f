"""Continuous-batching serving of GP solves over the C ABI (higp_server_*).

``Server`` wraps one native server; ``replay`` drives it open-loop with a
stream of requests arriving at given times and reports per-request latency
(completion − scheduled arrival), p50/p99 and throughput.  The host loop only
submits arrivals and calls ``step``: admission by HBM footprint, batching of
all active requests' MatVecs into one launch, the CG/Lanczos updates and the
retirement all happen in the native library.
"""
import ctypes
import math
import time

import numpy as np
import torch

from . import _lib
from .api import _dev, problem


class Server:
    def __init__(self, hbm_budget=64 << 30, max_active=64, stream=None, device="cuda:0"):
        self.device = torch.device(device)
        st = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._stream = st
        o = _lib.ServerOpts(hbm_budget=int(hbm_budget), max_active=int(max_active), reserved=0,
                            stream=ctypes.c_void_p(st.cuda_stream))
        h = ctypes.c_void_p()
        _lib.check(_lib.lib().higp_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, X, y, Z=None, l=0.1, f=1.0, s=1e-2, kernel=0, tol=1e-6, max_iter=1000,
               nsteps=40, precond_rank=0, symmetric=True):
        """Queue a solve; returns its id.  X (n×d), y (n), Z (n×nprobe) are
        float32 device tensors kept alive until the request is done.
        precond_rank > 0 solves with the Nyström preconditioner of that rank
        instead of Jacobi.  symmetric=False keeps a large request's
        single-column MatVecs in the full-block form."""
        p = problem(X, kernel, l, f, s, "fp32", symmetric)
        x_out = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
        nprobe = 0 if Z is None else Z.shape[1]
        r = _lib.Request(p=p, y=_dev(y, "y", torch.float32, (X.shape[0],)),
                         Z=_dev(Z, "Z", torch.float32) if Z is not None else None,
                         nprobe=nprobe, nsteps=int(nsteps) if nprobe else 0, tol=float(tol),
                         max_iter=int(max_iter), precond_rank=int(precond_rank),
                         x_out=ctypes.c_void_p(x_out.data_ptr()))
        rid = ctypes.c_int64()
        _lib.check(_lib.lib().higp_server_submit(self._h, ctypes.byref(r), ctypes.byref(rid)))
        self._keep[rid.value] = (X, y, Z, x_out)
        return rid.value

    def step(self):
        na, nq = ctypes.c_int32(), ctypes.c_int32()
        _lib.check(_lib.lib().higp_server_step(self._h, ctypes.byref(na), ctypes.byref(nq)))
        return na.value, nq.value

    def status(self, rid):
        st = _lib.RequestStatus()
        _lib.check(_lib.lib().higp_server_status(self._h, rid, ctypes.byref(st)))
        return st

    def result(self, rid):
        """(x, status) of a finished request (x is the float32 device tensor)."""
        return self._keep[rid][3], self.status(rid)

    def release(self, rid):
        self._keep.pop(rid, None)

    def close(self):
        if self._h:
            _lib.lib().higp_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def footprint(n, d, nprobe, nsteps, precond_rank=0):
    return int(_lib.lib().higp_request_footprint(n, d, nprobe, nsteps, precond_rank))


def replay(requests, server, upload, tol=1e-6, max_iter=1000, nsteps=40, time_scale=1.0,
           on_done=None, precond_rank=0):
    """Open-loop replay: request i is submitted once the wall clock passes its
    arrival time (× time_scale).  ``precond_rank`` is a rank or a function of
    the request giving one (0 = Jacobi).  ``upload(req)`` returns the device tensors
    (X, y, Z) of a request (done at arrival, outside the server).  Returns a
    dict of latencies (s), completion times and summary statistics."""
    n_req = len(requests)
    t0 = time.perf_counter()
    ids = {}
    done_at = {}
    nxt = 0
    while len(done_at) < n_req:
        now = time.perf_counter() - t0
        while nxt < n_req and requests[nxt].arrival * time_scale <= now:
            r = requests[nxt]
            X, y, Z = upload(r)
            rank = precond_rank(r) if callable(precond_rank) else precond_rank
            ids[server.submit(X, y, Z, l=r.l, tol=tol, max_iter=max_iter, nsteps=nsteps,
                              precond_rank=rank)] = nxt
            nxt += 1
        na, nq = server.step() if ids else (0, 0)
        now = time.perf_counter() - t0
        for rid, idx in list(ids.items()):
            if idx in done_at:
                continue
            st = server.status(rid)
            if st.state >= _lib.HIGP_REQ_DONE:
                done_at[idx] = now
                if on_done is not None:
                    on_done(idx, rid, st)
                server.release(rid)
        if na == 0 and nq == 0 and nxt < n_req:
            wait = requests[nxt].arrival * time_scale - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.05))
    lat = np.array([done_at[i] - requests[i].arrival * time_scale for i in range(n_req)])
    first = min(r.arrival for r in requests) * time_scale
    span = max(done_at.values()) - first
    return dict(latency=lat, p50=float(np.percentile(lat, 50, method="nearest")),
                p99=float(np.percentile(lat, 99, method="nearest")),
                throughput=n_req / span if span > 0 else math.inf, span=span)
