"""Seeded synthetic inputs for the GP MatVec workloads.

This module only draws random numbers and arranges them; it holds none of the
method's arithmetic, and both the HIP path's tests and the CPU oracle take
their inputs from it.  Every generator is a NumPy ``default_rng`` (PCG64)
stream keyed by ``[workload id, stream id]``: stream 0 = points X,
1 = observation noise of y, 2 = probe vectors, 3 = subsample permutation,
4 = the single MatVec vector, 5 = mixture centres and assignments,
6 = serving arrivals and request shapes.

The paper measures on UCI data sets and VLSE test functions (Numerical
Experiments section) that are not available here; these synthetic point
clouds (uniform in the unit cube, or a Gaussian mixture) stand in for them.
"""
import math
from dataclasses import dataclass, field

import numpy as np


def rng(workload, stream):
    return np.random.default_rng([int(workload), int(stream)])


def uniform_points(n, d, workload, stream=0):
    """n points uniform in [0, 1]^d, float64, row-major n×d."""
    return rng(workload, stream).random((n, d))


def sine_targets(X, workload, noise=0.1):
    """y = sin(2π·x₀) + noise·N(0, 1), float64 (the noisy observation set)."""
    e = rng(workload, 1).standard_normal(X.shape[0])
    return np.sin(2.0 * np.pi * X[:, 0]) + noise * e


def rademacher(n, k, workload, stream=2):
    """n×k matrix of independent ±1 entries, float64."""
    return rng(workload, stream).integers(0, 2, size=(n, k)).astype(np.float64) * 2.0 - 1.0


def gaussian_vectors(n, k, workload, stream=4):
    return rng(workload, stream).standard_normal((n, k))


def gaussian_mixture(n, d, ncentres, sigma, workload):
    """n points from an equal-weight mixture of ``ncentres`` isotropic
    Gaussians (std ``sigma``) with centres uniform in [0, 1]^d; no clipping.
    Component of each point: uniform integer assignment."""
    g = rng(workload, 5)
    centres = g.random((ncentres, d))
    comp = g.integers(0, ncentres, size=n)
    X = centres[comp] + sigma * rng(workload, 0).standard_normal((n, d))
    return X


def subsample_index(n, m, workload):
    """The first m entries of a seeded permutation of range(n)."""
    return rng(workload, 3).permutation(n)[:m]


# ---------------------------------------------------------------------------
# The five workloads (ids 1..5).

GAUSSIAN = 0
MATERN32 = 1


@dataclass
class Problem:
    X: np.ndarray
    kernel: int
    l: float
    f: float
    s: float
    extra: dict = field(default_factory=dict)


def workload_fp64_small(n=2000):
    """n=2,000 uniform points in [0,1]^3; Gaussian kernel f=1, l=0.5, s=0.01;
    y = sin(2π x₀) + N(0, 0.1²); one MatVec vector v ~ N(0,1); 10 Rademacher
    probes (for 30 Lanczos steps)."""
    X = uniform_points(n, 3, 1)
    return Problem(X, GAUSSIAN, 0.5, 1.0, 0.01, dict(
        y=sine_targets(X, 1), v=gaussian_vectors(n, 1, 1)[:, 0],
        Z=rademacher(n, 10, 1), cg_tol=1e-8, slq_steps=30))


def workload_fp32_matvec(n=100_000, kernel=GAUSSIAN, nprobe=32):
    """n=100,000 uniform points in [0,1]^3; f=1, l=0.1, s=1e-2;
    V = [y | 32 Rademacher probes] (k=33); PCG (Jacobi) to 1e-6; SLQ with 32
    probes × 50 steps."""
    X = uniform_points(n, 3, 2)
    y = sine_targets(X, 2)
    Z = rademacher(n, nprobe, 2)
    V = np.concatenate([y[:, None], Z], axis=1)
    return Problem(X, kernel, 0.1, 1.0, 1e-2, dict(
        y=y, Z=Z, V=V, cg_tol=1e-6, slq_steps=50))


def workload_bf16_mixture(n=500_000, sub=20_000):
    """n=500,000 points in d=8 from a mixture of 16 Gaussians (σ=0.05, centres
    uniform in [0,1]^8); Gaussian kernel f=1, l=0.3, s=1e-3; k=33
    (y and 32 Rademacher probes); refinement every 10 iterations; a seeded
    20,000-point subsample for the CPU comparison."""
    X = gaussian_mixture(n, 8, 16, 0.05, 3)
    y = sine_targets(X, 3)
    Z = rademacher(n, 32, 3)
    V = np.concatenate([y[:, None], Z], axis=1)
    return Problem(X, GAUSSIAN, 0.3, 1.0, 1e-3, dict(
        y=y, Z=Z, V=V, cg_tol=1e-6, refine_every=10,
        sub=subsample_index(n, sub, 3)))


def workload_grad(n=200_000):
    """n=200,000 uniform points in [0,1]^3; Gaussian kernel (f, l, s) =
    (1.0, 0.2, 0.05); y and 32 Hutchinson (Rademacher) probes."""
    X = uniform_points(n, 3, 4)
    y = sine_targets(X, 4)
    Z = rademacher(n, 32, 4)
    return Problem(X, GAUSSIAN, 0.2, 1.0, 0.05, dict(y=y, Z=Z, fd_h=1e-4))


def workload_paper_shape(n=30_000, m=3_000, d=20):
    """The shape of the paper's on-the-fly runs (n = 30,000 training points
    in d = 20; "Numerical Experiments"), as synthetic data standing in for
    its 20-D test-function data sets: points uniform in [0,1]^d, target
    sin(2π x₀) + Σ_c x_c/d + N(0, 0.1²), and like the paper, features and
    targets z-scored with the training set's statistics.  Returns
    (X_train, y_train, X_test, y_test)."""
    g = rng(6, 0)
    Xa = g.random((n + m, d))
    ya = np.sin(2.0 * np.pi * Xa[:, 0]) + Xa.mean(axis=1) + 0.1 * rng(6, 1).standard_normal(n + m)
    mu, sd = Xa[:n].mean(axis=0), Xa[:n].std(axis=0)
    Xa = (Xa - mu) / sd
    ym, ys = ya[:n].mean(), ya[:n].std()
    ya = (ya - ym) / ys
    return Xa[:n], ya[:n], Xa[n:], ya[n:]


@dataclass
class Request:
    rid: int
    arrival: float
    n: int
    d: int
    l: float
    X: np.ndarray
    y: np.ndarray
    Z: np.ndarray


STREAM_LEN = 512


def serving_stream(nreq=512, rate=200.0, nmin=1000, nmax=200_000,
                   dims=(2, 3, 8), nprobe=16, workload=5, materialise=True):
    """Independent GP solves arriving as a Poisson stream: exponential
    inter-arrival times at ``rate`` per second; n = ⌊exp U[ln nmin, ln nmax]⌋;
    d uniform over ``dims``; X uniform in [0,1]^d; l ~ U[0.05, 0.5]; f=1,
    s=1e-2 (Gaussian kernel); y as above and ``nprobe`` Rademacher probes.
    The stream is drawn for 512 requests (or ``nreq`` if larger) and the first
    ``nreq`` are returned, so a shorter replay is a prefix of the full one."""
    g = rng(workload, 6)
    m = max(nreq, STREAM_LEN)
    gaps = g.exponential(1.0 / rate, size=m)[:nreq]
    arrivals = np.cumsum(gaps) - gaps[0]
    ns = np.floor(np.exp(g.uniform(math.log(nmin), math.log(nmax), size=m))).astype(np.int64)[:nreq]
    ds = g.choice(np.asarray(dims), size=m)[:nreq]
    ls = g.uniform(0.05, 0.5, size=m)[:nreq]
    out = []
    for i in range(nreq):
        if materialise:
            X = rng(1000 + i, 0).random((int(ns[i]), int(ds[i])))
            y = np.sin(2.0 * np.pi * X[:, 0]) + 0.1 * rng(1000 + i, 1).standard_normal(int(ns[i]))
            Z = rademacher(int(ns[i]), nprobe, 1000 + i)
        else:
            X = y = Z = None
        out.append(Request(i, float(arrivals[i]), int(ns[i]), int(ds[i]), float(ls[i]), X, y, Z))
    return out


def random_problem(n, d, seed, kernel=GAUSSIAN, l=0.3, f=1.3, s=0.05, k=4):
    """A small random problem for parity tests: X uniform in [0,1]^d and
    V ~ N(0,1) of width k."""
    X = rng(10_000 + seed, 0).random((n, d))
    V = rng(10_000 + seed, 4).standard_normal((n, k))
    return Problem(X, kernel, l, f, s, dict(V=V))
