"""Benchmark of the on-the-fly kernel MatVec hot path on one MI355X.

A step is one K̂·V MatVec (n = 100,000 points uniform in [0,1]^3, Gaussian
kernel, f = 1, l = 0.1, s = 1e-2, V = [y | 32 Rademacher probes], k = 33,
FP32) with inputs resident in HBM.  The headline value is kernel evaluations
× vectors per second, n²·k / t.  After the timed steps, the same workload is
solved by block PCG (Jacobi) to 1e-6 and its log-determinant estimated by
SLQ (32 probes × 50 steps); their wall times are reported beside the
headline.  The FP64 CPU oracle is timed on a bounded row sample of the same
MatVec on the host cores.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_MFMA_FP32 = 157.3e12  # MI355X dense FP32 matrix peak, FLOP/s
PROFILE = os.path.join(ROOT, "profiles", "kmv_f32_gauss_n100000_k33.md")
KERNEL_SRC = os.path.join(ROOT, "paper_2503_02259_amd", "csrc", "kmatvec_f32.hip")


def measured_traffic():
    """HBM bytes per launch of the FP32 MatVec kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None if the kernel source has
    changed since the counters were taken."""
    import hashlib
    try:
        txt = open(PROFILE).read()
        sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in txt.splitlines()
                if line.startswith(("traffic_bytes_per_launch: ", "source_sha256_16: ")))
    if vals.get("source_sha256_16", "").strip() != sha:
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_baseline(prob, rows=None, workers=None):
    """Time the oracle MatVec on the first `rows` rows (all n columns)."""
    import oracle
    from threadpoolctl import threadpool_limits
    X, V = prob.X.astype(np.float32).astype(np.float64), prob.extra["V"].astype(np.float32).astype(np.float64)
    rows = min(rows or X.shape[0], X.shape[0])
    workers = workers or min(16, os.cpu_count() or 1)
    Xs = X  # all n points as columns; only `rows` rows of K̂ are formed
    n = X.shape[0]
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        from concurrent.futures import ThreadPoolExecutor
        blocks = [slice(i, min(i + 128, rows)) for i in range(0, rows, 128)]

        def one(b):
            K = oracle.kernel_value(oracle.sqdist(Xs[b], Xs), prob.kernel, prob.l)
            return prob.f ** 2 * (K @ V) + prob.s * V[b]

        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one, blocks))
        dt = time.perf_counter() - t0
    k = V.shape[1]
    return dict(value=rows * n * k / dt, unit="kernel-evals*vectors/s", cores=workers, kind="oracle",
                sample="FP64 oracle MatVec on rows 0..%d of the n=%d, k=%d workload "
                       "(%d×%d kernel values), %.1f s" % (rows - 1, n, k, rows, n, dt))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kernel", default="gaussian", choices=["gaussian", "matern32"])
    ap.add_argument("--no-solve", action="store_true", help="skip the PCG/SLQ wall-time legs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-rows", type=int, default=0, help="rows of the CPU oracle sample (0 = all)")
    ap.add_argument("--calib-copy", type=int, default=0, metavar="MIB",
                    help="run one plain device copy of this many MiB first (a known-size "
                         "reference for hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only; the multi-GPU path is not built "
              "(see the sharding design).  Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2503_02259_amd as hg
    from paper_2503_02259_amd import workloads as W

    dev = torch.device("cuda:0")
    kern = hg.GAUSSIAN if args.kernel == "gaussian" else hg.MATERN32
    prob = W.workload_fp32_matvec(kernel=kern)
    n, k = prob.X.shape[0], prob.extra["V"].shape[1]
    X = torch.from_numpy(prob.X).to(dev, torch.float32)
    V = torch.from_numpy(prob.extra["V"]).to(dev, torch.float32)
    Y = torch.empty_like(V)
    stream = torch.cuda.current_stream(dev)

    if args.calib_copy > 0:
        src = torch.ones(args.calib_copy << 18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(args.warmup):
        hg.kmatvec(X, V, kern, prob.l, prob.f, prob.s, out=Y)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        hg.kmatvec(X, V, kern, prob.l, prob.f, prob.s, out=Y)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / args.steps
    value = float(n) * n * k / (ms * 1e-3)
    flops = 2.0 * n * n * k
    achieved = flops / (ms * 1e-3)

    out = {
        "metric": "kernel-evals*vectors/s (n=1e5, d=3, k=33)",
        "value": value,
        "unit": "kernel-evals*vectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "on-the-fly MatVec Y=K̂V, n=100000 uniform [0,1]^3, %s kernel, "
                               "f=1 l=0.1 s=1e-2, V=[y|32 Rademacher] k=33, FP32" % args.kernel,
                   "n": n, "d": 3, "k": k, "kernel": args.kernel, "precision": "fp32"},
        "roofline": {"bound": "mfma", "achieved": achieved / 1e12, "peak": PEAK_MFMA_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_MFMA_FP32,
                     "traffic": measured_traffic() if kern == hg.GAUSSIAN else None},
        "wall_s_timed": wall,
    }

    if not args.no_solve:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = hg.pcg(X, V, kern, prob.l, prob.f, prob.s, tol=1e-6, max_iter=5000,
                         precond="jacobi")
        torch.cuda.synchronize()
        t_pcg = time.perf_counter() - t0
        Z = V[:, 1:].contiguous()
        t0 = time.perf_counter()
        ld, per = hg.slq_logdet(X, Z, kern, prob.l, prob.f, prob.s, 50, precond="jacobi")
        t_slq = time.perf_counter() - t0
        out["pcg_time_to_1e-6_s"] = t_pcg
        out["pcg_iters_max"] = int(info["iters"].max())
        out["pcg_converged"] = int(info["converged"].sum())
        out["pcg_relres_max"] = float(info["relres"].max())
        out["slq_time_s"] = t_slq
        out["slq_logdet"] = ld
        out["slq_stderr"] = float(per.std(ddof=1) / np.sqrt(per.size))

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, rows=args.cpu_rows or None)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
