"""Benchmark of the on-the-fly kernel MatVec hot path on one MI355X.

A step is one K̂·V MatVec (n = 100,000 points uniform in [0,1]^3, Gaussian
kernel, f = 1, l = 0.1, s = 1e-2, V = [y | 32 Rademacher probes], k = 33,
FP32) with inputs resident in HBM.  The headline value is kernel evaluations
× vectors per second, n²·k / t.  After the timed steps, the same workload is
solved by block PCG (Jacobi) to 1e-6 and its log-determinant estimated by
SLQ (32 probes × 50 steps); their wall times are reported beside the
headline.  Further legs (extra keys, not the headline): the plain FP64 method
at n = 2,000; the BF16 forms against the FP32 form at n = 500,000, d = 8; the
fused derivative MatVec at n = 200,000; hyper-parameter training with the
paper's end-to-end settings at n = 100,000; the continuous-batching server on
the Poisson request stream (p50/p99 latency, solves/s).  The FP64 CPU oracle is
timed on a bounded row sample of the MatVec on the host cores.

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
# Sources of the FP32 MatVec kernel the counters were taken on.
KERNEL_SRCS = [os.path.join(ROOT, "paper_2503_02259_amd", "csrc", f)
               for f in ("kmv_f32_tile.h", "kmatvec_f32.hip")]


def measured_traffic():
    """HBM bytes per launch of the FP32 MatVec kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None if the kernel source has
    changed since the counters were taken."""
    import hashlib
    try:
        txt = open(PROFILE).read()
        sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SRCS)).hexdigest()[:16]
    except OSError:
        return None
    vals = dict(line.split(": ", 1) for line in txt.splitlines()
                if line.startswith(("traffic_bytes_per_launch: ", "source_sha256_16: ")))
    if vals.get("source_sha256_16", "").strip() != sha:
        return None
    return float(vals["traffic_bytes_per_launch"])


def cpu_model():
    """The host CPU's model name (Linux), or the platform's processor string."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(prob, rows=None, workers=None):
    """Time the oracle MatVec (``oracle.kmatvec``, 128-row blocks on a thread
    pool, one BLAS thread per block) on the first `rows` rows (all n
    columns)."""
    import oracle
    from threadpoolctl import threadpool_limits
    X, V = prob.X.astype(np.float32).astype(np.float64), prob.extra["V"].astype(np.float32).astype(np.float64)
    n = X.shape[0]
    rows = min(rows or n, n)
    workers = workers or min(16, os.cpu_count() or 1)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        oracle.kmatvec(X, V, prob.kernel, prob.l, prob.f, prob.s, block=128, workers=workers,
                       rows=slice(0, rows))
        dt = time.perf_counter() - t0
    k = V.shape[1]
    return dict(value=rows * n * k / dt, unit="kernel-evals*vectors/s", cores=workers, kind="oracle",
                cpu_model=cpu_model(),
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
    ap.add_argument("--legs", default="fp64,bf16,grad,sym,train,estimators,paper,serve",
                    help="comma list of extra legs (fp64, bf16, grad, sym, train, estimators, "
                         "paper, serve) or 'none'")
    ap.add_argument("--serve", type=int, default=64, metavar="N",
                    help="requests of the serving stream to replay (the full stream has 512)")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed headline MatVecs (no PCIe-inclusive or other-kernel "
                         "MatVecs): the launches a profile of the headline kernel should see")
    ap.add_argument("--serve-slots", type=int, default=8,
                    help="max_active of the serving replays (concurrent requests; 8 gave the "
                         "lowest p50 at full throughput in a sweep over 4-64)")
    ap.add_argument("--serve-rank", type=int, default=512,
                    help="Nyström rank of the second serving replay (0: skip it)")
    ap.add_argument("--serve-skip-jacobi", action="store_true",
                    help="skip the Jacobi serving replay (e.g. to profile the Nyström one alone)")
    ap.add_argument("--serve-rates", default="", metavar="R1,R2,...",
                    help="also replay the same requests at these arrival rates (per second; "
                         "the stream's own rate is 200/s), Jacobi and Nyström: latency at "
                         "lower offered load, for context")
    ap.add_argument("--mixture-form", choices=("fp32", "bf16", "bf16x3"), default=None,
                    help="time only this form's MatVec on the n=500,000 d=8 mixture "
                         "(for profiling) and print its own JSON line")
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
    if args.mixture_form:
        mix = W.workload_bf16_mixture()
        Xm = torch.from_numpy(mix.X).to(dev, torch.float32)
        Vm = torch.from_numpy(mix.extra["V"]).to(dev, torch.float32)
        fn = lambda: hg.kmatvec(Xm, Vm, 0, mix.l, mix.f, mix.s, precision=args.mixture_form)
        for _ in range(args.warmup):
            fn()
        ms = _timed(fn, args.steps)
        nm = Xm.shape[0]
        print(json.dumps({"workload": "n=500000 d=8 16-Gaussian mixture, Gaussian l=0.3 s=1e-3, k=33",
                          "form": args.mixture_form, "ms": ms,
                          "kev_vec_per_s": float(nm) * nm * 33 / (ms * 1e-3)}))
        return
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

    if args.headline_only:
        print(json.dumps(out))
        return

    # The same MatVec when X and V start in (pinned) host memory and Y must go
    # back: the PCIe-inclusive rate, reported beside the HBM-resident value.
    Xh = torch.empty(X.shape, dtype=X.dtype, pin_memory=True)
    Vh = torch.empty(V.shape, dtype=V.dtype, pin_memory=True)
    Yh = torch.empty(V.shape, dtype=V.dtype, pin_memory=True)
    Xh.copy_(X)
    Vh.copy_(V)
    Xd, Vd = torch.empty_like(X), torch.empty_like(V)

    def roundtrip():
        Xd.copy_(Xh, non_blocking=True)
        Vd.copy_(Vh, non_blocking=True)
        Yd = hg.kmatvec(Xd, Vd, kern, prob.l, prob.f, prob.s)
        Yh.copy_(Yd, non_blocking=True)

    ms_rt = _timed(roundtrip, 5)
    out["pcie_inclusive"] = {"ms": ms_rt, "kev_vec_per_s": float(n) * n * k / (ms_rt * 1e-3),
                             "bytes_moved": int(X.numel() * 4 + 2 * V.numel() * 4)}
    del Xh, Vh, Yh, Xd, Vd

    # The other kernel of the same configuration (Matérn-3/2 when the headline
    # is Gaussian and the reverse), same points and vectors.
    other = hg.MATERN32 if kern == hg.GAUSSIAN else hg.GAUSSIAN
    ms_o = _timed(lambda: hg.kmatvec(X, V, other, prob.l, prob.f, prob.s, out=Y), 10)
    out["other_kernel"] = {"kernel": "matern32" if other == hg.MATERN32 else "gaussian", "ms": ms_o,
                           "kev_vec_per_s": float(n) * n * k / (ms_o * 1e-3),
                           "mfma_frac": 2.0 * n * n * k / (ms_o * 1e-3) / PEAK_MFMA_FP32}

    if not args.no_solve:
        # Time to 1e-6: the FP32 form stops on its recursive residual (its
        # true residual is limited by the FP32 floor and reported beside it);
        # with an FP64 recompute every 10 iterations the tolerance holds for
        # the true residual, in the FP32 and in the split-BF16 form.
        runs = (("pcg", dict()),
                ("pcg_fp32_refine_fp64", dict(refine_every=10, refine_prec="fp64")),
                ("pcg_bf16x3_refine_fp64", dict(precision="bf16x3", refine_every=10,
                                                refine_prec="fp64")),
                ("pcg_nystrom1024_refine_fp64", dict(precond="nystrom", rank=1024,
                                                     refine_every=10, refine_prec="fp64")))
        for name, kw in runs:
            r = _pcg_run(X, V, kern, prob, 5000, **kw)
            if name == "pcg":
                out["pcg_time_to_1e-6_s"] = r["time_s"]
                out["pcg_iters_max"] = r["iters_max"]
                out["pcg_converged"] = r["converged"]
                out["pcg_relres_max"] = r["relres_max"]
                out["pcg_true_relres_max"] = r["true_relres_max"]
            else:
                out[name] = r
        out["pcg_nystrom1024_refine_fp64"]["speedup_vs_fp32_refine_fp64"] = (
            out["pcg_fp32_refine_fp64"]["time_s"] / out["pcg_nystrom1024_refine_fp64"]["time_s"])
        out["pcg_bf16x3_refine_fp64"]["speedup_vs_fp32_refine_fp64"] = (
            out["pcg_fp32_refine_fp64"]["time_s"] / out["pcg_bf16x3_refine_fp64"]["time_s"])
        out["bf16x3_matvec_ms"] = _timed(
            lambda: hg.kmatvec(X, V, kern, prob.l, prob.f, prob.s, precision="bf16x3"), 10)
        Z = V[:, 1:].contiguous()
        t0 = time.perf_counter()
        ld, per = hg.slq_logdet(X, Z, kern, prob.l, prob.f, prob.s, 50, precond="jacobi")
        t_slq = time.perf_counter() - t0
        out["slq_time_s"] = t_slq
        out["slq_logdet"] = ld
        out["slq_stderr"] = float(per.std(ddof=1) / np.sqrt(per.size))
        _log("solve legs done")

    legs = set() if args.legs == "none" else set(args.legs.split(","))
    if "fp64" in legs:
        out["fp64_small"] = leg_fp64()
    if "bf16" in legs:
        out["bf16_precision_form"] = leg_bf16()
    if "grad" in legs:
        out["grad_matvec"] = leg_grad()
    if "train" in legs:
        out["train_e2e"] = leg_train()
        out["train_e2e_cg_logdet"] = leg_train("cg")
    if "estimators" in legs:
        out["nlml_estimators"] = leg_estimators()
    if "sym" in legs:
        out["symmetric_matvec"] = leg_symmetric()
    if "paper" in legs:
        for kname, kid in (("gaussian", 0), ("matern32", 1)):
            out["paper_shape_e2e_" + kname] = leg_paper_shape(kid)
    if "serve" in legs and args.serve > 0:
        if not args.serve_skip_jacobi:
            out["serving"] = leg_serve(args.serve, slots=args.serve_slots)
        if args.serve_rank > 0:
            out["serving_nystrom"] = leg_serve(args.serve, precond_rank=args.serve_rank,
                                               slots=args.serve_slots)
    if "serve" in legs and args.serve > 0 and args.serve_rates:
        sweep = []
        for rate in (float(x) for x in args.serve_rates.split(",")):
            for rank in (0, args.serve_rank):
                res = leg_serve(args.serve, precond_rank=rank, slots=args.serve_slots,
                                rate=rate)
                sweep.append(dict(rate_per_s=rate, precond="nystrom%d" % rank if rank else "jacobi",
                                  **{k: res[k] for k in ("p50_s", "p99_s", "solves_per_s",
                                                         "span_s", "converged")}))
        out["serving_rate_sweep"] = sweep
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(prob, rows=args.cpu_rows or None)
    print(json.dumps(out))


def _timed(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _pcg_run(X, B, kern, prob, max_iter, **kw):
    """Wall time of one PCG solve to 1e-6 (Jacobi) and its result; the true
    relative residual of the FP64 iterate is evaluated with the library's
    FP64 MatVec."""
    import torch
    import paper_2503_02259_amd as hg
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    kw.setdefault("precond", "jacobi")
    x, x64, info = hg.pcg(X, B, kern, prob.l, prob.f, prob.s, tol=1e-6, max_iter=max_iter,
                          return_fp64=True, **kw)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    B64 = B.double()
    r = B64 - hg.kmatvec(X.double(), x64, kern, prob.l, prob.f, prob.s)
    tr = (torch.linalg.vector_norm(r, dim=0) / torch.linalg.vector_norm(B64, dim=0)).max().item()
    _log("pcg %s/%s: %.2f s, %d iterations" % (kw.get("precision", "fp32"), kw["precond"], t,
                                             int(info["iters"].max())))
    return dict(time_s=t, iters_max=int(info["iters"].max()), converged=int(info["converged"].sum()),
                columns=int(B.shape[1]), relres_max=float(info["relres"].max()), true_relres_max=tr)


def leg_fp64():
    """Plain method, FP64: n = 2,000 uniform in [0,1]^3, Gaussian f=1, l=0.5,
    s=0.01; one MatVec, CG to 1e-8, SLQ 10 probes × 30 steps (wall times)."""
    import torch
    import paper_2503_02259_amd as hg
    from paper_2503_02259_amd import workloads as W
    p = W.workload_fp64_small()
    d = torch.device("cuda:0")
    X = torch.from_numpy(p.X).to(d)
    v = torch.from_numpy(p.extra["v"]).to(d)
    y = torch.from_numpy(p.extra["y"]).to(d)
    Z = torch.from_numpy(p.extra["Z"]).to(d)
    ms = _timed(lambda: hg.kmatvec(X, v, p.kernel, p.l, p.f, p.s), 20)
    t0 = time.perf_counter()
    x, info = hg.pcg(X, y, p.kernel, p.l, p.f, p.s, tol=1e-8, max_iter=5000, precond="none")
    t_cg = time.perf_counter() - t0
    t0 = time.perf_counter()
    ld, per = hg.slq_logdet(X, Z, p.kernel, p.l, p.f, p.s, 30)
    t_slq = time.perf_counter() - t0
    # The FP64 MatVec at the n = 100,000, k = 33 shape (the residual
    # replacement of the refined solves uses it every 10 iterations).
    q = W.workload_fp32_matvec()
    Xq = torch.from_numpy(q.X).to(d)
    Vq = torch.from_numpy(q.extra["V"]).to(d)
    ms_big = _timed(lambda: hg.kmatvec(Xq, Vq, q.kernel, q.l, q.f, q.s), 5)
    _log("fp64 leg done")
    return dict(workload="n=2000 d=3 Gaussian f=1 l=0.5 s=0.01, FP64", matvec_ms=ms,
                cg_time_to_1em8_s=t_cg, cg_iters=int(info["iters"]),
                slq_10x30_time_s=t_slq, slq_logdet=ld, pipeline_s=ms * 1e-3 + t_cg + t_slq,
                matvec_n100000_k33_ms=ms_big,
                matvec_n100000_k33_tflops=2 * q.X.shape[0] ** 2 * 33 / (ms_big * 1e-3) / 1e12)


def leg_bf16():
    """Precision forms: n = 500,000 points in d = 8 from a 16-component
    Gaussian mixture, Gaussian l = 0.3, s = 1e-3, k = 33.  MatVec time of the
    single-BF16 and split-BF16 forms against the FP32 form; then, on the
    seeded 20,000-point subsample, PCG to 1e-6 in the FP32 form, and in the
    FP32, literal single-BF16 and split-BF16 forms with the residual
    recomputed every 10 iterations in FP64 (an FP32 recompute has a floor
    u₃₂·‖|K̂||x|‖/‖b‖ of ~1e-2 on this problem, far above the tolerance).  The true
    relative residual of each FP64 iterate is evaluated with the library's
    FP64 MatVec."""
    import torch
    import paper_2503_02259_amd as hg
    from paper_2503_02259_amd import workloads as W
    prob = W.workload_bf16_mixture()
    d = torch.device("cuda:0")
    X = torch.from_numpy(prob.X).to(d, torch.float32)
    V = torch.from_numpy(prob.extra["V"]).to(d, torch.float32)
    n, k = X.shape[0], V.shape[1]
    res = dict(workload="n=500000 d=8 16-Gaussian mixture, Gaussian l=0.3 s=1e-3, k=33")
    for prec in ("bf16", "bf16x3", "fp32"):
        ms = _timed(lambda: hg.kmatvec(X, V, 0, prob.l, prob.f, prob.s, precision=prec), 3)
        res[prec + "_matvec_ms"] = ms
        res[prec + "_kev_vec_per_s"] = float(n) * n * k / (ms * 1e-3)
    res["bf16_matvec_speedup"] = res["fp32_matvec_ms"] / res["bf16_matvec_ms"]
    res["bf16x3_matvec_speedup"] = res["fp32_matvec_ms"] / res["bf16x3_matvec_ms"]
    idx = torch.from_numpy(prob.extra["sub"]).to(d)
    Xs, Vs = X[idx].contiguous(), V[idx].contiguous()
    runs = (("fp32_pcg", dict()),
            ("fp32_pcg_refine_fp64", dict(refine_every=10, refine_prec="fp64")),
            ("bf16_pcg_refine_fp64", dict(precision="bf16", refine_every=10, refine_prec="fp64")),
            ("bf16x3_pcg_refine_fp64", dict(precision="bf16x3", refine_every=10,
                                            refine_prec="fp64")))
    for name, kw in runs:
        res[name] = _pcg_run(Xs, Vs, 0, prob, 3000, **kw)
    res["bf16x3_pcg_refine_fp64"]["speedup_vs_fp32_refine_fp64"] = (
        res["fp32_pcg_refine_fp64"]["time_s"] / res["bf16x3_pcg_refine_fp64"]["time_s"])
    _log("bf16 leg done")
    return res


def leg_grad():
    """Derivative MatVec: n = 200,000 uniform in [0,1]^3, Gaussian (f, l, s) =
    (1.0, 0.2, 0.05), k = 33, FP32: K̂V, ∂K̂/∂l·V, ∂K̂/∂f·V from one fused pass."""
    import torch
    import paper_2503_02259_amd as hg
    from paper_2503_02259_amd import workloads as W
    p = W.workload_grad()
    d = torch.device("cuda:0")
    X = torch.from_numpy(p.X).to(d, torch.float32)
    V = torch.from_numpy(np.concatenate([p.extra["y"][:, None], p.extra["Z"]], 1)).to(d, torch.float32)
    n, k = X.shape[0], V.shape[1]
    ms = _timed(lambda: hg.kmatvec_grad(X, V, 0, p.l, p.f, p.s, want=("kv", "dl", "df")), 3)
    _log("grad leg done")
    return dict(workload="n=200000 d=3 Gaussian f=1 l=0.2 s=0.05, k=33, FP32", ms=ms,
                kev_vec_per_s=float(n) * n * k / (ms * 1e-3),
                mfma_tflops=4.0 * n * n * k / (ms * 1e-3) / 1e12)


def leg_train(logdet="slq"):
    """Hyper-parameter training with the paper's end-to-end settings (Adam,
    50 steps, learning rate 0.01, 20 CG iterations per solve, FP32) on the
    n = 100,000 workload (Gaussian, start Θ = (0.1, 1, 0.01)), 16 Rademacher
    probes, 20 Lanczos steps (logdet "slq") or the tridiagonals of the 20 CG
    iterations (logdet "cg"), Jacobi, softplus parameters."""
    import torch
    from paper_2503_02259_amd import workloads as W
    from paper_2503_02259_amd.autograd import GPRModel, train_gpr
    prob = W.workload_fp32_matvec()
    d = torch.device("cuda:0")
    X = torch.from_numpy(prob.X).to(d, torch.float32)
    y = torch.from_numpy(prob.extra["y"]).to(d, torch.float32)
    Z = torch.from_numpy(prob.extra["Z"][:, :16].copy()).to(d, torch.float32)
    model = GPRModel(X, y, Z, kernel=0, l=prob.l, f=prob.f, s=prob.s,
                     opts=dict(tol=1e-6, max_iter=20, nsteps=20, logdet=logdet),
                     transform="softplus")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = train_gpr(model, steps=50, lr=0.01)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    _log("train leg (%s) done" % logdet)
    return dict(workload="n=100000 d=3 Gaussian, 50 Adam steps lr 0.01, 20 CG its, 16 probes, "
                         + ("20 Lanczos steps" if logdet == "slq" else "log-det from the CG "
                            "tridiagonals") + ", FP32", time_s=t, ms_per_step=1e3 * t / 50,
                loss_first=hist[0]["loss"], loss_last=hist[-1]["loss"], theta_final=model.get_params())


def leg_symmetric():
    """k = 1 and k = 2 FP32 MatVecs on the n = 100,000 workload (Gaussian,
    l = 0.1): the symmetric form (each kernel value of a block pair used for
    both output blocks) against the full-block form."""
    import torch
    import paper_2503_02259_amd as hg
    from paper_2503_02259_amd import workloads as W
    prob = W.workload_fp32_matvec()
    d = torch.device("cuda:0")
    X = torch.from_numpy(prob.X).to(d, torch.float32)
    out = {}
    for k in (1, 2):
        V = torch.from_numpy(prob.extra["V"][:, :k].copy()).to(d, torch.float32)
        for sym in (True, False):
            for _ in range(2):
                hg.kmatvec(X, V, 0, prob.l, prob.f, prob.s, symmetric=sym)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(10):
                hg.kmatvec(X, V, 0, prob.l, prob.f, prob.s, symmetric=sym)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / 10
            out["k%d_%s_ms" % (k, "symmetric" if sym else "full_block")] = ms
            out["k%d_%s_kev_vec_per_s" % (k, "symmetric" if sym else "full_block")] = \
                prob.X.shape[0] ** 2 * k / (ms * 1e-3)
        out["k%d_speedup" % k] = out["k%d_full_block_ms" % k] / out["k%d_symmetric_ms" % k]
    _log("symmetric leg done")
    return dict(workload="n=100000 d=3 Gaussian l=0.1 f=1 s=1e-2, V = first k columns of [y|Z], "
                         "FP32", **out)


def leg_estimators():
    """One NLML evaluation (loss and gradient) on the n = 100,000 workload
    (Gaussian, Θ = (0.1, 1, 0.01), FP32) with the E2E settings (16 probes,
    20 CG iterations, 20 Lanczos steps, Jacobi) for each estimator form:
    SLQ + Hutchinson, CG tridiagonals + Hutchinson, SLQ + Hutch++."""
    import torch
    import paper_2503_02259_amd as hg
    from paper_2503_02259_amd import workloads as W
    prob = W.workload_fp32_matvec()
    d = torch.device("cuda:0")
    X = torch.from_numpy(prob.X).to(d, torch.float32)
    y = torch.from_numpy(prob.extra["y"]).to(d, torch.float32)
    Z = torch.from_numpy(prob.extra["Z"][:, :16].copy()).to(d, torch.float32)
    out = {}
    for name, kw in (("slq_hutchinson", {}), ("cg_logdet_hutchinson", dict(logdet="cg")),
                     ("slq_hutchpp", dict(trace="hutchpp"))):
        hg.nlml(X, y, Z, 0, prob.l, prob.f, prob.s, tol=1e-6, max_iter=20, nsteps=20, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        loss, grad, info = hg.nlml(X, y, Z, 0, prob.l, prob.f, prob.s, tol=1e-6, max_iter=20,
                                   nsteps=20, **kw)
        torch.cuda.synchronize()
        out[name] = dict(time_s=time.perf_counter() - t0, loss=loss, grad=[float(g) for g in grad],
                         logdet=info["logdet"])
    _log("estimators leg done")
    return dict(workload="n=100000 d=3 Gaussian (l, f, s) = (0.1, 1, 0.01), 16 probes, 20 CG its, "
                         "20 Lanczos steps, Jacobi, FP32", **out)


def leg_paper_shape(kernel):
    """End-to-end run at the shape of the paper's on-the-fly experiments
    (Table 2: n = 30,000 training points in d = 20) with its E2E settings:
    50 Adam steps at learning rate 0.01, 20 CG iterations per solve (16
    probes × 20 Lanczos steps), FP32; then prediction of 3,000 test points
    with 50 CG iterations and a rank-100 preconditioner (Nyström here, AFN in
    the paper).  Data: the synthetic z-scored stand-in of the workloads
    module.  Start Θ = (l, f, s) = (3, 1, 0.1); softplus parameters."""
    import torch
    import paper_2503_02259_amd as hg
    from paper_2503_02259_amd import workloads as W
    from paper_2503_02259_amd.autograd import GPRModel, train_gpr
    Xtr, ytr, Xte, yte = W.workload_paper_shape()
    d = torch.device("cuda:0")
    X = torch.from_numpy(Xtr).to(d, torch.float32)
    y = torch.from_numpy(ytr).to(d, torch.float32)
    Z = torch.from_numpy(W.rademacher(Xtr.shape[0], 16, 6)).to(d, torch.float32)
    Xq = torch.from_numpy(Xte).to(d, torch.float32)
    model = GPRModel(X, y, Z, kernel=kernel, l=3.0, f=1.0, s=0.1,
                     opts=dict(tol=1e-6, max_iter=20, nsteps=20), transform="softplus")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = train_gpr(model, steps=50, lr=0.01)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    th = model.get_params()
    t0 = time.perf_counter()
    mean, _, info = hg.gpr_predict(X, y, Xq, kernel, th["l"], th["f"], th["s"], tol=1e-6,
                                   max_iter=50, precond="nystrom", rank=100)
    torch.cuda.synchronize()
    t_pred = time.perf_counter() - t0
    rmse = float(np.sqrt(np.mean((mean.double().cpu().numpy() - yte) ** 2)))
    _log("paper-shape leg (%s) done" % ("gaussian" if kernel == 0 else "matern32"))
    return dict(workload="n=30000 d=20 (z-scored synthetic), %s, 50 Adam steps lr 0.01, 20 CG its, "
                         "predict 3000 points (50 CG its, Nystrom rank 100), FP32"
                         % ("RBF" if kernel == 0 else "Matern32"),
                train_s=t_train, predict_s=t_pred, e2e_s=t_train + t_pred, test_rmse=rmse,
                loss_first=hist[0]["loss"], loss_last=hist[-1]["loss"], theta_final=th,
                paper_context="paper, 2x12-core Xeon Gold 6248R, other data of the same shape: "
                              "Table 2 E2E RBF 190.8 s (Rosenbrock 20D), Matern32 198.5 s "
                              "(Rastrigin 20D); Table 4 Matern32 at 16 cores: training 229.9 s, "
                              "inference 1.76 s")


def leg_serve(nreq, precond_rank=0, slots=8, rate=200.0):
    """Continuous batching: the first `nreq` requests of the Poisson stream
    (rate 200/s; n log-uniform in [1e3, 2e5]; d ∈ {2,3,8}; l ~ U[0.05,0.5];
    s = 1e-2; FP32), each CG to 1e-6 (Jacobi, or the Nyström preconditioner
    of rank `precond_rank`) + SLQ 16 probes × 40 steps; at most `slots`
    requests active at once.  Another `rate` replays the same requests with
    their arrival times scaled by 200/rate."""
    import torch
    from paper_2503_02259_amd import workloads as W
    from paper_2503_02259_amd.serve import Server, replay
    reqs = W.serving_stream(nreq=nreq)
    d = torch.device("cuda:0")

    def upload(r):
        return (torch.from_numpy(r.X).to(d, torch.float32), torch.from_numpy(r.y).to(d, torch.float32),
                torch.from_numpy(r.Z).to(d, torch.float32))

    stats = []

    def done(i, rid, st):
        stats.append((st.iters, st.converged, st.rounds))
        _log("serve: %d/%d done (request %d, %d CG iterations)" % (len(stats), nreq, i, st.iters))

    srv = Server(hbm_budget=128 << 30, max_active=slots)
    r = replay(reqs, srv, upload, tol=1e-6, max_iter=1000, nsteps=40, on_done=done,
               precond_rank=precond_rank, time_scale=200.0 / rate)
    srv.close()
    pc = "Nystrom rank %d" % precond_rank if precond_rank else "Jacobi"
    return dict(workload="%d of 512 Poisson requests (%g/s), CG 1e-6 (%s) + SLQ 16x40, FP32, "
                         "%d slots" % (nreq, rate, pc, slots), slots=slots,
                requests=nreq, p50_s=r["p50"], p99_s=r["p99"], solves_per_s=r["throughput"],
                span_s=r["span"], cg_iters_mean=float(np.mean([x[0] for x in stats])),
                converged=int(sum(x[1] for x in stats)))


if __name__ == "__main__":
    main()
