"""Benchmark: FP64 GMRES(30) solves of the 32^3 periodic-box workload on one GPU.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

One step is one complete solve of A s = b to a true relative residual of
1e-8: right-hand side (boundary sweep + scattering), then restarted GMRES
(formal-solution sweep, scattering GEMM, Arnoldi, Givens, cycle-end update and
true residual) until convergence.  The problem's inputs are resident in HBM
before the timed region.  Kernel durations of the scattering GEMM (the
dominant kernel), the formal solver and the Arnoldi kernels are measured with
HIP events on the stream they run on, over the timed region.  A mixed-
precision leg (FP64 iterative refinement around an inner solve with FP32
vectors and a low-precision operator) runs on the same workload after the
timed FP64 region, and the FP64 oracle is timed on the host cores on a
bounded sample of the workload.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0

WORKLOAD = ("box32: 3D box 32x32x32 periodic in x,y; 64 ordinates (8 Gauss-Legendre mu x 8 "
            "azimuths), 32 frequencies; exponential + 20% log-normal opacity; eps 1e-4; "
            "dipole x PRD kernel as a dense 2048x2048 matrix; GMRES(30) to 1e-8; FP64")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--mixed-precision", default="fp16")
    return ap.parse_args()


def percentile(v, q):
    s = sorted(v)
    if not s:
        return None
    i = min(len(s) - 1, max(0, int(round(q / 100.0 * (len(s) - 1)))))
    return s[i]


def cpu_baseline(spec, gpu_iters, gpu_cycles):
    """Time the FP64 oracle on the host on a bounded sample of the workload:
    the right-hand side, one operator application and (if cheap enough) two
    GMRES iterations; scale to one solve with the GPU run's iteration and
    cycle counts."""
    import numpy as np
    from oracle import Problem as OProblem, gmres
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = 1
    t0 = time.perf_counter()
    op = OProblem(spec)
    b = op.rhs()
    t_rhs = time.perf_counter() - t0
    x = np.random.default_rng(0).standard_normal(op.n)
    t0 = time.perf_counter()
    op.apply(x)
    t_apply = time.perf_counter() - t0
    sample = "oracle set-up + right-hand side, one operator application"
    t_iter = t_apply
    if t_apply < 8.0:
        t0 = time.perf_counter()
        gmres(op.apply, b, restart=30, tol=1e-30, maxiter=2)
        t_g = time.perf_counter() - t0
        # two Arnoldi steps plus the initial and the final residual applications
        t_iter = max(t_apply, (t_g - 2.0 * t_apply) / 2.0)
        sample += ", two GMRES(30) iterations"
    t_solve = t_rhs + gpu_iters * t_iter + gpu_cycles * t_apply
    sample += (f" on the full box32 workload; scaled to one solve with the GPU run's "
               f"{gpu_iters} iterations and {gpu_cycles} restart cycles "
               f"(t_rhs={t_rhs:.2f}s, t_apply={t_apply:.2f}s, t_iter={t_iter:.2f}s)")
    return {"value": 1.0 / t_solve, "unit": "solves/s", "cores": int(threads),
            "kind": "oracle", "sample": sample}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}),
              file=sys.stderr)
        sys.exit(2)
    import torch
    import workloads as W
    from paper_2602_21958_amd import rt

    dev = torch.device("cuda:0")
    spec = W.box32()
    p = rt.Problem(spec, 0)
    n, n_r, n_s = p.n, p.n_r, p.n_s
    x = torch.empty(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        p.solve(x, rtol=1e-8, restart=30, stream=stream)
    torch.cuda.synchronize()

    rt.profile_enable(True)
    for k in ("lambda", "sigma", "arnoldi"):
        rt.profile_read(k, reset=True)
    lat, stats = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        st = p.solve(x, rtol=1e-8, restart=30, stream=stream)
        lat.append((time.perf_counter() - ts) * 1e3)
        stats.append(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rt.profile_enable(False)
    prof = {k: rt.profile_read(k, reset=True) for k in ("lambda", "sigma", "arnoldi")}

    elapsed = t1 - t0
    value = args.steps / elapsed
    ok = all(s["converged"] and s["relres"] <= 1e-8 for s in stats)

    sig_n, sig_ms = prof["sigma"]
    sig_avg = sig_ms / max(sig_n, 1)
    sig_flops = 2.0 * n_r * n_r * n_s
    sig_tf = sig_flops / (sig_avg * 1e-3) / 1e12
    lam_n, lam_ms = prof["lambda"]
    lam_avg = lam_ms / max(lam_n, 1)
    lam_bytes = 16.0 * n
    lam_gbs = lam_bytes / (lam_avg * 1e-3) / 1e9
    arn_n, arn_ms = prof["arnoldi"]

    out = {
        "metric": "solves/s to 1e-8 residual, mixed vs FP64; Λ HBM GB/s; Σ MFMA util; p99 ms",
        "value": value,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n_unknowns": n, "n_rays": n_r, "n_points": n_s,
                   "restart": 30, "rtol": 1e-8},
        "converged": ok,
        "iters": stats[-1]["iters"],
        "restart_cycles": stats[-1]["outer_iters"],
        "relres": stats[-1]["relres"],
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
        "roofline": {"kernel": "sigma_gemm_kernel<double> (FP64 MFMA 16x16x4)",
                     "bound": "mfma", "achieved": sig_tf, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": sig_tf / PEAK_FP64_TFLOPS, "traffic": None,
                     "launches": sig_n, "avg_ms": sig_avg,
                     "algorithmic_per_launch": f"2*N_r^2*N_s = {sig_flops:.4g} flop"},
        "lambda": {"kernel": "lambda_box_kernel<double>", "bound": "hbm", "achieved": lam_gbs,
                   "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": lam_gbs / PEAK_HBM_GBS,
                   "launches": lam_n, "avg_ms": lam_avg,
                   "algorithmic_per_launch": f"16 B x N = {lam_bytes:.4g} B"},
        "arnoldi": {"launches": arn_n, "total_ms_per_solve": arn_ms / args.steps},
    }

    if not args.no_mixed:
        prec = args.mixed_precision
        xm = torch.empty_like(x)
        p.solve(xm, rtol=1e-8, restart=30, precision=prec, stream=stream)  # warm
        torch.cuda.synchronize()
        rt.profile_enable(True)
        rt.profile_read("sigma", reset=True)
        m_steps = max(1, args.steps)
        tm0 = time.perf_counter()
        mst = None
        for _ in range(m_steps):
            mst = p.solve(xm, rtol=1e-8, restart=30, precision=prec, stream=stream)
        torch.cuda.synchronize()
        tm1 = time.perf_counter()
        rt.profile_enable(False)
        ms_n, ms_ms = rt.profile_read("sigma", reset=True)
        diff = (torch.linalg.vector_norm(xm - x) / torch.linalg.vector_norm(x)).item()
        out["mixed"] = {"precision": prec, "value": m_steps / (tm1 - tm0), "unit": "solves/s",
                        "speedup_vs_fp64": (m_steps / (tm1 - tm0)) / value,
                        "relres_fp64": mst["relres"], "converged": mst["converged"],
                        "inner_iters": mst["iters"], "outer_iters": mst["outer_iters"],
                        "rel_diff_vs_fp64_solution": diff,
                        "sigma_avg_ms": ms_ms / max(ms_n, 1)}

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, stats[-1]["iters"], stats[-1]["outer_iters"])

    p.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
