"""Benchmark of the S_N radiative-transfer Krylov path on one GPU.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
                [--no-box64] [--workload box32|batch512|serve|box64|slab64]

Default workload (box32): FP64 GMRES(30) solves of the 32^3 periodic box.

One step is one complete solve of A s = b to a true relative residual of
1e-8: right-hand side (boundary sweep + scattering), then restarted GMRES
(formal-solution sweep, scattering GEMM, Arnoldi, Givens, cycle-end update and
true residual) until convergence.  The problem's inputs are resident in HBM
before the timed region.  Kernel durations of the scattering GEMM (the
dominant kernel), the formal solver and the Arnoldi kernels are measured with
HIP events on the stream they run on, over the timed region.  A mixed-
precision leg (FP64 iterative refinement around an inner solve with FP32
vectors and a low-precision operator) runs on the same workload after the
timed FP64 region, then the same FP64 solve with the scattering step in
factored form (dipole rank 6 x frequency block, bound by HBM), and the FP64
oracle is timed on the host cores on a bounded sample of the workload.  A
second leg solves the 64^3 box (1.61e9 unknowns) in mixed precision
(16-bit or factored FP32 scattering, FP64 refinement): one timed solve per
variant, the kernel rates of its 16-bit GEMM and FP32 sweep, and the
oracle's FP64 residual of its solution (host processes, a few minutes).
Prints one JSON line.
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

# HBM traffic of the dominant kernels from two rocprofv3 --pmc passes
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, mean over the dispatches of
# one solve), scaled by what the same counters read for a 2 GiB device copy
# (read x2.000, write x1.000).  Each entry holds a hash of the kernel's
# sources and of the code that chooses its launches (the solver decides
# whether a GEMM reads x) at the time of measurement: once they change the
# figure is stale and the bench reports null.
TRAFFIC = {
    "sigma_f64_box32": {"files": ("gemm_dev.h", "sigma_gemm.hip", "solver.cpp", "abi.cpp"),
                        "sha": "8bad2c284fd50c9e",
                        "fetch_kib": 1.341e6, "write_kib": 5.243e5,
                        "fetch_scale": 2.000, "write_scale": 1.000,
                        "profile": "profiles/sigma_gemm_f64_box32_counters.md"},
}


def source_hash(files):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2602_21958_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_bytes(key):
    """Calibrated HBM bytes per launch, or None when the kernel changed."""
    t = TRAFFIC.get(key)
    if t is None or source_hash(t["files"]) != t["sha"]:
        return None
    return (t["fetch_kib"] * t["fetch_scale"] + t["write_kib"] * t["write_scale"]) * 1024.0


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
    ap.add_argument("--no-box64", action="store_true",
                    help="default run: skip the 64^3 mixed-precision leg")
    ap.add_argument("--oracle-procs", type=int, default=12,
                    help="host processes of the oracle's box64 sweeps (cpu_baseline leg)")
    ap.add_argument("--mixed-precision", default="fp16")
    ap.add_argument("--workload", default="box32",
                    choices=["box32", "batch512", "serve", "box64", "slab64", "apply",
                             "solve"])
    ap.add_argument("--problem", default="box64", choices=["box32", "box64", "slab64"],
                    help="apply / solve: the problem whose operator is applied or solved")
    ap.add_argument("--precond", default="none", choices=["none", "local"],
                    help="solve: the physics-based preconditioner")
    ap.add_argument("--restart", type=int, default=30, help="solve: GMRES restart length")
    ap.add_argument("--sigma-form", default="dense", choices=["dense", "factored", "ozaki"],
                    help="apply: scattering form of FP64 / FP32 applications")
    ap.add_argument("--precision", default=None,
                    help="operator precision for batch512 / serve / box64")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: stream length (s)")
    ap.add_argument("--basis16", action="store_true",
                    help="serve: fp16 Krylov bases in the engine (16-bit precisions)")
    ap.add_argument("--rate", type=float, default=200.0, help="serve: arrivals per second")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 2 GiB device-to-device copy before the timed region; its "
                         "memory counters calibrate the HBM traffic of the other kernels")
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
        print(json.dumps({"error": "the solver runs on one GPU (a problem and its workspace live on one device); --gpus must be 1"}),
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch512":
        return bench_batch512(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "box64":
        return bench_box64(args)
    if args.workload == "slab64":
        return bench_slab64(args)
    if args.workload == "solve":
        return bench_solve(args)
    if args.workload == "apply":
        return bench_apply(args)
    import torch
    import workloads as W
    from paper_2602_21958_amd import rt

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        copy_calibration()
    spec = W.box32()
    p = rt.Problem(spec, 0)
    n, n_r, n_s = p.n, p.n_r, p.n_s
    x = torch.empty(n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        p.solve(x, rtol=1e-8, restart=30, stream=stream)
    torch.cuda.synchronize()

    rt.profile_enable(True)
    for k in rt.KCLASS:
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
    prof = {k: rt.profile_read(k, reset=True) for k in rt.KCLASS}

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
                     "unit": "TFLOP/s", "frac": sig_tf / PEAK_FP64_TFLOPS,
                     "traffic": traffic_bytes("sigma_f64_box32"),
                     "traffic_unit": "B per launch (calibrated FETCH_SIZE + WRITE_SIZE)",
                     "launches": sig_n, "avg_ms": sig_avg,
                     "algorithmic_per_launch": f"2*N_r^2*N_s = {sig_flops:.4g} flop"},
        "lambda": {"kernel": "lambda_box_kernel<double>", "bound": "hbm", "achieved": lam_gbs,
                   "peak": PEAK_HBM_GBS, "unit": "GB/s", "frac": lam_gbs / PEAK_HBM_GBS,
                   "launches": lam_n, "avg_ms": lam_avg,
                   "algorithmic_per_launch": f"16 B x N = {lam_bytes:.4g} B"},
        "arnoldi": {"launches": arn_n, "total_ms_per_solve": arn_ms / args.steps},
    }

    # the same FP64 solve with one Arnoldi step per pass over the basis (the
    # library's default takes them in pairs: one dots and one update pass
    # over the basis per two steps)
    x2 = torch.empty_like(x)
    p.solve(x2, rtol=1e-8, restart=30, two_step=0, stream=stream)  # warm
    torch.cuda.synchronize()
    rt.profile_enable(True)
    rt.profile_read("arnoldi", reset=True)
    t2a = time.perf_counter()
    st2 = None
    for _ in range(args.steps):
        st2 = p.solve(x2, rtol=1e-8, restart=30, two_step=0, stream=stream)
    torch.cuda.synchronize()
    t2b = time.perf_counter()
    rt.profile_enable(False)
    a2_n, a2_ms = rt.profile_read("arnoldi", reset=True)
    out["fp64_one_step"] = {
        "value": args.steps / (t2b - t2a), "unit": "solves/s",
        "converged": st2["converged"], "relres": st2["relres"], "iters": st2["iters"],
        "rel_diff_vs_fp64_solution":
            (torch.linalg.vector_norm(x2 - x) / torch.linalg.vector_norm(x)).item(),
        "arnoldi_ms_per_solve": a2_ms / args.steps}

    if not args.no_mixed:
        prec = args.mixed_precision
        xm = torch.empty_like(x)
        p.solve(xm, rtol=1e-8, restart=30, precision=prec, stream=stream)  # warm
        torch.cuda.synchronize()
        rt.profile_enable(True)
        _profile_summary(rt)
        m_steps = max(1, args.steps)
        tm0 = time.perf_counter()
        mst = None
        for _ in range(m_steps):
            mst = p.solve(xm, rtol=1e-8, restart=30, precision=prec, stream=stream)
        torch.cuda.synchronize()
        tm1 = time.perf_counter()
        rt.profile_enable(False)
        mprof = _profile_summary(rt)
        lo_n, lo_ms = mprof["sigma_lo"]["launches"], mprof["sigma_lo"]["total_ms"]
        hi_n, hi_ms = mprof["sigma"]["launches"], mprof["sigma"]["total_ms"]
        diff = (torch.linalg.vector_norm(xm - x) / torch.linalg.vector_norm(x)).item()
        out["mixed"] = {"precision": prec, "value": m_steps / (tm1 - tm0), "unit": "solves/s",
                        "speedup_vs_fp64": (m_steps / (tm1 - tm0)) / value,
                        "relres_fp64": mst["relres"], "converged": mst["converged"],
                        "inner_iters": mst["iters"], "outer_iters": mst["outer_iters"],
                        "rel_diff_vs_fp64_solution": diff,
                        "inner_sigma": {
                            "kernel": (f"sigma16 {prec} " + p.gemm16_tile(prec))
                            if prec in ("bf16", "fp16", "bf16x3") else "FP32 MFMA 128x128",
                            "launches": lo_n, "avg_ms": lo_ms / max(lo_n, 1),
                            "TFLOP/s": sig_flops / (lo_ms / max(lo_n, 1) * 1e-3) / 1e12},
                        "outer_sigma_fp64": {
                            "launches": hi_n, "avg_ms": hi_ms / max(hi_n, 1),
                            "TFLOP/s": sig_flops / (hi_ms / max(hi_n, 1) * 1e-3) / 1e12
                            if hi_n else None},
                        "kernel_ms_per_solve": {k: v["total_ms"] / m_steps
                                                for k, v in mprof.items()}}
        if prec in ("bf16", "fp16", "bf16x3"):
            # the same refinement with the inner Krylov basis kept in fp16
            p.solve(xm, rtol=1e-8, restart=30, precision=prec, basis_fp16=1, stream=stream)
            torch.cuda.synchronize()
            tm0 = time.perf_counter()
            for _ in range(m_steps):
                hst = p.solve(xm, rtol=1e-8, restart=30, precision=prec, basis_fp16=1,
                              stream=stream)
            torch.cuda.synchronize()
            tm1 = time.perf_counter()
            diff = (torch.linalg.vector_norm(xm - x) / torch.linalg.vector_norm(x)).item()
            out["mixed"]["fp16_basis"] = {
                "value": m_steps / (tm1 - tm0), "unit": "solves/s",
                "speedup_vs_fp64": (m_steps / (tm1 - tm0)) / value,
                "relres_fp64": hst["relres"], "converged": hst["converged"],
                "inner_iters": hst["iters"], "outer_iters": hst["outer_iters"],
                "rel_diff_vs_fp64_solution": diff}

    # the same FP64 solve with the scattering step in factored form (dipole
    # rank 6 x frequency block: HBM-bound passes instead of the dense GEMM)
    print("box32: factored FP64 leg", file=sys.stderr, flush=True)
    p.set_sigma("factored")
    xf = torch.empty_like(x)
    p.solve(xf, rtol=1e-8, restart=30, stream=stream)  # warm
    torch.cuda.synchronize()
    rt.profile_enable(True)
    _profile_summary(rt)
    tf0 = time.perf_counter()
    stf = None
    for _ in range(args.steps):
        stf = p.solve(xf, rtol=1e-8, restart=30, stream=stream)
    torch.cuda.synchronize()
    tf1 = time.perf_counter()
    rt.profile_enable(False)
    fprof = _profile_summary(rt)
    # the factored passes alone, y = (1 - eps) Mhat L (no x term, as in the
    # Arnoldi steps): read L, write y, and W, Z of R x N_nu x N_s each
    # written once and read once
    yf = torch.empty_like(x)
    for _ in range(2):
        p.apply_sigma(x, None, yf, stream=stream)
    torch.cuda.synchronize()
    rt.profile_enable(True)
    _profile_summary(rt)
    for _ in range(5):
        p.apply_sigma(x, None, yf, stream=stream)
    torch.cuda.synchronize()
    rt.profile_enable(False)
    aprof = _profile_summary(rt)
    del yf
    p.set_sigma("dense")
    rank = p.footprint().sigma_rank
    n_nu_b, n_om_b = spec.n_nu, spec.n_omega
    f_n, f_ms = aprof["sigma"]["launches"], aprof["sigma"]["total_ms"]
    f_avg = f_ms / max(f_n, 1)
    wz = rank * n_nu_b * n_s
    f_bytes = 8.0 * (2 * n + 4 * wz)
    out["fp64_factored_sigma"] = {
        "value": args.steps / (tf1 - tf0), "unit": "solves/s",
        "speedup_vs_dense": (args.steps / (tf1 - tf0)) / value,
        "converged": stf["converged"], "relres": stf["relres"], "iters": stf["iters"],
        "rel_diff_vs_dense_solution":
            (torch.linalg.vector_norm(xf - x) / torch.linalg.vector_norm(x)).item(),
        "sigma_ms_per_solve_in_solves": fprof["sigma"]["total_ms"] / args.steps,
        "kernel_ms_per_solve": {k: v["total_ms"] / args.steps for k, v in fprof.items()},
        "flop_per_apply": {"dense": sig_flops,
                           "factored": 4.0 * rank * n + 2.0 * rank * n_nu_b * n_nu_b * n_s},
        "roofline": {"kernel": "fsig_reduce + fsig_mix + fsig_expand <double>", "bound": "hbm",
                     "achieved": f_bytes / (f_avg * 1e-3) / 1e9, "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": f_bytes / (f_avg * 1e-3) / 1e9 / PEAK_HBM_GBS,
                     "avg_ms": f_avg, "launches": f_n,
                     "algorithmic_per_launch": f"read L, write y (16 B x N) + W and Z "
                                               f"({rank} x N_nu x N_s doubles each, written "
                                               f"and read) = {f_bytes:.4g} B"},
    }

    # the same system with the physics-based preconditioner (right
    # preconditioning: the same residual and tolerance), in FP64 and in the
    # mixed precision, with the dense and the factored scattering form (FP64
    # outer residuals and, for fp32, the inner operator); the first solve
    # builds the preconditioner's tables
    print("box32: preconditioned legs", file=sys.stderr, flush=True)
    out["preconditioned"] = {}
    xp = torch.empty_like(x)
    for label, form, kw in (("fp64", "dense", {}),
                            (args.mixed_precision, "dense", {"precision": args.mixed_precision}),
                            ("fp64/factored", "factored", {}),
                            ("fp32/factored", "factored", {"precision": "fp32"}),
                            ("fp32/factored/basis16", "factored",
                             {"precision": "fp32", "basis_fp16": 1})):
        p.set_sigma(form)
        tp0 = time.perf_counter()
        p.solve(xp, rtol=1e-8, restart=30, precond="local", stream=stream, **kw)
        torch.cuda.synchronize()
        t_first = time.perf_counter() - tp0
        rt.profile_enable(True)
        _profile_summary(rt)
        tp0 = time.perf_counter()
        pst = None
        for _ in range(args.steps):
            pst = p.solve(xp, rtol=1e-8, restart=30, precond="local", stream=stream, **kw)
        torch.cuda.synchronize()
        tp1 = time.perf_counter()
        rt.profile_enable(False)
        pprof = _profile_summary(rt)
        out["preconditioned"][label] = {
            "value": args.steps / (tp1 - tp0), "unit": "solves/s",
            "speedup_vs_fp64": (args.steps / (tp1 - tp0)) / value,
            "converged": pst["converged"], "relres_fp64": pst["relres"],
            "iters": pst["iters"], "outer_iters": pst["outer_iters"],
            "rel_diff_vs_fp64_solution":
                (torch.linalg.vector_norm(xp - x) / torch.linalg.vector_norm(x)).item(),
            "first_solve_s_incl_setup": t_first,
            "kernel_ms_per_solve": {k: v["total_ms"] / args.steps for k, v in pprof.items()}}
    p.set_sigma("dense")
    del xp

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, stats[-1]["iters"], stats[-1]["outer_iters"])
    p.close()
    del x, x2
    if not args.no_mixed:
        del xm
    del xf
    torch.cuda.empty_cache()

    if not args.no_box64:
        out["box64"] = box64_leg(BOX64_DEFAULT, oracle_check=not args.no_cpu_baseline,
                                 procs=args.oracle_procs)
    print(json.dumps(out), flush=True)


# --------------------------------------------------------------------------
def _profile_summary(rt, names=None):
    names = rt.KCLASS if names is None else names
    return {k: dict(zip(("launches", "total_ms"), rt.profile_read(k, reset=True))) for k in names}


def bench_batch512(args):
    """512 independent slabs (N_z, N_nu, N_mu, eps, depth drawn per slab) in one
    engine; one step = all 512 solved to the FP64 1e-8 residual."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2602_21958_amd import rt

    prec = args.precision or "bf16x3"
    specs = W.batch_slabs(512)
    probs = [rt.Problem(s) for s in specs]
    n_tot = sum(p.n for p in probs)
    xs = [torch.empty(p.n, dtype=torch.float64, device="cuda:0") for p in probs]

    def run(precision, profile=False, basis_fp16=False, precond="none"):
        eng = rt.Batch(precision=precision, hbm_budget=64 << 30, max_slots=512,
                       basis_fp16=basis_fp16)
        tk = [eng.submit(p, x, restart=30, rtol=1e-8, max_iters=4000, max_outer=200,
                         precond=precond)
              for p, x in zip(probs, xs)]
        if profile:
            rt.profile_enable(True)
            _profile_summary(rt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 0
        while eng.step() > 0:
            steps += 1
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = None
        if profile:
            rt.profile_enable(False)
            prof = _profile_summary(rt)
        st = [eng.poll(t) for t in tk]
        run.tile = eng.gemm16_tile()
        eng.close()
        return el, steps, st, prof

    for _ in range(args.warmup):
        run(prec)
    times, st, prof, steps = [], None, None, 0
    for k in range(args.steps):
        el, steps, st, pr = run(prec, profile=(k == args.steps - 1))
        times.append(el)
        prof = pr or prof
    tile = run.tile
    el = sum(times) / len(times)
    conv = sum(1 for s in st if s["converged"])
    its = np.array([s["iters"] for s in st])
    variants = {}
    for v, b16 in (("fp64", False), ("fp16", False), ("bf16", False), ("fp16", True),
                   (prec, True)):
        if v == prec and not b16:
            continue
        label = v + ("/basis16" if b16 else "")
        if label in variants:
            continue
        e2, s2, st2, _ = run(v, basis_fp16=b16)
        variants[label] = {"solves_per_s": 512 / e2,
                           "converged": sum(1 for s in st2 if s["converged"]),
                           "iters_median": float(np.median([s["iters"] for s in st2])),
                           "steps": s2}
    # the physics-based preconditioner on every slab (its tables are built
    # on each problem at its first admission: an untimed run first)
    for v in (prec, "fp64"):
        run(v, precond="local")
        e2, s2, st2, _ = run(v, precond="local")
        variants[v + "/precond"] = {
            "solves_per_s": 512 / e2, "converged": sum(1 for s in st2 if s["converged"]),
            "iters_median": float(np.median([s["iters"] for s in st2])),
            "iters_max": int(max(s["iters"] for s in st2)), "steps": s2}
    # per-slab FP64 loop through the single-problem solver on a sample
    sample = list(range(0, 512, 16))
    t0 = time.perf_counter()
    for i in sample:
        probs[i].solve(xs[i], rtol=1e-8, restart=30, record_history=0)
    torch.cuda.synchronize()
    loop_per_slab = (time.perf_counter() - t0) / len(sample)
    sig = prof["sigma" if prec == "fp64" else "sigma_lo"]
    out = {
        "metric": "solves/s to 1e-8 residual (512 heterogeneous slabs, one engine)",
        "value": 512 / el, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": el * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": "batch512: 512 slabs, N_z~U[32,256], N_nu~U[16,64], "
                               "N_mu in {8..16}, eps log-U[1e-6,1e-2], depth log-U[1e2,1e6]; "
                               f"FP32 Lambda + {prec} Sigma + FP64 refinement; GMRES(30) "
                               "inner cycles; hipGraph-replayed engine steps",
                   "n_unknowns_total": n_tot},
        "converged": conv, "engine_steps": steps,
        "iters": {"median": float(np.median(its)), "p90": float(np.percentile(its, 90)),
                  "max": int(its.max()), "min": int(its.min())},
        "kernel_ms_per_run": {k: v["total_ms"] for k, v in prof.items()},
        "variants": variants,
        "per_slab_fp64_loop": {"s_per_slab": loop_per_slab, "solves_per_s": 1 / loop_per_slab,
                               "sample": f"{len(sample)} slabs through rt_solve FP64",
                               "engine_speedup": (512 / el) * loop_per_slab},
        "sigma_avg_ms": sig["total_ms"] / max(sig["launches"], 1),
        "sigma_tile": tile,
    }
    if not args.no_cpu_baseline:
        from oracle import Problem as OProblem, gmres
        t0 = time.perf_counter()
        done = 0
        for i in range(0, 512, 64):
            op = OProblem(specs[i])
            gmres(op.apply, op.rhs(), restart=30, tol=1e-8)
            done += 1
            if time.perf_counter() - t0 > 20:
                break
        per = (time.perf_counter() - t0) / done
        out["cpu_baseline"] = {"value": 1 / per, "unit": "solves/s", "cores": _threads(),
                               "kind": "oracle",
                               "sample": f"full oracle GMRES(30) solves of {done} of the 512 "
                                         "slabs (every 64th); solves/s = 1 / mean time"}
    for p in probs:
        p.close()
    print(json.dumps(out), flush=True)


def _threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [1]))
    except Exception:
        return 1


def bench_serve(args):
    """Continuous batching: Poisson arrivals (90 % slabs, 10 % 16^3 boxes); a
    producer thread builds each request's problem at its arrival time, the
    main loop submits and steps the engine; latency = completion - arrival."""
    import queue as pyqueue
    import threading
    import numpy as np
    import torch
    import workloads as W
    from paper_2602_21958_amd import rt

    prec = args.precision or "bf16x3"
    stream = W.serve_stream(duration_s=args.duration, rate_hz=args.rate)
    eng = rt.Batch(precision=prec, hbm_budget=96 << 30, max_slots=1024,
                   basis_fp16=args.basis16)
    ready = pyqueue.Queue()
    t_start = time.perf_counter() + 0.5

    def producer(lo, step):
        for i in range(lo, len(stream), step):
            t_arr, kind, seed = stream[i]
            delay = t_start + t_arr - time.perf_counter()
            if delay > 0:
                time.sleep(delay)
            spec = W.serve_request(kind, seed)
            ready.put((i, t_arr, kind, rt.Problem(spec)))

    threads = [threading.Thread(target=producer, args=(k, 4), daemon=True) for k in range(4)]
    for th in threads:
        th.start()
    live = {}
    lat = {"slab": [], "box": []}
    timeline = []
    done = 0
    n_req = len(stream)
    last_tl = 0.0
    while done < n_req:
        try:
            while True:
                i, t_arr, kind, prob = ready.get_nowait()
                x = torch.empty(prob.n, dtype=torch.float64, device="cuda:0")
                tk = eng.submit(prob, x, restart=30, rtol=1e-8, max_iters=4000, max_outer=200,
                                record_history=0)
                live[tk] = (t_arr, kind, prob, x)
        except pyqueue.Empty:
            pass
        if live:
            eng.step()
        else:
            time.sleep(0.0005)
        now = time.perf_counter() - t_start
        for tk in list(live):
            st = eng.poll(tk)
            if st is not None:
                t_arr, kind, prob, x = live.pop(tk)
                lat[kind].append((now - t_arr) * 1e3 if st["converged"] else float("nan"))
                prob.close()
                done += 1
        if now - last_tl >= 1.0:
            inf = eng.info()
            timeline.append([round(now, 2), inf["active"], inf["queued"], done,
                             round(inf["bytes_in_use"] / 2**30, 2)])
            last_tl = now
    wall = time.perf_counter() - t_start
    allv = np.array([v for k in lat for v in lat[k]])
    ok = allv[np.isfinite(allv)]
    out = {
        "metric": "serving: p50/p99 latency (ms) and solves/s, 1e-8 residual",
        "value": len(ok) / wall, "unit": "solves/s", "n_gpus": 1, "steps": n_req, "warmup": 0,
        "ms_per_step": wall * 1e3 / max(n_req, 1), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": prec, "data": "synthetic",
        "config": {"workload": f"serve: Poisson {args.rate}/s for {args.duration}s, 90% slabs "
                               "(batch512 recipe) / 10% 16^3 boxes (4 mu x 8 az, 24 freq); "
                               f"{prec} Sigma + FP32 Lambda + FP64 refinement; admission by "
                               "HBM footprint (96 GiB arena)",
                   "krylov_basis": "fp16" if args.basis16 else "fp32"},
        "requests": n_req, "converged": int(len(ok)),
        "latency_ms": {"p50": float(np.percentile(ok, 50)), "p99": float(np.percentile(ok, 99)),
                       "slab_p50": float(np.nanpercentile(lat["slab"], 50)) if lat["slab"] else None,
                       "box_p50": float(np.nanpercentile(lat["box"], 50)) if lat["box"] else None,
                       "box_p99": float(np.nanpercentile(lat["box"], 99)) if lat["box"] else None},
        "timeline_t_active_queued_done_GiB": timeline[:: max(1, len(timeline) // 30)],
    }
    eng.close()
    print(json.dumps(out), flush=True)


def bench_slab64(args):
    """The 1D slab (64 depths, 8 mu, 21 frequencies, N = 10 752) in FP64:
    K GMRES(30) solves to 1e-8; the oracle's full solve is the CPU baseline."""
    import torch
    import workloads as W
    from paper_2602_21958_amd import rt

    spec = W.slab64()
    p = rt.Problem(spec)
    x = torch.empty(p.n, dtype=torch.float64, device="cuda:0")
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        p.solve(x, rtol=1e-8, restart=30, stream=stream)
    torch.cuda.synchronize()
    lat, st = [], None
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        st = p.solve(x, rtol=1e-8, restart=30, stream=stream)
        lat.append((time.perf_counter() - ts) * 1e3)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    out = {
        "metric": "solves/s to 1e-8 residual (1D slab, FP64)", "value": args.steps / el,
        "unit": "solves/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": el * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "slab64: 64 log-spaced depths (tau_c 1e-4..1e4), 8 mu, 21 "
                               "frequencies, eps 1e-4, dipole x PRD; GMRES(30) to 1e-8; FP64",
                   "n_unknowns": p.n},
        "converged": st["converged"], "iters": st["iters"], "relres": st["relres"],
        "latency_ms": {"p50": percentile(lat, 50), "p99": percentile(lat, 99)},
    }
    if not args.no_cpu_baseline:
        from oracle import Problem as OProblem, gmres
        t0 = time.perf_counter()
        op = OProblem(spec)
        ref = gmres(op.apply, op.rhs().ravel(), restart=30, tol=1e-8)
        t_or = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 1.0 / t_or, "unit": "solves/s", "cores": _blas_threads(),
                               "kind": "oracle",
                               "sample": f"one full oracle GMRES(30) solve ({ref['iters']} "
                                         f"iterations, set-up included)"}
    p.close()
    print(json.dumps(out), flush=True)


def _blas_threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] or [1]))
    except Exception:
        return 1


# ---------------------------------------------------------------- box64
# (label, operator precision, inner restart, fp16 basis, scattering form of
# the FP64 / FP32 applications[, preconditioner]; the 16-bit inner operators are always the
# dense GEMM, so "factored" or "ozaki" (the FP64 GEMM emulated with int8
# products) with a 16-bit precision changes only the FP64 outer residuals):
# the default run's box64 leg, then the rest of the variants that
# --workload box64 times.  An fp16 basis leaves room for GMRES(30) inner
# cycles; an FP32 GMRES(30) basis would not fit 288 GB beside the FP64
# vectors, so FP32-basis variants take GMRES(20).
BOX64_DEFAULT = [("fp16/basis16/m30", "fp16", 30, 1, "dense"),
                 ("fp16/basis16/m30/ozaki-outer", "fp16", 30, 1, "ozaki"),
                 ("bf16/basis16/m30", "bf16", 30, 1, "dense"),
                 ("fp16/basis16/m30/factored-outer", "fp16", 30, 1, "factored"),
                 ("fp16/m20/precond", "fp16", 20, 0, "dense", "local"),
                 ("fp16/m20/precond/factored-outer", "fp16", 20, 0, "factored", "local"),
                 ("fp32/factored/m20/precond", "fp32", 20, 0, "factored", "local"),
                 ("fp32/factored/basis16/m20/precond", "fp32", 20, 1, "factored", "local")]
BOX64_MORE = [("fp32/factored/m20", "fp32", 20, 0, "factored"),
              ("bf16/m20/precond/factored-outer", "bf16", 20, 0, "factored", "local"),
              ("fp16/m20", "fp16", 20, 0, "dense"), ("bf16/m20", "bf16", 20, 0, "dense"),
              ("bf16x3/m20", "bf16x3", 20, 0, "dense"), ("fp32/m20", "fp32", 20, 0, "dense")]


_SWEEP = {}


def _sweep_init(k_line, omega, fac_nu, i_top, i_bot):
    _SWEEP.update(k_line=k_line, omega=omega, fac_nu=fac_nu, i_top=i_top, i_bot=i_bot)


def _sweep_worker(job):
    """Oracle sweeps of one ordinate (spawned host process): the intensity
    with boundary radiation for the source s_o (Lambda_0 s + I_bc) and for a
    zero source (I_bc)."""
    import numpy as np
    from oracle.transfer import sweep_box
    o, s_o = job
    g = _SWEEP
    om = g["omega"][o:o + 1]
    i_x = sweep_box(g["k_line"], om, g["fac_nu"], s_o[None], g["i_top"], g["i_bot"])
    i_0 = sweep_box(g["k_line"], om, g["fac_nu"], np.zeros_like(s_o)[None], g["i_top"],
                    g["i_bot"])
    return o, i_x, i_0


def oracle_residual_box(spec, x_host, procs):
    """FP64 relative residual ||b - A x|| / ||b|| of a box solution, evaluated
    by the oracle: its sweeps (one ordinate per task over `procs` spawned
    host processes, which never touch the GPU) and its scattering block,
    chunked over points.  With I_x = Lambda_0 x + I_bc and I_bc the sweeps of
    x and of a zero source with boundary radiation, b = (1 - eps) Mhat I_bc
    + t and b - A x = (1 - eps) Mhat I_x + t - x (the sweep is linear in the
    source).  Returns the residual and the host seconds of the sweeps and of
    the products."""
    import multiprocessing as mp
    import numpy as np
    from oracle import Problem as OProblem
    op = OProblem(spec)
    n_om, n_nu = op.n_omega, op.n_nu
    shape = (n_om, n_nu * spec.nz * spec.ny * spec.nx)
    src = np.asarray(x_host, dtype=np.float64).reshape(shape)
    i_x = np.empty(shape)
    i_0 = np.empty(shape)
    sub = (n_nu, spec.nz, spec.ny, spec.nx)
    t0 = time.perf_counter()
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS")}
    os.environ["OMP_NUM_THREADS"] = os.environ["OPENBLAS_NUM_THREADS"] = "1"
    try:
        ctx = mp.get_context("spawn")
        with ctx.Pool(procs, initializer=_sweep_init,
                      initargs=(np.asarray(spec.k_line, float), op.omega, op.phi + spec.r,
                                spec.i_top, spec.i_bot)) as pool:
            jobs = ((o, src[o].reshape(sub)) for o in range(n_om))
            done = 0
            for o, a, b in pool.imap_unordered(_sweep_worker, jobs):
                i_x[o] = a.reshape(-1)
                i_0[o] = b.reshape(-1)
                done += 1
                if done % 16 == 0:
                    print(f"oracle residual: {done}/{n_om} ordinates swept "
                          f"({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    assert done == n_om
    t_sweep = time.perf_counter() - t0
    ix = i_x.reshape(op.n_r, op.n_s)
    i0 = i_0.reshape(op.n_r, op.n_s)
    xs = src.reshape(op.n_r, op.n_s)
    t0 = time.perf_counter()
    rr = bb = 0.0
    step = 16384
    for c in range(0, op.n_s, step):
        sl = slice(c, min(op.n_s, c + step))
        t_c = op.t[:, sl]
        b_c = op.scatter_points(i0[:, sl], sl) + t_c
        r_c = op.scatter_points(ix[:, sl], sl) + t_c - xs[:, sl]
        rr += float(np.sum(r_c * r_c))
        bb += float(np.sum(b_c * b_c))
        if (c // step) % 4 == 3:
            print(f"oracle residual: Sigma over {sl.stop}/{op.n_s} points "
                  f"({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    t_sig = time.perf_counter() - t0
    return float(np.sqrt(rr / bb)), t_sweep, t_sig


def box64_leg(variants, oracle_check=True, procs=12):
    """The 64^3 box (128 ordinates x 48 frequencies, N = 1.61e9) in mixed
    precision: FP32 Lambda, 16-bit (or factored FP32) Sigma, FP64
    refinement with FP64 outer residuals.  One timed solve per variant after
    an untimed one-iteration solve that sizes the workspace and tunes the
    16-bit tile (and builds a preconditioner's tables); kernel classes from
    HIP events; then single applications of the 16-bit operator for its
    kernel rates, and the oracle's FP64 residual of the fastest converged
    variant's solution."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2602_21958_amd import rt

    spec = W.box64()
    t0 = time.perf_counter()
    p = rt.Problem(spec)
    t_create = time.perf_counter() - t0
    n, n_r, n_s = p.n, p.n_r, p.n_s
    flops = 2.0 * n_r * n_r * n_s
    x = torch.empty(n, dtype=torch.float64, device="cuda:0")
    res, x_check = {}, None
    for label, prec, m, b16, form, *rest in variants:
        pc = rest[0] if rest else "none"
        p.set_sigma(form)
        t_first = time.perf_counter()
        p.solve(x, rtol=1e-8, restart=m, precision=prec, max_outer=1, max_iters=1,
                basis_fp16=b16, record_history=0, precond=pc)
        torch.cuda.synchronize()
        t_first = time.perf_counter() - t_first
        rt.profile_enable(True)
        _profile_summary(rt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = p.solve(x, rtol=1e-8, restart=m, precision=prec, max_outer=40, max_iters=2000,
                     basis_fp16=b16, record_history=0, precond=pc)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rt.profile_enable(False)
        prof = _profile_summary(rt)
        sig64 = prof["sigma"]
        res[label] = {"s_per_solve": el, "solves_per_s": 1.0 / el, "converged": st["converged"],
                      "relres_fp64": st["relres"], "precision": prec, "restart": m,
                      "basis": "fp16" if b16 else "fp32", "sigma_form": form,
                      "precond": pc, "first_call_s_incl_setup": t_first,
                      "inner_iters": st["iters"], "outer_iters": st["outer_iters"],
                      "kernel_ms": {k: v["total_ms"] for k, v in prof.items()},
                      "kernel_launches": {k: v["launches"] for k, v in prof.items()},
                      "sigma16_tile": p.gemm16_tile(prec) if prec in ("bf16", "fp16", "bf16x3")
                      else None}
        if form in ("dense", "ozaki") and sig64["launches"]:
            # FP64 outer residuals: the MFMA GEMM, or its int8 emulation
            # priced at the dense GEMM's flops
            a = sig64["total_ms"] / sig64["launches"]
            if form == "dense":
                res[label]["outer_sigma_fp64"] = {
                    "avg_ms": a, "TFLOP/s": flops / a / 1e9,
                    "frac_of_78.6TF": flops / a / 1e9 / PEAK_FP64_TFLOPS}
            else:
                res[label]["outer_sigma_fp64"] = {
                    "avg_ms": a, "kernel": "int8 emulation (15 int8 GEMMs + CRT)",
                    "TFLOP/s_dense_equivalent": flops / a / 1e9}
        print(json.dumps({"box64_variant": label, **res[label]}), file=sys.stderr, flush=True)
        # the oracle evaluates the residual of the fastest converged variant
        if st["converged"] and (x_check is None or el < res[x_check[0]]["s_per_solve"]):
            x_check = None
            x_check = (label, x.cpu().numpy())
    p.set_sigma("dense")
    conv = [(v["s_per_solve"], k) for k, v in res.items() if v["converged"]]
    best = min(conv) if conv else (float("nan"), None)
    dense = [c for c in conv if (res[c[1]]["sigma_form"] == "dense" or
                                 res[c[1]]["precision"] in ("bf16", "fp16", "bf16x3")) and
             res[c[1]]["precond"] == "none"]
    best_dense = min(dense) if dense else (float("nan"), None)
    plain = [c for c in conv if res[c[1]]["precond"] == "none"]
    best_plain = min(plain) if plain else (float("nan"), None)
    # single applications at full size: FP32 vector -> FP32 Lambda emitting
    # the k4 fp16 operand (4 B read + 2 B written per unknown) -> fp16 Sigma
    xf = torch.randn(n, dtype=torch.float32, device="cuda:0")
    yf = torch.empty_like(xf)
    kern = {}
    for prec in ("fp16", "bf16"):
        p.apply(xf, yf, precision=prec)
        torch.cuda.synchronize()
        rt.profile_enable(True)
        _profile_summary(rt)
        for _ in range(3):
            p.apply(xf, yf, precision=prec)
        torch.cuda.synchronize()
        rt.profile_enable(False)
        pr = _profile_summary(rt)
        sig_ms = pr["sigma_lo"]["total_ms"] / max(pr["sigma_lo"]["launches"], 1)
        lam_ms = pr["lambda_lo"]["total_ms"] / max(pr["lambda_lo"]["launches"], 1)
        kern[prec] = {
            "sigma16": {"kernel": f"sigma16 {prec} " + p.gemm16_tile(prec), "bound": "mfma",
                        "avg_ms": sig_ms, "achieved": flops / sig_ms / 1e9,
                        "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s",
                        "frac": flops / sig_ms / 1e9 / PEAK_BF16_TFLOPS,
                        "algorithmic_per_launch": f"2*N_r^2*N_s = {flops:.4g} flop"},
            "lambda_k4": {"kernel": "lambda_box_kernel<float -> k4 16-bit>", "bound": "hbm",
                          "avg_ms": lam_ms, "achieved": 6.0 * n / lam_ms / 1e6,
                          "peak": PEAK_HBM_GBS, "unit": "GB/s",
                          "frac": 6.0 * n / lam_ms / 1e6 / PEAK_HBM_GBS,
                          "algorithmic_per_launch": f"6 B x N = {6.0 * n:.4g} B"}}
    del xf, yf, x
    p.close()
    torch.cuda.empty_cache()
    out = {"workload": "box64: 64^3 box, 128 ordinates (8 mu x 16 az), 48 frequencies, "
                       "N = 1.61e9; FP32 Lambda + 16-bit or factored FP32 Sigma + FP64 "
                       "refinement to 1e-8",
           "n_unknowns": n, "create_s": t_create,
           "value": 1.0 / best[0], "unit": "solves/s", "best_variant": best[1],
           "best_dense_inner_variant": best_dense[1],
           "best_dense_inner_solves_per_s": 1.0 / best_dense[0],
           "best_unpreconditioned_variant": best_plain[1],
           "best_unpreconditioned_solves_per_s": 1.0 / best_plain[0],
           "variants": res, "kernels_single_apply": kern,
           "roofline": kern["fp16"]["sigma16"], "lambda": kern["fp16"]["lambda_k4"]}
    if oracle_check and x_check is not None:
        label, xh = x_check
        rel, t_sw, t_sig = oracle_residual_box(spec, xh, procs)
        del xh
        v = res[label]
        n_apply = v["inner_iters"] + v["outer_iters"]
        t_apply = 0.5 * t_sw + 0.5 * t_sig    # one sweep and one product of the two
        out["oracle_residual"] = {"variant": label, "relres_fp64_oracle": rel,
                                  "host_s": t_sw + t_sig}
        out["cpu_baseline"] = {
            "value": 1.0 / (n_apply * t_apply), "unit": "solves/s",
            "cores": max(procs, _blas_threads()), "kind": "oracle",
            "sample": f"one oracle operator application timed while evaluating the FP64 "
                      f"residual of the {label} solution (sweeps of {spec.n_mu * spec.n_az} "
                      f"ordinates over {procs} host processes: {0.5 * t_sw:.1f} s per sweep; "
                      f"Sigma chunked over points with {_blas_threads()} BLAS threads: "
                      f"{0.5 * t_sig:.1f} s per product), extrapolated to {n_apply} "
                      f"applications (the GPU solve's inner + outer iterations); an oracle "
                      f"GMRES at this size would hold 12.9 GB per basis vector"}
    return out


def bench_apply(args):
    """--workload apply: K operator applications y = A x of one problem in
    one precision (a short, fixed program for kernel traces and memory
    counters); reports the kernel classes' mean durations and rates."""
    import torch
    import workloads as W
    from paper_2602_21958_amd import rt

    spec = {"box32": W.box32, "box64": W.box64, "slab64": W.slab64}[args.problem]()
    prec = args.precision or "fp64"
    p = rt.Problem(spec)
    p.set_sigma(args.sigma_form)
    n, n_r, n_s = p.n, p.n_r, p.n_s
    dt = torch.float64 if prec == "fp64" else torch.float32
    x = torch.randn(n, dtype=dt, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(max(1, args.warmup)):
        p.apply(x, y, precision=prec)
    torch.cuda.synchronize()
    rt.profile_enable(True)
    _profile_summary(rt)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        p.apply(x, y, precision=prec)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rt.profile_enable(False)
    pr = _profile_summary(rt)
    lam_k = "lambda" if prec == "fp64" else "lambda_lo"
    sig_k = "sigma" if prec == "fp64" else "sigma_lo"
    lam_ms = pr[lam_k]["total_ms"] / max(pr[lam_k]["launches"], 1)
    sig_ms = pr[sig_k]["total_ms"] / max(pr[sig_k]["launches"], 1)
    lam_b = {"fp64": 16.0, "fp32": 8.0}.get(prec, 6.0) * n
    flops = 2.0 * n_r * n_r * n_s
    out = {"metric": "operator applications per second", "value": args.steps / el,
           "unit": "applies/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": el * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": prec, "data": "synthetic",
           "config": {"workload": f"apply: {args.problem}, {prec}, {args.sigma_form} Sigma",
                      "n_unknowns": n},
           "lambda": {"avg_ms": lam_ms, "GB/s": lam_b / lam_ms / 1e6,
                      "frac_of_8TB/s": lam_b / lam_ms / 1e6 / PEAK_HBM_GBS,
                      "algorithmic_bytes": lam_b},
           "sigma": {"avg_ms": sig_ms, "TFLOP/s_dense_equivalent": flops / sig_ms / 1e9}}
    p.close()
    print(json.dumps(out), flush=True)


def copy_calibration():
    """One 2 GiB device-to-device copy: its FETCH_SIZE / WRITE_SIZE readings
    calibrate the memory counters of the other kernels in the same run."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def bench_solve(args):
    """--workload solve: K solves to 1e-8 of one problem in one precision,
    scattering form and preconditioner (a short, fixed program for kernel
    traces); reports solves/s, iterations and the kernel classes' totals."""
    import torch
    import workloads as W
    from paper_2602_21958_amd import rt

    if args.copy_calibration:
        copy_calibration()
    spec = {"box32": W.box32, "box64": W.box64, "slab64": W.slab64}[args.problem]()
    prec = args.precision or "fp64"
    p = rt.Problem(spec)
    p.set_sigma(args.sigma_form)
    x = torch.empty(p.n, dtype=torch.float64, device="cuda:0")
    kw = dict(rtol=1e-8, restart=args.restart, precision=prec, precond=args.precond,
              max_outer=40, record_history=0, basis_fp16=1 if args.basis16 else 0)
    t0 = time.perf_counter()
    for _ in range(max(1, args.warmup)):
        p.solve(x, **kw)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t0
    rt.profile_enable(True)
    _profile_summary(rt)
    t0 = time.perf_counter()
    st = None
    for _ in range(args.steps):
        st = p.solve(x, **kw)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rt.profile_enable(False)
    pr = _profile_summary(rt)
    out = {"metric": "solves/s to 1e-8 residual", "value": args.steps / el, "unit": "solves/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": el * 1e3 / args.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": prec, "data": "synthetic",
           "config": {"workload": f"solve: {args.problem}, {prec}, {args.sigma_form} Sigma, "
                                  f"preconditioner {args.precond}, GMRES({args.restart}), "
                                  f"{'fp16' if args.basis16 else 'working-precision'} basis",
                      "n_unknowns": p.n},
           "iters": st["iters"], "outer_iters": st["outer_iters"], "relres": st["relres"],
           "converged": st["converged"], "warmup_s": t_warm,
           "kernel_classes": {k: {"launches": v["launches"],
                                  "ms_per_solve": v["total_ms"] / args.steps}
                              for k, v in pr.items()}}
    p.close()
    print(json.dumps(out), flush=True)


def bench_box64(args):
    """--workload box64: every variant; one JSON line."""
    variants = BOX64_DEFAULT + BOX64_MORE
    if args.precision:
        variants = [v for v in variants if v[1] == args.precision]
    leg = box64_leg(variants, oracle_check=not args.no_cpu_baseline, procs=args.oracle_procs)
    out = {
        "metric": "solves/s to 1e-8 residual (64^3 box, mixed precision)",
        "value": leg["value"], "unit": "solves/s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": 1e3 / leg["value"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": leg["variants"][leg["best_variant"]]["precision"],
        "data": "synthetic",
        "config": {"workload": leg["workload"], "variant": leg["best_variant"],
                   "n_unknowns": leg["n_unknowns"]},
        **{k: v for k, v in leg.items() if k not in ("value", "unit", "workload")},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
