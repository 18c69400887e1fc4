#!/usr/bin/env python3
"""Benchmark of the ACR hot path on one MI355X.

One step = factorisation (FP32 factors, eps = 1e-2, HODLR leaf 64) of the
n = 128 nonsymmetric convection-diffusion operator (N = 2,097,152) plus an FP64
right-preconditioned GMRES(30) solve to relative residual 1e-8 with the
factorisation as preconditioner.  Inputs are synthetic (seeded lognormal
kappa, random divergence-free velocity at cell Peclet 1, f ~ N(0, 1)) and are
resident in device memory before the timed region.  The plain FP64 form
(FP64 factors, same eps and GMRES) is measured once beside it.

Prints one JSON line; progress goes to stderr.
"""
import argparse
import ctypes
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "factor+solve s & solve DOF/s at n=128; FP32+IR vs FP64 at rel resid 1e-8"
# MI355X published peaks
PEAK = {"hbm": 8000.0, "fp64": 78.6, "fp32": 157.3}
HBM_CLASSES = ("solve_leaf", "solve_inner", "copy")
FP64_CLASSES = ("jacobi", "jacobi_lds", "svd_wave", "core_left", "qrcp", "qrcp_lds", "pchol", "gram", "wtilde")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_table(lib):
    from paper_1701_00182_amd import lib as _lib  # noqa: F401

    class KT(ctypes.Structure):
        _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                    ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]
    lib.acr_get_kernel_times.argtypes = [ctypes.c_void_p, ctypes.c_int32]
    lib.acr_get_kernel_times.restype = ctypes.c_int32
    n = lib.acr_get_kernel_times(None, 0)
    arr = (KT * max(n, 1))()
    lib.acr_get_kernel_times(ctypes.cast(arr, ctypes.c_void_p), n)
    return [{"name": a.name.decode(), "launches": a.launches, "ms": a.total_ms, "flops": a.flops,
             "bytes": a.bytes} for a in arr[:n]]


def roofline(table, precision):
    if not table:
        return None
    dom = max(table, key=lambda r: r["ms"])
    avg_s = dom["ms"] / 1e3 / max(dom["launches"], 1)
    name = dom["name"]
    if name in HBM_CLASSES:
        bound, unit = "hbm", "GB/s"
        achieved = dom["bytes"] / max(dom["launches"], 1) / avg_s / 1e9
        peak = PEAK["hbm"]
    else:
        bound, unit = "alu", "TFLOP/s"
        achieved = dom["flops"] / max(dom["launches"], 1) / avg_s / 1e12
        fp64 = name in FP64_CLASSES or precision == "fp64"
        peak = PEAK["fp64"] if fp64 else PEAK["fp32"]
    return {"bound": bound, "kernel": name, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": None,
            "avg_launch_ms": avg_s * 1e3, "launches_per_step": None,
            "algorithmic_per_launch": (dom["bytes"] if bound == "hbm" else dom["flops"]) / max(dom["launches"], 1),
            "share_of_kernel_time": dom["ms"] / sum(r["ms"] for r in table)}


def run_form(acr, coef_d, b, args, precision, timed_steps, warmup):
    import torch
    N = b.numel()
    rec = []
    for step in range(warmup + timed_steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac = acr.Factor(coef_d, eps=args.eps, leaf=args.leaf, precision=precision)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, info = fac.solve_refined(b, tol=args.tol, method="gmres", restart=30, maxit=300)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if step >= warmup:
            rec.append((t1 - t0, t2 - t1, info))
        st = fac.stats()
        # one preconditioner application, replayed from its graph
        fac.solve(b)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(5):
            fac.solve(b)
        torch.cuda.synchronize()
        t_apply = (time.perf_counter() - ta) / 5
        fac.free()
        log(f"{precision} step {step}: factor {t1 - t0:.3f}s solve {t2 - t1:.3f}s its {info['iterations']} "
            f"relres {info['relres']:.2e} apply {t_apply * 1e3:.2f}ms")
    if not rec:
        return None, None
    tf = sum(r[0] for r in rec) / len(rec)
    ts = sum(r[1] for r in rec) / len(rec)
    info = rec[-1][2]
    return {"t_factor_s": tf, "t_solve_s": ts, "factor_plus_solve_s": tf + ts,
            "solve_dof_per_s": N / ts, "apply_ms": t_apply * 1e3, "apply_dof_per_s": N / t_apply,
            "iterations": info["iterations"], "relres": info["relres"],
            "relres_before_refinement": info["relres0"], "max_rank": st["max_rank"],
            "avg_rank": st["avg_rank"], "factor_GB": st["factor_bytes"] / 1e9,
            "solve_bytes_GB": st["solve_bytes"] / 1e9}, x


def cpu_baseline(n, eps, leaf):
    """The oracle (plain dense-block ACR with truncated-SVD HODLR blocks, FP64) on a
    bounded sample: the same operator family at a small n, factor + one solve."""
    from oracle.acr import OracleACR
    from workloads import problem, rhs_normal
    threads = os.cpu_count()
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 0) for i in info] + [1])
    except Exception:
        pass
    coef = problem("convdiff", n)
    f = rhs_normal(n ** 3)
    t0 = time.perf_counter()
    o = OracleACR(coef, leaf, eps)
    o.solve(f)
    dt = time.perf_counter() - t0
    return {"value": n ** 3 / dt, "unit": "DOF/s", "cores": threads, "kind": "oracle",
            "sample": f"oracle factor + one solve of the convection-diffusion operator at n={n} "
                      f"(N={n ** 3}), eps={eps}, leaf {leaf}, FP64 dense plane blocks; {dt:.2f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--eps", type=float, default=1e-2)
    ap.add_argument("--leaf", type=int, default=64)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-fp64-form", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=24)
    args = ap.parse_args()
    ws = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or ws != 1:
        print("bench.py measures one GPU only: the cyclic-reduction hot path is built and timed on a "
              "single MI355X (multi-GPU plane distribution is design-only); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1701_00182_amd as acr
    from workloads import problem, rhs_normal

    n = args.n
    N = n ** 3
    log(f"building inputs n={n}")
    coef = problem("convdiff", n)
    f = rhs_normal(N)
    dev = torch.device("cuda:0")
    coef_d = torch.from_numpy(coef).to(dev)
    b = torch.from_numpy(f).to(dev)
    torch.cuda.synchronize()

    L = acr.lib()
    L.acr_set_kernel_timing.argtypes = [ctypes.c_int32]
    L.acr_set_kernel_timing.restype = None
    # warmup without instrumentation, timed steps with per-kernel event timing
    log("warmup")
    run_form(acr, coef_d, b, args, args.precision, 0, args.warmup)
    L.acr_set_kernel_timing(1)
    log("timed steps")
    main_form, x_main = run_form(acr, coef_d, b, args, args.precision, args.steps, 0)
    L.acr_set_kernel_timing(0)
    table = kernel_table(L)
    rl = roofline(table, args.precision)
    if rl is not None:
        per_step = next(r for r in table if r["name"] == rl["kernel"])["launches"] / args.steps
        rl["launches_per_step"] = per_step

    out = {
        "metric": METRIC,
        "value": N / main_form["factor_plus_solve_s"],
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_form["factor_plus_solve_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": f"convection-diffusion n={n} (N={N}), lognormal kappa, divergence-free "
                               f"velocity at cell Peclet 1, eps={args.eps}, HODLR leaf {args.leaf}, "
                               f"{args.precision.upper()} factors + FP64 GMRES(30) to {args.tol:g}",
                   "n": n, "N": N, "eps": args.eps, "leaf": args.leaf, "precision": args.precision,
                   "refinement": "fp64 gmres(30)", "tol": args.tol},
        "value_definition": "N / (t_factor + t_solve) for one step (whole job, inputs resident)",
        "form": main_form,
        "kernel_table": sorted(table, key=lambda r: -r["ms"])[:8],
        "roofline": rl,
    }
    if not args.no_fp64_form and args.precision != "fp64":
        log("fp64 form")
        f64, x64 = run_form(acr, coef_d, b, args, "fp64", 1, 0)
        f64["error_vs_fp64_form"] = 0.0
        out["fp64_form"] = f64
        out["form"]["error_vs_fp64_form"] = float(torch.linalg.norm(x_main - x64) / torch.linalg.norm(x64))
    if not args.no_cpu_baseline:
        log(f"cpu baseline (oracle) n={args.cpu_n}")
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, args.eps, args.leaf)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
