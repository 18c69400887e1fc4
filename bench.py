#!/usr/bin/env python3
"""Benchmark of the ACR hot path on one MI355X.

Default workload (the headline line): one step = factorisation (FP32 factors,
eps = 1e-2, HODLR leaf 128 and the two-kernel core SVD -- the autotuner's choice
for this operator; --autotune runs it on an 8-plane sample before the timed
region instead) of the n = 128 nonsymmetric convection-diffusion
operator (N = 2,097,152) plus an FP64 right-preconditioned GMRES(30) solve to
relative residual 1e-8 with the factorisation as preconditioner.  Inputs are
synthetic (seeded lognormal kappa, random divergence-free velocity at cell
Peclet 1, f ~ N(0, 1)) and resident in device memory before the timed region.
The plain FP64 form and the BF16 variant (every block product of the
factorisation on BF16 matrix-core inputs with per-block scaling; same eps and
GMRES) are measured once beside it (the FP64 form with its own kernel table and roofline), the
factorisation is measured as a CG preconditioner of the paper's Table precond
problem over its eps sweep, and the oracle is timed on the host on a bounded
sample.

Other workloads (--workload, one JSON line each, not the headline):
  helmholtz_mrhs  indefinite Helmholtz n = 64, FP32 factors, eps = 1e-3, 256
                  right-hand sides in one graph-replayed solve
  poisson_ir      Poisson n = 64, eps = 1e-4: plain FP64 factor + solve against
                  FP32 factors + FP64 iterative refinement to 1e-8
  gradient        Poisson n = 64: loss and gradient with respect to all N nodal
                  kappa values (forward refined solve, adjoint transpose solve,
                  per-cell gradient kernel)
  paper_precond   the paper's Table precond problem (-lap u = 1 at n = 128,
                  CG to 1e-6) over an eps sweep, beside the paper's numbers
  helmholtz27     the paper's 27-point finite-element Helmholtz problem
                  (k = n/2) at n = 32 and 64, GMRES to 1e-10, beside its
                  Table ACRHelConfiguration
  copy_calibration  a plain 1 GiB device copy (reference dispatch for scaling
                  the rocprofv3 FETCH_SIZE / WRITE_SIZE counters)

Prints one JSON line; progress goes to stderr.
"""
import argparse
import ctypes
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "factor+solve s & solve DOF/s at n=128; FP32+IR vs FP64 at rel resid 1e-8"
# MI355X published peaks (GB/s, dense TFLOP/s)
PEAK = {"hbm": 8000.0, "fp64": 78.6, "fp32": 157.3, "bf16": 2500.0, "fp16": 2500.0}
HBM_CLASSES = ("solve_leaf", "solve_inner", "copy")
FP64_CLASSES = ("jacobi", "jacobi_lds", "svd_wave", "svd_block", "core_left", "qrcp", "qrcp_lds", "pchol", "gram",
                "wtilde")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pmc_traffic.json")
STATS_FILE = os.path.join(ROOT, "profiles", "kernel_stats.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_table(lib):
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


def set_timing(lib, level):
    lib.acr_set_kernel_timing.argtypes = [ctypes.c_int32]
    lib.acr_set_kernel_timing.restype = None
    lib.acr_set_kernel_timing(level)


def class_bound(name, precision):
    """(bound, peak, unit) of a kernel class."""
    if name in HBM_CLASSES:
        return "hbm", PEAK["hbm"], "GB/s"
    if name in ("gemm", "seg_gemm"):
        return "mfma", PEAK["fp64"] if precision == "fp64" else PEAK["fp32"], "TFLOP/s"
    if name == "gemm_bf16":
        return "mfma", PEAK["bf16"], "TFLOP/s"
    if name == "gemm_f16":
        return "mfma", PEAK["fp16"], "TFLOP/s"
    fp64 = name in FP64_CLASSES or precision == "fp64"
    return "alu", PEAK["fp64"] if fp64 else PEAK["fp32"], "TFLOP/s"


def _current_record(path, section, cls):
    """A class record of a committed rocprofv3 summary, if it was taken on the
    current source of the kernel (SHA-256 of its files), else None."""
    try:
        with open(path) as fh:
            rec = json.load(fh)[section][cls]
        h = hashlib.sha256()
        for src in rec["sources"]:
            with open(os.path.join(ROOT, src), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != rec["sha256"]:
            return None
        return rec
    except (OSError, KeyError, ValueError):
        return None


def measured_traffic(cls, precision="fp32"):
    """HBM bytes per launch of a kernel class from the committed rocprofv3 PMC
    summary, if that summary was taken on the current source of the kernel."""
    if precision != "fp32":
        return None
    rec = _current_record(TRAFFIC_FILE, "classes", cls)
    return rec["bytes_per_launch"] if rec else None


def profiled_launch_ms(cls, precision):
    """Average duration of one launch of a kernel class in the committed
    rocprofv3 kernel statistics (kernel_stats.json), for the current source."""
    rec = _current_record(STATS_FILE, precision, cls)
    return rec["avg_ms"] if rec else None


def roofline(table, precision, steps):
    if not table:
        return None
    dom = max(table, key=lambda r: r["ms"])
    nl = max(dom["launches"], 1)
    avg_s = dom["ms"] / 1e3 / nl
    bound, peak, unit = class_bound(dom["name"], precision)
    per_launch = (dom["bytes"] if bound == "hbm" else dom["flops"]) / nl
    scale = 1e9 if bound == "hbm" else 1e12
    achieved = per_launch / avg_s / scale
    out = {"bound": bound, "kernel": dom["name"], "achieved": achieved, "peak": peak, "unit": unit,
           "frac": achieved / peak, "traffic": measured_traffic(dom["name"], precision),
           "avg_launch_ms": avg_s * 1e3, "launches_per_step": dom["launches"] / max(steps, 1),
           "algorithmic_per_launch": per_launch,
           "algorithmic_bytes_per_launch": dom["bytes"] / nl,
           "share_of_kernel_time": dom["ms"] / sum(r["ms"] for r in table)}
    # the same figure from the committed rocprofv3 average of this class
    pms = profiled_launch_ms(dom["name"], precision)
    if pms:
        out["rocprof"] = {"avg_launch_ms": pms, "achieved": per_launch / (pms / 1e3) / scale,
                          "frac": per_launch / (pms / 1e3) / scale / peak, "source": os.path.relpath(STATS_FILE, ROOT)}
    return out


def brief_table(table, precision, k=12):
    """Per kernel class: time, the bound it is measured against and its rate,
    plus algorithmic bytes per launch and, where the committed PMC summary is
    current, the counted HBM bytes per launch and their ratio."""
    out = []
    for r in sorted(table, key=lambda r: -r["ms"])[:k]:
        bound, peak, unit = class_bound(r["name"], precision)
        sec = max(r["ms"] / 1e3, 1e-12)
        rate = (r["bytes"] / 1e9 if bound == "hbm" else r["flops"] / 1e12) / sec
        nl = max(r["launches"], 1)
        row = {"class": r["name"], "launches": r["launches"], "ms": round(r["ms"], 3), "bound": bound,
               "achieved": rate, "unit": unit, "frac": rate / peak,
               "alg_bytes_per_launch": r["bytes"] / nl, "alg_GBps": r["bytes"] / 1e9 / sec,
               "flops_per_launch": r["flops"] / nl}
        tr = measured_traffic(r["name"], precision)
        if tr is not None and r["bytes"] > 0:
            row["hbm_bytes_per_launch"] = tr
            row["hbm_over_alg"] = tr / (r["bytes"] / nl)
        out.append(row)
    return out


def host_cpu():
    """Model name and logical CPU count of the host (from /proc/cpuinfo)."""
    model, count = "unknown", 0
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    count += 1
                    model = line.split(":", 1)[1].strip()
    except OSError:
        pass
    return model, count


# ----------------------------------------------------------------- headline
def run_form(acr, coef_d, b, args, precision, timed_steps, warmup):
    import torch
    N = b.numel()
    rec = []
    st = None
    t_apply = float("nan")
    x = None
    for step in range(warmup + timed_steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac = acr.Factor(coef_d, eps=args.eps, leaf=args.leaf, precision=precision,
                         svd_fused_lds=args.svd_fused_lds, gemm_tiles=args.gemm_tiles)
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
            "iterations": info["iterations"], "converged": info["converged"], "relres": info["relres"],
            "relres_before_refinement": info["relres0"], "max_rank": st["max_rank"],
            "avg_rank": st["avg_rank"], "factor_GB": st["factor_bytes"] / 1e9,
            "solve_bytes_GB": st["solve_bytes"] / 1e9, "flops_svd": st["flops_svd"],
            "flops_gemm": st["flops_gemm"]}, x


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
    model, logical = host_cpu()
    return {"value": n ** 3 / dt, "unit": "DOF/s", "cores": threads, "kind": "oracle",
            "cpu_model": model, "host_logical_cpus": logical, "affinity_cpus": len(os.sched_getaffinity(0)),
            "sample": f"oracle factor + one solve of the convection-diffusion operator at n={n} "
                      f"(N={n ** 3}), eps={eps}, leaf {leaf}, FP64 dense plane blocks; {dt:.2f} s"}


def headline(args, torch, acr):
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
    tune = None
    if args.autotune:
        # leaf size and core-SVD dispatch from a sample of the operator (untimed)
        t0 = time.perf_counter()
        tune = acr.autotune(coef_d, eps=args.eps, precision=args.precision, leaf=args.leaf,
                            sample_planes=args.tune_planes)
        tune["tuning_s"] = time.perf_counter() - t0
        args.leaf, args.svd_fused_lds, args.gemm_tiles = tune["leaf"], tune["svd_fused_lds"], tune["gemm_tiles"]
        log(f"autotune: leaf {args.leaf}, svd_fused_lds {args.svd_fused_lds}, gemm_tiles {args.gemm_tiles} "
            f"({tune['tuning_s']:.1f} s)")
    log("warmup")
    run_form(acr, coef_d, b, args, args.precision, 0, args.warmup)
    log("timed steps")
    main_form, x_main = run_form(acr, coef_d, b, args, args.precision, args.steps, 0)
    # one more step, outside the timed ones, with HIP events around every
    # factorisation launch on its stream: the per-class kernel table and roofline
    log("instrumented step (kernel table)")
    set_timing(L, 1)
    run_form(acr, coef_d, b, args, args.precision, 1, 0)
    set_timing(L, 0)
    table = kernel_table(L)
    rl = roofline(table, args.precision, 1)
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
        "dtype": "f64" if args.precision == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"convection-diffusion n={n} (N={N}), lognormal kappa, divergence-free "
                               f"velocity at cell Peclet 1, eps={args.eps}, HODLR leaf {args.leaf}, "
                               f"{args.precision.upper()} factors + FP64 GMRES(30) to {args.tol:g}",
                   "n": n, "N": N, "eps": args.eps, "leaf": args.leaf, "svd_fused_lds": args.svd_fused_lds,
                   "gemm_tiles": args.gemm_tiles,
                   "autotune": tune, "precision": args.precision, "refinement": "fp64 gmres(30)",
                   "tol": args.tol},
        "value_definition": "N / (t_factor + t_solve) for one step (whole job, inputs resident)",
        "form": main_form,
        "kernel_table": brief_table(table, args.precision),
        "roofline": rl,
    }
    if not args.no_fp64_form and args.precision != "fp64":
        log("fp64 form")
        f64, x64 = run_form(acr, coef_d, b, args, "fp64", 1, 0)
        set_timing(L, 1)
        run_form(acr, coef_d, b, args, "fp64", 1, 0)
        set_timing(L, 0)
        t64 = kernel_table(L)
        f64["kernel_table"] = brief_table(t64, "fp64")
        f64["roofline"] = roofline(t64, "fp64", 1)
        f64["error_vs_fp64_form"] = 0.0
        out["fp64_form"] = f64
        out["form"]["error_vs_fp64_form"] = float(torch.linalg.norm(x_main - x64) / torch.linalg.norm(x64))
        if not args.no_lowp_form:
            log("bf16 form")
            fb, xb = run_form(acr, coef_d, b, args, "fp32_bf16", 1, 0)
            set_timing(L, 1)
            run_form(acr, coef_d, b, args, "fp32_bf16", 1, 0)
            set_timing(L, 0)
            tb = kernel_table(L)
            fb["kernel_table"] = brief_table(tb, "fp32", k=6)
            fb["error_vs_fp64_form"] = float(torch.linalg.norm(xb - x64) / torch.linalg.norm(x64))
            out["bf16_form"] = fb
    if not args.no_precond_sweep:
        log("preconditioner eps sweep (Table precond problem)")
        out["precond_sweep"] = precond_sweep(acr, torch, n, args.leaf, args.precision, args.eps_list, warm=False)
    if not args.no_cpu_baseline:
        log(f"cpu baseline (oracle) n={args.cpu_n}")
        out["cpu_baseline"] = cpu_baseline(args.cpu_n, args.eps, args.leaf)
    return out


# ------------------------------------------------------- other workloads
def helmholtz_mrhs(args, torch, acr):
    from workloads import problem, rhs_normal
    n, nrhs, eps, leaf = 64, args.nrhs, 1e-3, 64
    N = n ** 3
    coef_d = torch.from_numpy(problem("helmholtz", n)).cuda()
    B = torch.from_numpy(rhs_normal(N, nrhs=nrhs).T.copy()).cuda()   # (nrhs, N): one row per right-hand side
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fac = acr.Factor(coef_d, eps=eps, leaf=leaf, precision="fp32")
    torch.cuda.synchronize()
    t_factor = time.perf_counter() - t0
    X = fac.solve(B)                       # records the plan and its graph
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        fac.solve(B, out=X)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fac.solve(B, out=X)
    torch.cuda.synchronize()
    t_solve = (time.perf_counter() - t0) / args.steps
    L = acr.lib()
    set_timing(L, 2)                        # one instrumented replay for the kernel table
    fac.solve(B, out=X)
    torch.cuda.synchronize()
    set_timing(L, 0)
    table = kernel_table(L)
    rel = []
    for j in range(nrhs):
        r = fac.residual(X[j].contiguous(), B[j].contiguous())
        rel.append(float(r.norm() / B[j].norm()))
    rel.sort()
    x0, info = fac.solve_refined(B[0].contiguous(), tol=1e-8, method="gmres", maxit=300, raise_on_fail=False)
    st = fac.stats()
    fac.free()
    log(f"helmholtz n={n}: factor {t_factor:.3f}s, {nrhs}-RHS solve {t_solve * 1e3:.2f} ms, "
        f"GMRES rhs0 {info['iterations']} its relres {info['relres']:.2e}")
    # factors GMRES can use: eps = 1e-6 with the operation-internal truncations
    # at eps / 100 (at eps = 1e-3 the indefinite Schur complements amplify the
    # truncation errors beyond what GMRES(30) recovers from; at eps = 1e-5 the
    # iteration count moves between 25 and more than 120 with rounding-level
    # differences in the factors)
    ue, ur = 1e-6, 0.01
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fu = acr.Factor(coef_d, eps=ue, leaf=leaf, precision="fp32", inner_eps_ratio=ur)
    torch.cuda.synchronize()
    tu = time.perf_counter() - t0
    Xu = fu.solve(B)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fu.solve(B, out=Xu)
    torch.cuda.synchronize()
    tus = time.perf_counter() - t0
    relu = sorted(float(fu.residual(Xu[j].contiguous(), B[j].contiguous()).norm() / B[j].norm())
                  for j in range(nrhs))
    per_rhs = []
    for j in range(args.refine_rhs):
        _, inf = fu.solve_refined(B[j].contiguous(), tol=1e-8, method="gmres", maxit=300, raise_on_fail=False)
        per_rhs.append({"rhs": j, "iterations": inf["iterations"], "converged": inf["converged"],
                        "relres": inf["relres"]})
    stu = fu.stats()
    fu.free()
    log(f"helmholtz n={n} eps={ue:g} inner ratio {ur:g}: factor {tu:.3f}s, {nrhs}-RHS solve {tus * 1e3:.2f} ms, "
        f"GMRES its {[r['iterations'] for r in per_rhs]}")
    usable = {"eps": ue, "inner_eps_ratio": ur, "t_factor_s": tu, "solve_ms": tus * 1e3,
              "solve_dof_per_s": N * nrhs / tus, "max_rank": stu["max_rank"], "factor_GB": stu["factor_bytes"] / 1e9,
              "relres_unrefined": {"min": relu[0], "median": relu[len(relu) // 2], "max": relu[-1]},
              "gmres_per_rhs": per_rhs}
    return {
        "metric": f"multi-RHS solve DOF/s (Helmholtz n={n}, {nrhs} RHS, FP32 factors)",
        "value": N * nrhs / t_solve, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_solve * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"indefinite Helmholtz n={n} (N={N}), c = 1 + 0.3 smoothed noise, 10 points per "
                               f"wavelength, eps={eps}, leaf {leaf}, FP32 factors, {nrhs} RHS per graph replay",
                   "n": n, "nrhs": nrhs, "eps": eps, "leaf": leaf},
        "t_factor_s": t_factor, "max_rank": st["max_rank"], "factor_GB": st["factor_bytes"] / 1e9,
        "relres_unrefined": {"min": rel[0], "median": rel[len(rel) // 2], "max": rel[-1]},
        "gmres_rhs0": {"iterations": info["iterations"], "converged": info["converged"], "relres": info["relres"]},
        "refinable_factors": usable,
        "kernel_table": brief_table(table, "fp32"),
        "roofline": roofline(table, "fp32", 1),
    }


def poisson_ir(args, torch, acr):
    from workloads import problem, rhs_normal
    n, eps, leaf = 64, 1e-4, 64
    N = n ** 3
    coef_d = torch.from_numpy(problem("poisson", n)).cuda()
    b = torch.from_numpy(rhs_normal(N)).cuda()
    res = {}
    for prec in ("fp64", "fp32"):
        for step in range(args.warmup + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fac = acr.Factor(coef_d, eps=eps, leaf=leaf, precision=prec)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            if prec == "fp64":
                x = fac.solve(b)
                torch.cuda.synchronize()
                r = fac.residual(x, b)
                info = {"iterations": 0, "relres": float(r.norm() / b.norm())}
            else:
                x, info = fac.solve_refined(b, tol=1e-8, method="ir", maxit=100)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            fac.free()
        res[prec] = {"t_factor_s": t1 - t0, "t_solve_s": t2 - t1, "factor_plus_solve_s": t2 - t0,
                     "iterations": info["iterations"], "relres": info["relres"], "x": x}
        log(f"poisson n={n} {prec}: factor {t1 - t0:.3f}s solve {t2 - t1:.3f}s relres {info['relres']:.2e}")
    err = float(torch.linalg.norm(res["fp32"]["x"] - res["fp64"]["x"]) / torch.linalg.norm(res["fp64"]["x"]))
    for v in res.values():
        v.pop("x")
    return {
        "metric": f"factor+solve DOF/s (Poisson n={n}, FP32 factors + FP64 IR to 1e-8)",
        "value": N / res["fp32"]["factor_plus_solve_s"], "unit": "DOF/s", "n_gpus": 1, "steps": 1,
        "warmup": args.warmup, "ms_per_step": res["fp32"]["factor_plus_solve_s"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"variable-coefficient Poisson n={n} (N={N}), lognormal kappa, eps={eps}, "
                               f"leaf {leaf}", "n": n, "eps": eps, "leaf": leaf},
        "fp32_ir": res["fp32"], "fp64_plain": res["fp64"], "fp32_ir_vs_fp64_plain_rel_diff": err,
    }


def gradient(args, torch, acr):
    from workloads import lognormal_kappa, rhs_normal, observation_cells, observation_noise
    n = 64
    N = n ** 3
    kappa = torch.from_numpy(lognormal_kappa(n)).cuda()
    f = torch.from_numpy(rhs_normal(N)).cuda()
    obs = torch.from_numpy(observation_cells(N, count=512)).cuda()
    data = torch.from_numpy(observation_noise(512)).cuda()   # a data vector of the right shape
    times = []
    gnorm = float("nan")
    for step in range(args.warmup + args.steps):
        k = kappa.clone().requires_grad_(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u = acr.ACRSolve.apply(k, f, 1e-4, 64, "fp32", 1e-12)
        r = u[obs] - data
        loss = 0.5 * (r * r).sum()
        loss.backward()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if step >= args.warmup:
            times.append(dt)
        gnorm = float(k.grad.norm())
        log(f"gradient step {step}: {dt:.3f}s loss {float(loss.detach()):.4e}")
    t = sum(times) / len(times)
    return {
        "metric": f"loss+gradient DOF/s (Poisson n={n}, all nodal kappa)",
        "value": N / t, "unit": "DOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"Poisson n={n} (N={N}), lognormal kappa, 512 observation cells, eps=1e-4, "
                               f"FP32 factors, forward and adjoint solves refined to 1e-12", "n": n},
        "grad_norm": gnorm,
    }


# the paper's Table precond (Poisson -lap u = 1 on 128^3, CG to 1e-6, CPU
# cluster): H_eps -> (factorisation s, one application s, CG iterations, total s)
PAPER_PRECOND = {6e-1: (18.55, 0.050, 43, 20.72), 3e-1: (21.33, 0.053, 34, 23.14), 1e-1: (26.56, 0.058, 25, 28.01),
                 1e-2: (51.24, 0.064, 11, 51.94), 1e-3: (89.32, 0.104, 4, 89.73), 1e-4: (149.06, 0.127, 3, 149.44)}


def precond_sweep(acr, torch, n, leaf, precision, eps_list, warm=True):
    """Rows of the preconditioner sweep: constant-coefficient Poisson with f = 1,
    CG to 1e-6 preconditioned by the factorisation at each eps."""
    from workloads import problem
    N = n ** 3
    coef_d = torch.from_numpy(problem("laplace", n)).cuda()
    b = torch.ones(N, dtype=torch.float64, device="cuda")
    rows = []
    for eps in eps_list:
        if warm:
            fac = acr.Factor(coef_d, eps=eps, leaf=leaf, precision=precision)   # warm-up
            fac.free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac = acr.Factor(coef_d, eps=eps, leaf=leaf, precision=precision)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, info = fac.solve_refined(b, tol=1e-6, method="cg", maxit=500, raise_on_fail=False)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        fac.solve(b)
        torch.cuda.synchronize()
        ta = time.perf_counter()
        for _ in range(5):
            fac.solve(b)
        torch.cuda.synchronize()
        t_apply = (time.perf_counter() - ta) / 5
        st = fac.stats()
        fac.free()
        paper = PAPER_PRECOND.get(eps)
        row = {"eps": eps, "t_factor_s": t1 - t0, "t_cg_s": t2 - t1, "total_s": t2 - t0, "apply_s": t_apply,
               "cg_iterations": info["iterations"], "converged": info["converged"], "relres": info["relres"],
               "relres_before_refinement": info["relres0"], "max_rank": st["max_rank"],
               "factor_GB": st["factor_bytes"] / 1e9}
        if paper:
            row["paper"] = {"t_factor_s": paper[0], "apply_s": paper[1], "cg_iterations": paper[2],
                            "total_s": paper[3]}
        rows.append(row)
        log(f"laplace n={n} eps={eps:g}: factor {t1 - t0:.3f}s CG {t2 - t1:.3f}s ({info['iterations']} its, "
            f"relres {info['relres']:.1e}) apply {t_apply * 1e3:.2f}ms max rank {st['max_rank']}")
    return rows


def paper_precond(args, torch, acr):
    """ACR as a CG preconditioner on the paper's own problem: constant-coefficient
    Poisson with f = 1 at n = 128, eps swept as in its Table precond."""
    n, leaf = 128, args.leaf
    N = n ** 3
    rows = precond_sweep(acr, torch, n, leaf, args.precision, args.eps_list)
    best = min((r for r in rows if r["converged"]), key=lambda r: r["total_s"])
    paper_best = min(v[3] for v in PAPER_PRECOND.values())
    return {
        "metric": "factor + CG-solve DOF/s (Poisson -lap u = 1, n=128, CG to 1e-6, best eps of the sweep)",
        "value": N / best["total_s"], "unit": "DOF/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": best["total_s"] * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": (N / best["total_s"]) / (N / paper_best),
        "vs_baseline_definition": "ratio to the paper's best total time in its Table precond (20.72 s at H_eps 0.6, "
                                  "CPU cluster, standard admissibility, core count not stated)",
        "dtype": "f32" if args.precision != "fp64" else "f64", "data": "synthetic",
        "config": {"workload": f"constant-coefficient Poisson n={n} (N={N}), f = 1, Dirichlet, HODLR leaf {leaf}, "
                               f"{args.precision.upper()} factors, FP64 flexible CG to 1e-6",
                   "n": n, "leaf": leaf, "eps_list": args.eps_list},
        "best_eps": best["eps"], "sweep": rows,
    }


# the paper's Table ACRHelConfiguration: n -> (H_eps, eta, leaf, relres, average rank, largest rank)
PAPER_HELM27 = {32: (5e-3, 4, 32, 1.67e-2, 5, 8), 64: (5e-8, 8, 32, 2.63e-2, 30, 56),
                128: (5e-13, 16, 32, 1.07e-2, 113, 260)}


def helmholtz27(args, torch, acr):
    """The paper's indefinite Helmholtz problem (Section 5.3): -(lap u + k^2 u) = 1
    on the unit cube, Dirichlet, trilinear finite elements (27-point stencil),
    k = n / 2 (about 12 points per wavelength); FP32 factors with the
    operation-internal truncations at eps / 100, FP64 GMRES(30) to 1e-10."""
    from workloads import problem
    rows = []
    for n, eps in zip(args.h27_n, args.h27_eps):
        N = n ** 3
        coef_d = torch.from_numpy(problem("fem_helmholtz27", n)).cuda()
        b = torch.ones(N, dtype=torch.float64, device="cuda")
        fac = acr.Factor(coef_d, eps=eps, leaf=args.h27_leaf, precision="fp32", inner_eps_ratio=0.01)  # warm-up
        fac.free()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fac = acr.Factor(coef_d, eps=eps, leaf=args.h27_leaf, precision="fp32", inner_eps_ratio=0.01)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, info = fac.solve_refined(b, tol=1e-10, method="gmres", maxit=300, raise_on_fail=False)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        st = fac.stats()
        fac.free()
        row = {"n": n, "N": N, "wavenumber": n / 2, "eps": eps, "leaf": args.h27_leaf, "t_factor_s": t1 - t0,
               "t_gmres_s": t2 - t1, "gmres_applications": info["iterations"], "converged": info["converged"],
               "relres": info["relres"], "relres_before_refinement": info["relres0"],
               "avg_rank": st["avg_rank"], "max_rank": st["max_rank"], "factor_GB": st["factor_bytes"] / 1e9}
        if n in PAPER_HELM27:
            pe = PAPER_HELM27[n]
            row["paper"] = {"H_eps": pe[0], "eta": pe[1], "leaf": pe[2], "relres": pe[3], "avg_rank": pe[4],
                            "max_rank": pe[5]}
        rows.append(row)
        log(f"helmholtz27 n={n} eps={eps:g}: factor {t1 - t0:.3f}s, unrefined relres {info['relres0']:.2e}, "
            f"GMRES {info['iterations']} its to {info['relres']:.1e} in {t2 - t1:.3f}s, ranks {st['avg_rank']:.1f}/"
            f"{st['max_rank']}")
    last = rows[-1]
    return {
        "metric": f"factor + GMRES-solve DOF/s (27-point FEM Helmholtz, n={last['n']}, k=n/2, GMRES to 1e-10)",
        "value": last["N"] / (last["t_factor_s"] + last["t_gmres_s"]), "unit": "DOF/s", "n_gpus": 1, "steps": 1,
        "warmup": 1, "ms_per_step": (last["t_factor_s"] + last["t_gmres_s"]) * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "indefinite Helmholtz -(lap u + k^2 u) = 1, trilinear finite elements (27-point), "
                               "k = n/2, HODLR FP32 factors (inner truncations at eps/100), FP64 GMRES(30)",
                   "n": args.h27_n, "eps": args.h27_eps, "leaf": args.h27_leaf},
        "rows": rows,
    }


def copy_calibration(torch):
    """A plain device copy of exactly 1 GiB, the reference dispatch for scaling
    rocprofv3's FETCH_SIZE / WRITE_SIZE counters to bytes."""
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    return {"copy_bytes": src.numel() * 4, "dispatches": 3}


# kernel name prefix -> (traffic class, source files whose SHA-256 gates the figures)
PMC_CLASSES = [
    ("k_jacobi<float, true", "jacobi_lds", ["paper_1701_00182_amd/csrc/svd.hip", "paper_1701_00182_amd/csrc/wave.h"]),
    ("k_jacobi<float, false", "jacobi", ["paper_1701_00182_amd/csrc/svd.hip", "paper_1701_00182_amd/csrc/wave.h"]),
    ("k_qrcp<float, true", "qrcp_lds", ["paper_1701_00182_amd/csrc/svd.hip", "paper_1701_00182_amd/csrc/wave.h"]),
    ("k_qrcp<float, false", "qrcp", ["paper_1701_00182_amd/csrc/svd.hip", "paper_1701_00182_amd/csrc/wave.h"]),
    ("k_svd_wave<float>", "svd_wave", ["paper_1701_00182_amd/csrc/svd.hip", "paper_1701_00182_amd/csrc/wave.h"]),
    ("k_svd_block<float", "svd_block", ["paper_1701_00182_amd/csrc/svd.hip", "paper_1701_00182_amd/csrc/wave.h"]),
    ("k_core_left<float>", "core_left", ["paper_1701_00182_amd/csrc/svd.hip"]),
    ("k_gemm_f32", "gemm", ["paper_1701_00182_amd/csrc/gemm_mfma.hip"]),
    ("k_qr_lds<float", "qr_lds", ["paper_1701_00182_amd/csrc/la_lds.hip", "paper_1701_00182_amd/csrc/wave.h"]),
    ("k_applyq_lds<float", "applyq_lds", ["paper_1701_00182_amd/csrc/la_lds.hip", "paper_1701_00182_amd/csrc/wave.h"]),
    ("k_pchol", "pchol", ["paper_1701_00182_amd/csrc/gram.hip", "paper_1701_00182_amd/csrc/wave.h"]),
    ("k_gram", "gram", ["paper_1701_00182_amd/csrc/gemm_mfma.hip", "paper_1701_00182_amd/csrc/gram.hip"]),
    ("k_wtilde<float>", "wtilde", ["paper_1701_00182_amd/csrc/gram.hip"]),
    ("k_inverse<float", "inverse", ["paper_1701_00182_amd/csrc/la_kernels.hip"]),
    ("k_inverse_blk<float", "inverse", ["paper_1701_00182_amd/csrc/la_kernels.hip"]),
    ("k_copy<float>", "copy", ["paper_1701_00182_amd/csrc/la_kernels.hip"]),
    ("k_apply_leaf_vec<float>", "solve_leaf", ["paper_1701_00182_amd/csrc/solve_kernels.hip"]),
    ("k_inner_vec<float>", "solve_inner", ["paper_1701_00182_amd/csrc/solve_kernels.hip"]),
]
# kernel classes whose one launch (one timing record) is several dispatches:
# the Gram partials and their ordered reduction
DISPATCHES_PER_LAUNCH = {"gram": 2}
# classes grouped for the kernel statistics only (no PMC figures taken)
STATS_ONLY_CLASSES = [
    ("k_seg_gemm<float>", "seg_gemm", ["paper_1701_00182_amd/csrc/gemm_mfma.hip"]),
    ("k_gemm_f64", "gemm", ["paper_1701_00182_amd/csrc/gemm_mfma.hip"]),
    ("k_gemm_lowp", "gemm_lowp", ["paper_1701_00182_amd/csrc/gemm_mfma.hip"]),
    ("k_materialize_r", "materialize_r", ["paper_1701_00182_amd/csrc/gram.hip"]),
    ("k_qr<float", "qr", ["paper_1701_00182_amd/csrc/la_lds.hip", "paper_1701_00182_amd/csrc/wave.h"]),
]


def _class_of(kernel):
    """Kernel class of a rocprofv3 kernel name (either precision)."""
    k = kernel.replace("<double", "<float")
    for pre, cls, srcs in PMC_CLASSES + STATS_ONLY_CLASSES:
        if k.startswith(pre):
            return cls, srcs
    return None, None


def summarize_stats(d, precision, workload):
    """profiles/kernel_stats.json, section `precision`: per kernel class, calls,
    total and average duration from the rocprofv3 --stats CSV in d, with the
    SHA-256 of the class's sources (bench.py uses a class's average only while
    they are unchanged)."""
    import csv
    import glob
    import re
    acc = {}
    for path in glob.glob(os.path.join(d, "**", "*_kernel_stats.csv"), recursive=True):
        for r in csv.DictReader(open(path)):
            name = re.sub(r"acr::\(anonymous namespace\)::", "", r["Name"])
            name = re.sub(r"\(.*", "", name).replace("void ", "").strip()
            cls, srcs = _class_of(name)
            if not cls:
                continue
            a = acc.setdefault(cls, {"kernels": set(), "calls": 0, "total_ns": 0.0, "sources": srcs})
            a["kernels"].add(name)
            a["calls"] += int(r["Calls"])
            a["total_ns"] += float(r["TotalDurationNs"])
    try:
        with open(STATS_FILE) as fh:
            out = json.load(fh)
    except (OSError, ValueError):
        out = {}
    sec = {}
    for cls, a in sorted(acc.items(), key=lambda kv: -kv[1]["total_ns"]):
        h = hashlib.sha256()
        for src in a["sources"]:
            with open(os.path.join(ROOT, src), "rb") as fh:
                h.update(fh.read())
        sec[cls] = {"kernels": sorted(a["kernels"]), "calls": a["calls"], "total_ms": a["total_ns"] / 1e6,
                    "avg_ms": a["total_ns"] / 1e6 / a["calls"], "sources": a["sources"], "sha256": h.hexdigest()}
        print(f"{cls:12s} {a['calls']:7d} {a['total_ns'] / 1e6:10.1f} ms {a['total_ns'] / 1e6 / a['calls']:9.4f} ms")
    out[precision] = sec
    out.setdefault("workloads", {})[precision] = workload
    with open(STATS_FILE, "w") as fh:
        json.dump(out, fh, indent=1)


def summarize_pmc(d, workload):
    """profiles/pmc_traffic.json from the rocprofv3 FETCH_SIZE / WRITE_SIZE runs
    in d/{fetch,write} (bench) and d/{cfetch,cwrite} (copy calibration)."""
    import csv
    import glob
    import re

    def per_kernel(sub):
        acc = {}
        for path in glob.glob(os.path.join(d, sub, "*_counter_collection.csv")):
            for r in csv.DictReader(open(path)):
                name = re.sub(r"acr::\(anonymous namespace\)::", "", r["Kernel_Name"])
                name = re.sub(r"\(.*", "", name).replace("void ", "").strip()
                a = acc.setdefault(name, [0, 0.0])
                a[0] += 1
                a[1] += float(r["Counter_Value"])
        return acc

    cf, cw = per_kernel("cfetch"), per_kernel("cwrite")
    copy = next(k for k in cf if "copyBuffer" in k)
    copy_bytes = float(1 << 30)
    fetch_kib, write_kib = cf[copy][1] / cf[copy][0], cw[copy][1] / cw[copy][0]
    scale_f, scale_w = copy_bytes / (fetch_kib * 1024), copy_bytes / (write_kib * 1024)
    bf, bw = per_kernel("fetch"), per_kernel("write")
    classes = {}
    for cls in dict.fromkeys(c for _, c, _ in PMC_CLASSES):
        prefixes = [pre for pre, c, _ in PMC_CLASSES if c == cls]
        srcs = next(sr for _, c, sr in PMC_CLASSES if c == cls)
        names = sorted(k for k in bf if any(k.startswith(pre) for pre in prefixes))
        if not names:
            continue
        nd = sum(bf[k][0] for k in names)
        fk = sum(bf[k][1] for k in names) / nd
        wk = sum(bw.get(k, [1, 0.0])[1] for k in names) / nd
        h = hashlib.sha256()
        for src in srcs:
            with open(os.path.join(ROOT, src), "rb") as fh:
                h.update(fh.read())
        per_launch = DISPATCHES_PER_LAUNCH.get(cls, 1)
        classes[cls] = {"kernels": names, "sources": srcs, "sha256": h.hexdigest(), "dispatches": nd,
                        "dispatches_per_launch": per_launch,
                        "fetch_kib_per_dispatch": round(fk, 1), "write_kib_per_dispatch": round(wk, 1),
                        "bytes_per_launch": per_launch * (fk * scale_f + wk * scale_w) * 1024}
    out = {"workload": workload,
           "calibration": {"kernel": f"{copy} (torch copy of 1 GiB, bench.py --workload copy_calibration)",
                           "copy_bytes": int(copy_bytes), "fetch_kib": round(fetch_kib, 2),
                           "write_kib": round(write_kib, 2), "scale_fetch": scale_f, "scale_write": scale_w},
           "classes": classes}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(out, fh, indent=1)
    for cls, rec in classes.items():
        print(f"{cls:12s} {rec['dispatches']:6d} {rec['fetch_kib_per_dispatch']:14,.0f} "
              f"{rec['write_kib_per_dispatch']:14,.0f} {rec['bytes_per_launch'] / 1e9:10.3f} GB per launch")
    print(f"calibration: fetch x{scale_f:.5f}, write x{scale_w:.5f}")


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="convdiff",
                    choices=["convdiff", "helmholtz_mrhs", "poisson_ir", "gradient", "paper_precond",
                             "helmholtz27", "copy_calibration"])
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--eps", type=float, default=1e-2)
    ap.add_argument("--leaf", type=int, default=128, help="leaf size (also one of the autotuner's candidates)")
    ap.add_argument("--svd-fused-lds", type=int, default=-1, help="core-SVD dispatch (acr_options_t.svd_fused_lds)")
    ap.add_argument("--gemm-tiles", type=int, default=0, help="acr_options_t.gemm_tiles (0: 128 x 32 tiles for "
                                                              "narrow outputs, 1: 64 x 64 only)")
    ap.add_argument("--autotune", action="store_true", help="pick --leaf / --svd-fused-lds with acr_autotune")
    ap.add_argument("--no-autotune", action="store_true", help="use --leaf / --svd-fused-lds as given (default)")
    ap.add_argument("--summarize-pmc", metavar="DIR",
                    help="write profiles/pmc_traffic.json from rocprofv3 FETCH_SIZE / WRITE_SIZE runs in "
                         "DIR/{fetch,write,cfetch,cwrite} (CPU only) and exit")
    ap.add_argument("--tune-planes", type=int, default=8)
    ap.add_argument("--precision", default="fp32",
                    choices=["fp32", "fp64", "fp32_bf16leaf", "fp32_fp16leaf", "fp32_bf16", "fp32_fp16"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--nrhs", type=int, default=256)
    ap.add_argument("--refine-rhs", type=int, default=8, help="helmholtz_mrhs: right-hand sides refined by GMRES")
    ap.add_argument("--h27-n", type=int, nargs="+", default=[32, 64], help="helmholtz27: grid sizes")
    ap.add_argument("--h27-eps", type=float, nargs="+", default=[5e-3, 1e-5], help="helmholtz27: eps per size")
    ap.add_argument("--h27-leaf", type=int, default=32)
    ap.add_argument("--eps-list", type=float, nargs="+", default=[6e-1, 3e-1, 1e-1, 1e-2, 1e-3])
    ap.add_argument("--no-fp64-form", action="store_true")
    ap.add_argument("--no-lowp-form", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precond-sweep", action="store_true",
                    help="skip the eps sweep of the preconditioner (Table precond problem) in the default run")
    ap.add_argument("--summarize-stats", nargs=2, metavar=("DIR", "PRECISION"),
                    help="write the PRECISION section of profiles/kernel_stats.json from the rocprofv3 "
                         "--stats CSV files in DIR (CPU only) and exit")
    ap.add_argument("--cpu-n", type=int, default=22)
    args = ap.parse_args()
    if args.summarize_stats:
        summarize_stats(args.summarize_stats[0], args.summarize_stats[1],
                        f"convection-diffusion n={args.n}, {args.summarize_stats[1].upper()} factors, "
                        f"eps={args.eps:g}, leaf {args.leaf}, svd_fused_lds {args.svd_fused_lds}")
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc,
                      f"convection-diffusion n={args.n}, FP32 factors, eps={args.eps:g}, leaf {args.leaf}, "
                      f"svd_fused_lds {args.svd_fused_lds} (bench.py --steps 1 --warmup 0 --no-fp64-form "
                      f"--no-lowp-form --no-cpu-baseline)")
        return
    ws = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or ws != 1:
        print("bench.py measures one GPU only: the cyclic-reduction hot path is built and timed on a "
              "single MI355X (multi-GPU plane distribution is design-only); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch
    if args.workload == "copy_calibration":
        print(json.dumps(copy_calibration(torch)), flush=True)
        return
    import paper_1701_00182_amd as acr
    fn = {"convdiff": headline, "helmholtz_mrhs": helmholtz_mrhs, "poisson_ir": poisson_ir,
          "gradient": gradient, "paper_precond": paper_precond, "helmholtz27": helmholtz27}[args.workload]
    print(json.dumps(fn(args, torch, acr)), flush=True)


if __name__ == "__main__":
    main()
