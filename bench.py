#!/usr/bin/env python3
"""Benchmark: coupled solve time to 1e-8 relative residual on one MI355X.

Workload: the pressure-based coupled (p, Ux, Uy, Uz) 4x4 system on a
100^3 jittered, randomly renumbered hex mesh (1,000,000 cells, 2,970,000
internal faces; seeded synthetic input).  One step = the whole hot path on
resident device data: LDU -> block-CSR value conversion, AMG setup (FP32
hierarchy, FP64 block inverses and coarse solve) and the mixed-precision
AMG-BiCGStab solve to ||b - A x|| / ||b|| <= 1e-8 from x0 = 0.  The AMG
cycle: W on level 0, one pre- and two post-smoothing block-Jacobi sweeps,
damping 0.9 on level 0 and 1.4 below it (each a command-line option).

Also reported: the plain FP64 GPU path on the same system (mixed vs FP64),
the values-only re-setup + solve variant, the level-1 smoothing sweep (the
kernel launch with the largest share of the step with a W-cycle; the level-0
sweep with a V-cycle), the other level's sweep and the FP64 block SpMV
against the HBM roofline next to a measured copy peak, the CPU oracle timed
on the same system, and three other workloads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0


def seeded_normal(torch, count, dtype, dev, seed):
    """Standard normal device vector from a fixed seed (same values every run)."""
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    return torch.randn(count, dtype=dtype, device=dev, generator=g)

# Bytes per launch on the 100x100x100 p-U system, from FETCH_SIZE and
# WRITE_SIZE counter runs of `bench.py --kernels-only`, each scaled by what the
# counter reads for a 1 GiB copy (profiles/level_kernels_pu1M_hbm_counters.md);
# None where not measured for the current kernel code.  These counters count
# requests from the L2 to the memory fabric, which the 256 MB Infinity Cache
# (MALL) in front of HBM serves in part, so they bound HBM traffic from above.
TRAFFIC_PU1M = {"sweep": 542250086, "sweep_l1": 228149376, "spmv_internal": 1128992973,
                "spmv_caller": 1713110630}
TRAFFIC_KIND = ("L2-to-memory-fabric bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated); the Infinity "
                "Cache serves part of them, so HBM itself moves at most this much")
# Average duration of the same kernels inside timed bench steps (rocprofv3
# --kernel-trace of the default run: W-cycle on level 0, sweeps 1/2,
# coarse damping 1.4,
# profiles/bench_pu1M_kernel_stats.md); None where not measured for the
# current kernel code.
IN_STEP_US_PU1M = {"sweep": 84.32, "sweep_l1": 42.54, "spmv_internal": 182.65, "spmv_caller": None}
IN_STEP_CYCLE = (1, 1.4, 1, 2)          # w_levels, coarse_omega, pre and post sweeps of that run


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mesh", type=int, nargs=3, default=[100, 100, 100])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the other workloads (8M stretched density-based, 64-system batch, 2M adjoint)")
    ap.add_argument("--only", choices=["adjoint_pu_2M", "batch_64", "stretched_density_8M"],
                    help="measure only this one of the other workloads (for per-workload profiles)")
    ap.add_argument("--precond", choices=["amg", "sgs"], default="amg",
                    help="sgs: multicolour symmetric block Gauss-Seidel as the whole preconditioner")
    ap.add_argument("--max-iter", type=int, default=500)
    ap.add_argument("--smoother", choices=["dilu", "sgs", "ilu0", "bjacobi"], default="bjacobi")
    ap.add_argument("--dilu-levels", type=int, default=2)
    ap.add_argument("--pre-sweeps", type=int, default=1)
    ap.add_argument("--post-sweeps", type=int, default=2)
    ap.add_argument("--omega", type=float, default=0.9)
    ap.add_argument("--coarse-max", type=int, default=16)
    ap.add_argument("--passes", type=int, default=2)
    ap.add_argument("--solver", choices=["bicgstab", "fgmres", "gmres"], default="bicgstab")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--tail-rows", type=int, default=0,
                    help="V-cycle tail in one workgroup from levels of at most this many block rows "
                         "(0 = library default, -1 = off)")
    ap.add_argument("--row-split", type=int, default=0,
                    help="threads per scalar row on levels under 32,768 block rows (0 = automatic)")
    ap.add_argument("--scaled-sweeps", type=int, choices=[0, 1], default=1,
                    help="mixed block-Jacobi sweeps on row-scaled FP32 values (1) or with the FP64 D^-1 (0)")
    ap.add_argument("--w-levels", type=int, default=1,
                    help="AMG cycle: W-cycle on this many finest levels (the next level's cycle runs twice), "
                         "0 = V-cycle")
    ap.add_argument("--coarse-omega", type=float, default=1.4,
                    help="block-Jacobi damping below level 0 (0 = --omega on every level)")
    ap.add_argument("--kernel-reps", type=int, default=50)
    ap.add_argument("--assembly", action="store_true",
                    help="only the device assemblies (cbs_assemble_luo, 5x5; cbs_assemble_pu, 4x4) on an "
                         "nx*ny*nz hex box, each against the LDU -> block-CSR conversion of the same pattern "
                         "(cbs_update_values)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="only the level-0 sweep, the FP64 block SpMV (both numberings) and a 1 GiB copy, "
                         "5 launches each, for counter runs")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _method_name(args):
    """The solve the headline step runs, e.g. 'mixed AMG-BiCGStab'."""
    solver = {"bicgstab": "BiCGStab", "fgmres": "FGMRES(30)", "gmres": "GMRES(30)"}[args.solver]
    if args.precond == "sgs":
        return "FP64 %s + symmetric Gauss-Seidel" % solver
    smoother = "" if args.smoother == "bjacobi" else " (%s smoother)" % args.smoother.upper()
    return "mixed AMG-%s%s" % (solver, smoother)


def spmv_bytes(N, nnzb, n, s=8):
    """Algorithmic bytes of one block SpMV: values + column indices + row
    pointers + x read once + y written once."""
    return nnzb * (n * n * s + 4) + (N + 1) * 4 + 2 * N * n * s


def sweep_bytes(N, nnzb, n, s=4, dinv=False):
    """Algorithmic bytes of one block-Jacobi sweep y = x + w Dinv (b - A x):
    values + column indices + row pointers + x, b read once + y written once.
    The FP64 sweep also reads the block inverses; the row-scaled FP32 sweep
    has them folded into its values and stores no diagonal blocks (the
    scaled diagonal block is the identity), so it reads nnzb - N blocks."""
    if dinv:
        return nnzb * (n * n * s + 4) + (N + 1) * 4 + 3 * N * n * s + N * n * n * 8
    return (nnzb - N) * (n * n * s + 4) + (N + 1) * 4 + 3 * N * n * s


def _host_cpu():
    """CPU model and the cores this process may run on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": len(os.sched_getaffinity(0)), "cpu_count": os.cpu_count(), "model": model}


def cpu_baseline(s, cyc, reps_max=3, budget_s=60.0):
    """The CPU oracle on the same system as the GPU step: LDU -> block CSR,
    reference AMG setup (block Jacobi, coarse_max 16, two matching passes,
    and the GPU step's cycle: its sweeps, dampings and W levels) and
    BiCGStab to 1e-8, FP64, with the OpenMP threads of
    the host.  One warm-up run, then the median of up to three runs (fewer
    when three would exceed the time budget).  Also one thread: conversion,
    setup and the first 5 iterations (the full solve would take minutes)."""
    import ctypes as C
    import oracle as O
    O.lib()
    gomp = C.CDLL("libgomp.so.1")            # the OpenMP runtime liboracle.so runs on
    threads = int(gomp.omp_get_max_threads())

    def run(maxit=500):
        t0 = time.perf_counter()
        A = O.from_system(s)
        t1 = time.perf_counter()
        amg = O.AMG(A, coarse_max=16, passes=2, smoother=O.SMOOTH_BJACOBI, nu1=cyc["pre_sweeps"],
                    nu2=cyc["post_sweeps"], omega=cyc["omega"], w_levels=cyc["w_levels"],
                    coarse_omega=cyc["coarse_omega"])
        t2 = time.perf_counter()
        _, st = O.bicgstab(A, s["b"], prec=O.PREC_AMG, amg=amg, tol=1e-8, maxit=maxit)
        t3 = time.perf_counter()
        del amg, A
        return {"total_s": t3 - t0, "convert_s": t1 - t0, "setup_s": t2 - t1, "solve_s": t3 - t2,
                "iterations": st["iterations"], "relres": st["relres"]}

    warm = run()
    log("cpu oracle warm-up: %.2f s (%d iterations)" % (warm["total_s"], warm["iterations"]))
    reps = reps_max if reps_max * warm["total_s"] <= budget_s else 1
    runs = [run() for _ in range(reps)]
    tot = sorted(r["total_s"] for r in runs)
    med = tot[len(tot) // 2]
    mid = [r for r in runs if r["total_s"] == med][0]
    log("cpu oracle: median %.2f s of %d runs, %d threads" % (med, reps, threads))
    gomp.omp_set_num_threads(1)
    try:
        one = run(maxit=5)
    finally:
        gomp.omp_set_num_threads(threads)
    log("cpu oracle, 1 thread: setup %.2f s, %.3f s per iteration" % (one["convert_s"] + one["setup_s"],
                                                                     one["solve_s"] / max(1, one["iterations"])))
    return {
        "value": round(med * 1e3, 1),
        "unit": "ms per solve (LDU conversion + AMG setup + BiCGStab to 1e-8)",
        "cores": threads,
        "kind": "oracle",
        "sample": "the whole bench system (%d cells): oracle LDU -> block CSR, reference AMG setup (block-Jacobi "
                  "sweeps %d/%d, omega %g, coarse omega %g, %s) and BiCGStab to 1e-8 in FP64 on %d OpenMP "
                  "threads; one warm-up run, then the median of %d runs"
                  % (s["N"], cyc["pre_sweeps"], cyc["post_sweeps"], cyc["omega"], cyc["coarse_omega"],
                     "W-cycle on the %d finest levels" % cyc["w_levels"] if cyc["w_levels"] else "V-cycle",
                     threads, reps),
        "runs_s": [round(r["total_s"], 3) for r in runs],
        "iterations": mid["iterations"],
        "phases_s": {k: round(mid[k], 3) for k in ("convert_s", "setup_s", "solve_s")},
        "one_thread": {"convert_setup_s": round(one["convert_s"] + one["setup_s"], 3),
                       "iterations_timed": one["iterations"],
                       "s_per_iteration": round(one["solve_s"] / max(1, one["iterations"]), 4),
                       "sample": "1 OpenMP thread: conversion, setup and the first %d BiCGStab iterations on the "
                                 "same system" % one["iterations"]},
        "host": _host_cpu(),
    }


def internal_system(P, torch, dev, sysm, N, n, la, ua, diag, upper, lower):
    """A second handle holding the same matrix in the solver's internal
    (aggregation-tree) row numbering, for the FP64 SpMV on that numbering."""
    order = sysm.get_level(0)["order"].long()
    pos = torch.empty_like(order)
    pos[order] = torch.arange(N, device=dev)
    return P.System(N, n, pos[la.long()].int(), pos[ua.long()].int(), diag[order], upper, lower)


class KernelTimer:
    """Average launch time of one library call over `reps` launches, with HIP
    events on the stream the library launches on (torch's current stream)."""

    def __init__(self, torch, reps):
        self.torch, self.reps = torch, reps

    def __call__(self, fn, warm=5):
        for _ in range(warm):
            fn()
        e0 = self.torch.cuda.Event(enable_timing=True)
        e1 = self.torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(self.reps):
            fn()
        e1.record()
        self.torch.cuda.synchronize()
        return e0.elapsed_time(e1) / self.reps       # ms


def level_sweep_call(P, torch, dev, sysm, n, level=0, op=None):
    """Closure running the smoothing sweep (or, with op, another level kernel)
    of one level of the current hierarchy on random vectors, and whether it
    runs in FP32."""
    import ctypes as C
    L = P.lib()
    op = P.LEVEL_SWEEP if op is None else op
    f = C.c_int32(0)
    L.cbs_level_apply(sysm.h, level, op, None, None, None, C.byref(f))
    n0 = sysm.get_level(level)["N"]
    dt = torch.float32 if f.value else torch.float64
    bv = seeded_normal(torch, n0 * n, dt, dev, 101)
    xv = seeded_normal(torch, n0 * n, dt, dev, 102)
    yv = torch.empty_like(xv)

    def run():
        rc = L.cbs_level_apply(sysm.h, level, op, C.c_void_p(bv.data_ptr()), C.c_void_p(xv.data_ptr()),
                               C.c_void_p(yv.data_ptr()), None)
        if rc < 0:
            raise P.CbsError(rc, "cbs_level_apply")
    return run, bool(f.value)


def spmv_call(P, torch, dev, system, N, n):
    import ctypes as C
    L = P.lib()
    xv = seeded_normal(torch, N * n, torch.float64, dev, 103)
    yv = torch.empty_like(xv)
    return lambda: L.cbs_spmv(system.h, C.c_void_p(xv.data_ptr()), C.c_void_p(yv.data_ptr()), 0)


def kernels_only(args, P, torch, dev, sysm, opt_mixed, N, n, nnzb, la, ua, diag, upper, lower):
    """Five launches each of the level-0 mixed-precision sweep, the FP64
    block SpMV on both numberings, and the sweep and residual of levels 1 and
    2, then a plain 1 GiB copy (the calibration kernel of the HBM byte
    counters)."""
    sysm.setup(opt_mixed)
    sweep, _ = level_sweep_call(P, torch, dev, sysm, n)
    sys2 = internal_system(P, torch, dev, sysm, N, n, la, ua, diag, upper, lower)
    coarse = [level_sweep_call(P, torch, dev, sysm, n, level=l, op=op)[0]
              for l in (1, 2) for op in (P.LEVEL_SWEEP, P.LEVEL_RESIDUAL)]
    for fn in (sweep, spmv_call(P, torch, dev, sysm, N, n), spmv_call(P, torch, dev, sys2, N, n), *coarse):
        for _ in range(5):
            fn()
        torch.cuda.synchronize()
    a = torch.empty(1 << 27, dtype=torch.float64, device=dev)     # 1 GiB
    a.fill_(1.0)
    bcopy = torch.empty_like(a)
    for _ in range(3):
        bcopy.copy_(a)
    torch.cuda.synchronize()
    sys2.close()
    lv = sysm.get_level(0)
    lvs = [sysm.get_level(l) for l in (1, 2)]
    print(json.dumps({"launches_per_kernel": 5, "order": ["sweep", "spmv caller", "spmv internal", "level-1 sweep",
                                                          "level-1 residual", "level-2 sweep", "level-2 residual",
                                                          "copy"],
                      "levels_1_2": [{"N": q["N"], "nnzb": q["nnzb"],
                                      "algorithmic_bytes_sweep": int(sweep_bytes(q["N"], q["nnzb"], n)),
                                      "algorithmic_bytes_residual": int(q["nnzb"] * (n * n * 4 + 4) + (q["N"] + 1) * 4
                                                                        + 3 * q["N"] * n * 4)} for q in lvs],
                      "algorithmic_bytes_sweep": int(sweep_bytes(lv["N"], lv["nnzb"], n)),
                      "algorithmic_bytes_spmv": int(spmv_bytes(N, nnzb, n)),
                      "copy_bytes_read": int(a.numel() * 8), "copy_bytes_written": int(a.numel() * 8)}))


def assembly_only(args, P, torch, dev):
    """Device assemblies of the 5x5 density-based matrix (cell states, face
    vectors) and of the 4x4 pressure-based matrix (face geometry and fluxes),
    each timed per call (HIP events; each call ends with its non-finite check
    read-back) next to the LDU -> block-CSR conversion that it replaces.
    Algorithmic bytes: the block-CSR values written, the slot map, row
    pointers and every per-face and per-cell input read once."""
    from workloads import luo_inputs
    nx, ny, nz = args.mesh
    t0 = time.time()
    d = luo_inputs(nx, ny, nz, seed=0)
    log("generated assembly inputs %dx%dx%d in %.1f s" % (nx, ny, nz, time.time() - t0))
    N, F = d["N"], d["F"]
    dv = lambda a: torch.tensor(a, device=dev)
    la, ua = dv(d["lower_addr"]), dv(d["upper_addr"])
    diag = torch.zeros((N, 5, 5), dtype=torch.float64, device=dev)
    upper = torch.zeros((F, 5, 5), dtype=torch.float64, device=dev)
    lower = torch.zeros((F, 5, 5), dtype=torch.float64, device=dev)
    Q, Sf, lv, vd = dv(d["Q"]), dv(d["Sf"]), dv(d["lam_visc"]), dv(d["v_dt"])
    with P.System(N, 5, la, ua, diag, upper, lower) as sysm:
        timer = KernelTimer(torch, args.kernel_reps)
        asm_ms = timer(lambda: sysm.assemble_luo(Q, Sf, lv, vd, d["gamma"]))
        conv_ms = timer(lambda: sysm.update_values(diag, upper, lower))
        del diag, upper, lower
    nnzb = N + 2 * F
    abytes = nnzb * 25 * 8 + nnzb * 4 + (N + 1) * 4 + N * 5 * 8 + F * (3 * 8 + 8 + 2 * 4) + N * 8
    cbytes = 2 * nnzb * 25 * 8 + nnzb * 4
    # the pressure-based (p, U) assembly on the same box
    from workloads import pu_inputs
    e = pu_inputs(nx, ny, nz, seed=0)
    d4 = torch.zeros((N, 4, 4), dtype=torch.float64, device=dev)
    u4 = torch.zeros((F, 4, 4), dtype=torch.float64, device=dev)
    l4 = torch.zeros((F, 4, 4), dtype=torch.float64, device=dev)
    pargs = [dv(e[k]) for k in ("Sf", "fx", "d", "flux", "nu", "vol", "uu_add", "pp_add")]
    with P.System(N, 4, la, ua, d4, u4, l4) as s4:
        timer = KernelTimer(torch, args.kernel_reps)
        pu_ms = timer(lambda: s4.assemble_pu(*pargs))
        pconv_ms = timer(lambda: s4.update_values(d4, u4, l4))
    pbytes = nnzb * 16 * 8 + nnzb * 4 + (N + 1) * 4 + F * (3 * 8 + 8 + 3 * 8 + 8 + 8 + 2 * 4) + N * 3 * 8
    # a plain 1 GiB copy, the calibration kernel of the HBM byte counters
    a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    a.fill_(1.0)
    bcopy = torch.empty_like(a)
    for _ in range(3):
        bcopy.copy_(a)
    torch.cuda.synchronize()
    del a, bcopy
    print(json.dumps({"metric": "coupled matrix assembly on the device", "unit": "ms",
                      "config": {"workload": "jittered hex box %dx%dx%d (N=%d, F=%d, nnzb=%d)"
                                             % (nx, ny, nz, N, F, nnzb)},
                      "assemble_ms": round(asm_ms, 4), "assemble_gbs": round(abytes / (asm_ms * 1e-3) / 1e9, 1),
                      "algorithmic_bytes_assemble": int(abytes),
                      "ldu_convert_ms": round(conv_ms, 4), "ldu_convert_gbs": round(cbytes / (conv_ms * 1e-3) / 1e9, 1),
                      "algorithmic_bytes_convert": int(cbytes),
                      "pu_assemble_ms": round(pu_ms, 4), "pu_assemble_gbs": round(pbytes / (pu_ms * 1e-3) / 1e9, 1),
                      "algorithmic_bytes_pu_assemble": int(pbytes), "pu_ldu_convert_ms": round(pconv_ms, 4)}))


def level_kobj(name, ms, nbytes):
    gb = nbytes / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": name, "achieved": round(gb, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gb / HBM_PEAK_GBS, 4), "avg_launch_us": round(ms * 1e3, 2), "algorithmic_bytes": int(nbytes)}


def measure_system(P, torch, dev, s, opt, steps, key, name, transposed=False):
    """Upload one generated system (or batch), then time `steps` steps of
    update_values + setup + solve from x0 = 0 (after one warm-up step), and
    the level-0 block-Jacobi sweep and FP64 block SpMV alone (HIP events)."""
    n = s["n"]
    dv = lambda a: torch.tensor(a, device=dev)
    la, ua, diag, upper, lower = (dv(s[k]) for k in ("lower_addr", "upper_addr", "diag", "upper", "lower"))
    b = dv(s["b"]).reshape(-1)
    x = torch.zeros_like(b)
    kw = {"cell_off": s["cell_off"], "face_off": s["face_off"]} if "cell_off" in s else {}
    sysm = P.System(s["N"], n, la, ua, diag, upper, lower, **kw)
    N, nnzb = s["N"], sysm.info()["nnzb"]

    def step():
        sysm.update_values(diag, upper, lower)
        sysm.setup(opt)
        x.zero_()
        _, st = sysm.solve(b, x0=x)
        return st

    step()
    torch.cuda.synchronize()
    per = []
    for _ in range(steps):
        t0 = time.perf_counter()
        st = step()
        torch.cuda.synchronize()
        per.append((time.perf_counter() - t0) * 1e3)
    sts = st if isinstance(st, list) else [st]
    its = [q["iterations"] for q in sts]
    res = {"workload": name, "ms_per_step": round(float(np.median(per)), 3),
           "step": "update_values + setup + solve", "steps": steps, "step_ms_all": [round(t, 3) for t in per],
           "iterations": its[0] if len(its) == 1 else {"min": min(its), "max": max(its),
                                                      "mean": round(float(np.mean(its)), 2)},
           "setup_ms": round(sts[0]["t_setup_ms"], 3), "solve_ms": round(sts[0]["t_solve_ms"], 3),
           "status_ok": all(q["status"] == P.OK for q in sts),
           "precision_fallback": max(q["precision_fallback"] for q in sts),
           "rel_res_true_max": max(q["rel_res_true"] for q in sts), "levels": sts[0]["levels"]}
    log("%s: %.1f ms/step, iterations %s, setup %.1f ms, solve %.1f ms" % (key, res["ms_per_step"], res["iterations"],
                                                                           res["setup_ms"], res["solve_ms"]))
    timer = KernelTimer(torch, 20)
    if transposed:
        g = seeded_normal(torch, N * n, torch.float64, dev, 104)
        sysm.solve_transpose(g)                          # builds the transposed hierarchy
        t0 = time.perf_counter()
        lam, stt = sysm.solve_transpose(g)
        torch.cuda.synchronize()
        res["transposed_solve_ms"] = round((time.perf_counter() - t0) * 1e3, 3)
        res["transposed_iterations"] = stt["iterations"]
        xs, _ = sysm.solve(b)
        gd = torch.empty((N, n, n), dtype=torch.float64, device=dev)
        gu = torch.empty((s["F"], n, n), dtype=torch.float64, device=dev)
        gl = torch.empty_like(gu)
        import ctypes as C
        L = P.lib()
        res["gradient_us"] = round(timer(lambda: L.cbs_gradient(
            sysm.h, C.c_void_p(lam.data_ptr()), C.c_void_p(xs.data_ptr()), C.c_void_p(gd.data_ptr()),
            C.c_void_p(gu.data_ptr()), C.c_void_p(gl.data_ptr()))) * 1e3, 2)
        del gd, gu, gl
        log("%s: transposed solve %.1f ms (%d iterations)" % (key, res["transposed_solve_ms"],
                                                              res["transposed_iterations"]))
    lv0 = sysm.get_level(0)
    sweep, fp32 = level_sweep_call(P, torch, dev, sysm, n)
    sweep_ms = timer(sweep)
    res["level0_sweep"] = level_kobj("level-0 block-Jacobi sweep, %s" % ("FP32 row-scaled" if fp32 else "FP64"),
                                     sweep_ms, sweep_bytes(lv0["N"], lv0["nnzb"], n, 4 if fp32 else 8,
                                                           dinv=not fp32))
    spmv_ms = timer(spmv_call(P, torch, dev, sysm, N, n))
    res["spmv_fp64"] = level_kobj("block SpMV FP64, caller's numbering", spmv_ms, spmv_bytes(N, nnzb, n))
    log("%s: level-0 sweep %.1f us (%.2f of peak), spmv %.1f us (%.2f)" % (
        key, sweep_ms * 1e3, res["level0_sweep"]["frac"], spmv_ms * 1e3, res["spmv_fp64"]["frac"]))
    sysm.close()
    del la, ua, diag, upper, lower, b, x
    torch.cuda.empty_cache()
    return res


def other_configs(args, P, torch, dev, only=None):
    """The other synthetic workloads, each in its own launch configuration:
    the 8M-cell density-based system on a boundary-layer mesh (mixed
    AMG-FGMRES(30)), the 64-system batch (one batched mixed AMG-BiCGStab
    solve) and the 2M-cell p-U adjoint (mixed forward and transposed solves,
    LDU gradient).  The p-U system takes the main run's cycle shape; the two
    density-based workloads run V-cycles, since a W-cycle on level 0 leaves
    their iteration counts unchanged (3 per batch system, 80 on the stretched
    mesh) and only adds work."""
    from workloads import jacobian_batch, jacobian_stretched, pressure_velocity
    out = {}
    if only is None or only == "adjoint_pu_2M":
        out.update(_adjoint_2M(P, torch, dev, pressure_velocity, dict(
            w_levels=args.w_levels, coarse_omega=args.coarse_omega, pre_sweeps=args.pre_sweeps,
            post_sweeps=args.post_sweeps, omega=args.omega)))
    if only is None or only == "batch_64":
        out.update(_batch_64(P, torch, dev, jacobian_batch, 0))
    if only is None or only == "stretched_density_8M":
        out.update(_stretched_8M(P, torch, dev, jacobian_stretched, 0))
    return out


def _adjoint_2M(P, torch, dev, pressure_velocity, cyc):
    out = {}
    t0 = time.time()
    s = pressure_velocity(200, 100, 100, seed=0)
    log("generated 2M p-U in %.1f s" % (time.time() - t0))
    out["adjoint_pu_2M"] = measure_system(
        P, torch, dev, s, P.default_options(precision=P.PRECISION_MIXED, tol=1e-8, **cyc), 3, "adjoint_pu_2M",
        "pressure-based p-U 4x4, 200x100x100 jittered renumbered hex mesh (N=%d); mixed AMG-BiCGStab to 1e-8, "
        "forward and transposed" % s["N"], transposed=True)
    return out


def _batch_64(P, torch, dev, jacobian_batch, wl):
    out = {}
    t0 = time.time()
    s = jacobian_batch(64, seed=0)
    log("generated the 64-system batch (%d cells) in %.1f s" % (s["N"], time.time() - t0))
    out["batch_64"] = measure_system(
        P, torch, dev, s, P.default_options(precision=P.PRECISION_MIXED, tol=1e-8, w_levels=wl), 3, "batch_64",
        "64 density-based 5x5 systems, 10k-500k cells each (N=%d in total); one batched mixed AMG-BiCGStab "
        "solve to 1e-8 per system" % s["N"])
    return out


def _stretched_8M(P, torch, dev, jacobian_stretched, wl):
    out = {}
    t0 = time.time()
    s = jacobian_stretched(200, 200, 200, seed=0)
    log("generated 8M stretched in %.1f s" % (time.time() - t0))
    out["stretched_density_8M"] = measure_system(
        P, torch, dev, s, P.default_options(precision=P.PRECISION_MIXED, solver=P.SOLVER_FGMRES, restart=30,
                                            tol=1e-8, w_levels=wl), 2, "stretched_density_8M",
        "density-based 5x5, 200^3 boundary-layer mesh (wall-normal ratio 1.2, aspect ratio up to 1e3, "
        "N=%d); mixed AMG-FGMRES(30) to 1e-8" % s["N"])
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X; "
              "a row-partitioned multi-GPU solve is not implemented", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2403_07882_amd as P
    from workloads import pressure_velocity

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.assembly:
        assembly_only(args, P, torch, dev)
        return
    if args.only:
        print(json.dumps(other_configs(args, P, torch, dev, only=args.only)), flush=True)
        return
    nx, ny, nz = args.mesh
    log("generating pressure-velocity system %dx%dx%d" % (nx, ny, nz))
    t0 = time.time()
    s = pressure_velocity(nx, ny, nz, seed=0)
    log("generated in %.1f s: N=%d F=%d" % (time.time() - t0, s["N"], s["F"]))
    N, F, n = s["N"], s["F"], s["n"]
    la = torch.tensor(s["lower_addr"], device=dev)
    ua = torch.tensor(s["upper_addr"], device=dev)
    diag = torch.tensor(s["diag"], device=dev)
    upper = torch.tensor(s["upper"], device=dev)
    lower = torch.tensor(s["lower"], device=dev)
    # right-hand side as per-variable fields (p, Ux, Uy, Uz), as a CFD code holds them
    b_fields = torch.tensor(np.ascontiguousarray(s["b"].T), device=dev)
    x_fields = torch.empty_like(b_fields)
    b = P.pack_fields(b_fields).reshape(-1)
    x = torch.zeros_like(b)
    s_host = s                     # host LDU arrays, for the CPU oracle at the end
    del s
    sysm = P.System(N, n, la, ua, diag, upper, lower)
    nnzb = sysm.info()["nnzb"]
    common = dict(solver={"fgmres": P.SOLVER_FGMRES, "gmres": P.SOLVER_GMRES}.get(args.solver, P.SOLVER_BICGSTAB),
                  precond=P.PREC_SGS if args.precond == "sgs" else P.PREC_AMG, tol=1e-8, max_iter=args.max_iter,
                  smoother={"dilu": P.SMOOTH_DILU, "sgs": P.SMOOTH_SGS, "ilu0": P.SMOOTH_ILU0}.get(args.smoother, P.SMOOTH_BJACOBI),
                  dilu_levels=args.dilu_levels, pre_sweeps=args.pre_sweeps, post_sweeps=args.post_sweeps,
                  omega=args.omega, coarse_max=args.coarse_max, match_passes=args.passes,
                  row_split=args.row_split, tail_rows=args.tail_rows, scaled_sweeps=args.scaled_sweeps,
                  w_levels=args.w_levels, coarse_omega=args.coarse_omega)
    opt_mixed = P.default_options(precision=P.PRECISION_MIXED, **common)
    opt_reuse = P.default_options(precision=P.PRECISION_MIXED, reuse_aggregates=1, **common)
    opt_fp64 = P.default_options(precision=P.PRECISION_FP64, **common)
    if args.kernels_only:
        kernels_only(args, P, torch, dev, sysm, opt_mixed, N, n, nnzb, la, ua, diag, upper, lower)
        return

    L = P.lib()
    import ctypes as C
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def step(opt):
        # pack fields -> LDU values to block CSR -> setup -> solve -> unpack fields
        L.cbs_pack_fields(N, n, C.c_void_p(b_fields.data_ptr()), C.c_void_p(b.data_ptr()), stream)
        sysm.update_values(diag, upper, lower)
        sysm.setup(opt)
        x.zero_()
        st = P.Stats()
        rc = L.cbs_solve(sysm.h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), C.byref(st))
        if rc < 0:
            raise P.CbsError(rc, "cbs_solve")
        L.cbs_unpack_fields(N, n, C.c_void_p(x.data_ptr()), C.c_void_p(x_fields.data_ptr()), stream)
        return st.as_dict()

    def run_steps(opt, k):
        """Time k steps: total over the bracketed region, and each step."""
        per = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            t1 = time.perf_counter()
            st = step(opt)
            torch.cuda.synchronize()
            per.append((time.perf_counter() - t1) * 1e3)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / k * 1e3, per, st

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        step(opt_mixed)
    torch.cuda.synchronize()
    log("timing %d steps (mixed)" % args.steps)
    t_mixed, per_step, st = run_steps(opt_mixed, args.steps)
    if st["precision_fallback"]:
        log("WARNING: the mixed-precision hierarchy escalated to FP64")
    log("mixed: %.2f ms/step (median %.2f), iterations %d, relres %.3e, setup %.2f ms, solve %.2f ms"
        % (t_mixed, float(np.median(per_step)), st["iterations"], st["rel_res_true"], st["t_setup_ms"],
           st["t_solve_ms"]))
    # values-only re-setup (aggregates kept) + solve: the branch of the
    # nonlinear loop where only the coefficients change
    t_reuse, per_reuse, st_reuse = run_steps(opt_reuse, max(1, args.steps))
    log("values-only re-setup + solve: %.2f ms/step (setup %.2f ms)" % (t_reuse, st_reuse["t_setup_ms"]))

    # plain FP64 GPU path on the same system
    t_fp64, st64 = float("nan"), {"iterations": -1}
    if not args.skip_fp64:
        for _ in range(max(1, args.warmup // 2)):
            step(opt_fp64)
        t_fp64, _, st64 = run_steps(opt_fp64, max(1, args.steps // 2))
        log("fp64: %.2f ms/step, iterations %d" % (t_fp64, st64["iterations"]))

    # the remaining rows of the path on the same system: field packing, the
    # adjoint (transposed solve + LDU gradient), each timed with HIP events
    timer = KernelTimer(torch, args.kernel_reps)
    pack_ms = timer(lambda: L.cbs_pack_fields(N, n, C.c_void_p(b_fields.data_ptr()), C.c_void_p(b.data_ptr()), stream))
    unpack_ms = timer(lambda: L.cbs_unpack_fields(N, n, C.c_void_p(x.data_ptr()), C.c_void_p(x_fields.data_ptr()),
                                                  stream))
    sysm.setup(opt_mixed)
    gvec = seeded_normal(torch, N * n, torch.float64, dev, 104)
    lam = torch.zeros_like(gvec)
    xsol = torch.zeros_like(gvec)
    st_f = P.Stats()
    L.cbs_solve(sysm.h, C.c_void_p(b.data_ptr()), C.c_void_p(xsol.data_ptr()), C.byref(st_f))
    st_t = P.Stats()

    def adjoint_solve():
        lam.zero_()
        rc = L.cbs_solve_transpose(sysm.h, C.c_void_p(gvec.data_ptr()), C.c_void_p(lam.data_ptr()), C.byref(st_t))
        if rc < 0:
            raise P.CbsError(rc, "cbs_solve_transpose")
    adjoint_solve()                                     # builds the transposed hierarchy once
    adj_ms = KernelTimer(torch, 3)(adjoint_solve, warm=1)
    gd = torch.empty((N, n, n), dtype=torch.float64, device=dev)
    gu = torch.empty((F, n, n), dtype=torch.float64, device=dev)
    gl = torch.empty((F, n, n), dtype=torch.float64, device=dev)
    grad_ms = timer(lambda: L.cbs_gradient(sysm.h, C.c_void_p(lam.data_ptr()), C.c_void_p(xsol.data_ptr()),
                                           C.c_void_p(gd.data_ptr()), C.c_void_p(gu.data_ptr()),
                                           C.c_void_p(gl.data_ptr())))
    del gd, gu, gl
    log("pack %.1f us, unpack %.1f us; transposed solve %.2f ms (%d iterations), gradient %.1f us"
        % (pack_ms * 1e3, unpack_ms * 1e3, adj_ms, st_t.iterations, grad_ms * 1e3))

    r64 = seeded_normal(torch, N * n, torch.float64, dev, 105)
    z64 = torch.empty_like(r64)
    vcyc_ms = timer(lambda: L.cbs_apply_precond(sysm.h, C.c_void_p(r64.data_ptr()), C.c_void_p(z64.data_ptr())),
                    warm=2)
    log("V-cycle (cbs_apply_precond, mixed): %.3f ms" % vcyc_ms)

    # kernels, each timed alone with HIP events on the library's stream; the
    # roofline kernel is the block-Jacobi sweep, so a run with a coloured
    # smoother or preconditioner times it on a block-Jacobi AMG hierarchy of
    # the same system
    sysm.setup(opt_mixed if args.smoother == "bjacobi" and args.precond == "amg" else
               P.default_options(precision=P.PRECISION_MIXED,
                                 **dict(common, precond=P.PREC_AMG, smoother=P.SMOOTH_BJACOBI)))
    lv0 = sysm.get_level(0)
    sweep, sweep_fp32 = level_sweep_call(P, torch, dev, sysm, n)
    sweep_ms = timer(sweep)
    sbytes = sweep_bytes(lv0["N"], lv0["nnzb"], n, 4 if sweep_fp32 else 8, dinv=not sweep_fp32)
    sweep_gbs = sbytes / (sweep_ms * 1e-3) / 1e9
    log("level-0 sweep (%s): %.1f us, %.0f GB/s" % ("fp32" if sweep_fp32 else "fp64", sweep_ms * 1e3, sweep_gbs))
    lv1 = sysm.get_level(1)
    sweep1, _ = level_sweep_call(P, torch, dev, sysm, n, level=1)
    sweep1_ms = timer(sweep1)
    sbytes1 = sweep_bytes(lv1["N"], lv1["nnzb"], n, 4 if sweep_fp32 else 8, dinv=not sweep_fp32)
    log("level-1 sweep: %.1f us, %.0f GB/s" % (sweep1_ms * 1e3, sbytes1 / (sweep1_ms * 1e-3) / 1e9))
    byts = spmv_bytes(N, nnzb, n)
    spmv_user_ms = timer(spmv_call(P, torch, dev, sysm, N, n))
    gbs_user = byts / (spmv_user_ms * 1e-3) / 1e9
    log("spmv fp64 (caller numbering): %.1f us, %.0f GB/s" % (spmv_user_ms * 1e3, gbs_user))
    sys2 = internal_system(P, torch, dev, sysm, N, n, la, ua, diag, upper, lower)
    spmv_ms = timer(spmv_call(P, torch, dev, sys2, N, n))
    sys2.close()
    gbs = byts / (spmv_ms * 1e-3) / 1e9
    log("spmv fp64 (internal numbering): %.1f us, %.0f GB/s" % (spmv_ms * 1e3, gbs))
    # measured copy peak: 1 GiB device-to-device copy (read + write bytes)
    a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    a.fill_(1.0)
    bcopy = torch.empty_like(a)
    copy_ms = KernelTimer(torch, 10)(lambda: bcopy.copy_(a), warm=2)
    copy_gbs = 2 * a.numel() * 8 / (copy_ms * 1e-3) / 1e9
    del a, bcopy
    log("1 GiB copy: %.1f us, %.0f GB/s" % (copy_ms * 1e3, copy_gbs))
    full = (nx, ny, nz) == (100, 100, 100)

    sweep_desc = "FP32 row-scaled off-diagonal" if sweep_fp32 else "FP64"

    def kobj(name, ms, nbytes, key):
        gb = nbytes / (ms * 1e-3) / 1e9
        o = {"bound": "hbm", "kernel": name, "achieved": round(gb, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": round(gb / HBM_PEAK_GBS, 4), "traffic": TRAFFIC_PU1M[key] if full else None,
             "traffic_kind": TRAFFIC_KIND, "avg_launch_us": round(ms * 1e3, 2), "algorithmic_bytes": int(nbytes)}
        cyc = (args.w_levels, args.coarse_omega, args.pre_sweeps, args.post_sweeps)
        us = IN_STEP_US_PU1M[key] if full and cyc == IN_STEP_CYCLE else None
        if us:
            o["in_step"] = {"avg_launch_us": us, "frac": round(nbytes / (us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                            "source": "rocprofv3 kernel trace of timed bench steps"}
        return o

    out = {
        "metric": "coupled solve time to 1e-8 rel. residual; block-SpMV GB/s; mixed vs FP64",
        "value": round(t_mixed, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(t_mixed, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 outer / f32 AMG",
        "data": "synthetic",
        "config": {"workload": "pressure-based coupled p-U 4x4, %dx%dx%d jittered hex mesh, cells "
                               "randomly renumbered (N=%d, F=%d, nnzb=%d); %s to 1e-8"
                               % (nx, ny, nz, N, F, nnzb, _method_name(args)),
                   "step": "pack fields + update_values + setup + solve + unpack fields",
                   "precond": args.precond, "max_iter": args.max_iter,
                   "solver": args.solver, "smoother": args.smoother, "dilu_levels": args.dilu_levels,
                   "pre_sweeps": args.pre_sweeps, "post_sweeps": args.post_sweeps, "omega": args.omega,
                   "coarse_omega": args.coarse_omega, "coarse_max": args.coarse_max,
                   "match_passes": args.passes, "row_split": args.row_split,
                   "tail_rows": args.tail_rows, "scaled_sweeps": args.scaled_sweeps, "w_levels": args.w_levels},
        "step_ms_median": round(float(np.median(per_step)), 3),
        "step_ms_all": [round(t, 3) for t in per_step],
        "iterations": st["iterations"],
        "precision_fallback": st["precision_fallback"],
        "rel_res_true": st["rel_res_true"],
        "levels": st["levels"],
        "op_complexity": round(st["op_complexity"], 3),
        "setup_ms": round(st["t_setup_ms"], 3),
        "solve_ms": round(st["t_solve_ms"], 3),
        "convert_ms": round(st["t_convert_ms"], 3),
        "values_only_resetup_ms_per_step": round(t_reuse, 3),
        "values_only_setup_ms": round(st_reuse["t_setup_ms"], 3),
        "fp64_ms_per_step": round(t_fp64, 3),
        "fp64_iterations": st64["iterations"],
        "mixed_vs_fp64_speedup": round(t_fp64 / t_mixed, 3) if t_fp64 == t_fp64 else None,
        "vcycle_ms": round(vcyc_ms, 4),
        "pack_fields_us": round(pack_ms * 1e3, 2),
        "unpack_fields_us": round(unpack_ms * 1e3, 2),
        "transposed_solve_ms": round(adj_ms, 3),
        "transposed_iterations": st_t.iterations,
        "gradient_us": round(grad_ms * 1e3, 2),
        # the W-cycle visits level 1 twice per cycle: its sweep then has the
        # largest share of the step (17% against 15% for level 0's)
        "roofline": (kobj("level-1 block-Jacobi sweep, %s (k_rows, %d block rows, %d blocks); the kernel launch "
                          "with the largest share of the step" % (sweep_desc, lv1["N"], lv1["nnzb"]),
                          sweep1_ms, sbytes1, "sweep_l1") if args.w_levels >= 1 else
                     kobj("level-0 block-Jacobi sweep, %s (k_rows, internal numbering); the kernel launch with the "
                          "largest share of the step" % sweep_desc, sweep_ms, sbytes, "sweep")),
        ("level0_sweep" if args.w_levels >= 1 else "level1_sweep"):
            (kobj("level-0 block-Jacobi sweep, %s (k_rows, internal numbering)" % sweep_desc, sweep_ms, sbytes,
                  "sweep") if args.w_levels >= 1 else
             kobj("level-1 block-Jacobi sweep, %s (k_rows)" % sweep_desc, sweep1_ms, sbytes1, "sweep_l1")),
        "spmv_fp64": kobj("block SpMV FP64 (k_rows mode 0), internal numbering", spmv_ms, byts, "spmv_internal"),
        "spmv_fp64_caller_numbering": kobj("block SpMV FP64 (k_rows mode 0), caller's random numbering",
                                           spmv_user_ms, byts, "spmv_caller"),
        "copy_peak": {"achieved": round(copy_gbs, 1), "unit": "GB/s", "kernel": "1 GiB device copy (torch copy_)"},
    }
    sysm.close()
    del la, ua, diag, upper, lower, b, x, b_fields, x_fields, gvec, lam, xsol, r64, z64
    torch.cuda.empty_cache()
    if not args.no_extra and full:
        out["other_configs"] = other_configs(args, P, torch, dev)
    if not args.no_cpu_baseline:
        log("cpu baseline on the bench system")
        out["cpu_baseline"] = cpu_baseline(s_host, dict(
            w_levels=args.w_levels, coarse_omega=args.coarse_omega, pre_sweeps=args.pre_sweeps,
            post_sweeps=args.post_sweeps, omega=args.omega))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
