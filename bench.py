#!/usr/bin/env python3
"""Benchmark: coupled solve time to 1e-8 relative residual on one MI355X.

Workload: the pressure-based coupled (p, Ux, Uy, Uz) 4x4 system on a
100^3 jittered, randomly renumbered hex mesh (1,000,000 cells, 2,970,000
internal faces; seeded synthetic input).  One step = the whole hot path on
resident device data: LDU -> block-CSR value conversion, AMG setup (FP32
hierarchy, FP64 block inverses and coarse solve) and the mixed-precision
AMG-BiCGStab solve to ||b - A x|| / ||b|| <= 1e-8 from x0 = 0.

Also reported: the plain FP64 GPU path on the same system (mixed vs FP64),
the FP64 block-SpMV kernel against the HBM roofline, and the CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0
# HBM bytes per launch of the FP64 SpMV on the internal numbering of the
# 100x100x100 p-U system, from FETCH_SIZE and WRITE_SIZE counter runs scaled
# by the readings of a 1 GiB copy kernel (factors 2.0 and 1.0):
# profiles/block_spmv_fp64_pu1M_hbm_counters.md
SPMV_TRAFFIC_PU1M = 1133719389


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mesh", type=int, nargs=3, default=[100, 100, 100])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, nargs=3, default=[80, 80, 80])
    ap.add_argument("--spmv-reps", type=int, default=50)
    ap.add_argument("--smoother", choices=["dilu", "bjacobi"], default="bjacobi")
    ap.add_argument("--dilu-levels", type=int, default=2)
    ap.add_argument("--sweeps", type=int, default=2)
    ap.add_argument("--omega", type=float, default=0.9)
    ap.add_argument("--coarse-max", type=int, default=16)
    ap.add_argument("--passes", type=int, default=2)
    ap.add_argument("--solver", choices=["bicgstab", "fgmres"], default="bicgstab")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--row-split", type=int, default=0,
                    help="threads per scalar row on levels under 65,536 block rows (0 = automatic)")
    ap.add_argument("--spmv-only", action="store_true",
                    help="only the FP64 block SpMV (both numberings) and a 1 GiB copy, for counter runs")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spmv_bytes(N, nnzb, n, s=8):
    """Algorithmic bytes of one block SpMV: values + column indices + row
    pointers + x read once + y written once."""
    return nnzb * (n * n * s + 4) + (N + 1) * 4 + 2 * N * n * s


def cpu_baseline(shape):
    import oracle as O
    from workloads import pressure_velocity
    s = pressure_velocity(*shape, seed=0)
    A = O.from_system(s)
    t0 = time.perf_counter()
    amg = O.AMG(A, coarse_max=16, passes=2, smoother=O.SMOOTH_BJACOBI, nu1=2, nu2=2, omega=0.9)
    x, st = O.bicgstab(A, s["b"], prec=O.PREC_AMG, amg=amg, tol=1e-8, maxit=500)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": dt * 1e3 * (1_000_000 / s["N"]),
        "unit": "ms per 1M-cell solve (scaled)",
        "cores": threads,
        "kind": "oracle",
        "sample": "oracle AMG(block-Jacobi V(2,2), omega 0.9)-BiCGStab FP64 setup+solve to 1e-8 on the same "
                  "pressure-velocity construction at %dx%dx%d (%d cells, %d iterations, %.2f s), "
                  "scaled linearly to 1M cells" % (*shape, s["N"], st["iterations"], dt),
        "measured_s": dt,
    }


def spmv_only(args, P, torch, dev, sysm, N, n, nnzb, la, ua, diag, upper, lower):
    """FP64 block SpMV launches on both numberings plus a plain 1 GiB copy
    (the calibration kernel of the HBM byte counters)."""
    import ctypes as C
    L = P.lib()
    xv = torch.randn(N * n, dtype=torch.float64, device=dev)
    yv = torch.empty_like(xv)
    sysm.setup(P.default_options(precision=P.PRECISION_MIXED))
    order = sysm.get_level(0)["order"].long()
    pos = torch.empty_like(order)
    pos[order] = torch.arange(N, device=dev)
    sys2 = P.System(N, n, pos[la.long()].int(), pos[ua.long()].int(), diag[order], upper, lower)
    res = {}
    for name, system in (("caller", sysm), ("internal", sys2)):
        for _ in range(args.spmv_reps):
            L.cbs_spmv(system.h, C.c_void_p(xv.data_ptr()), C.c_void_p(yv.data_ptr()), 0)
        torch.cuda.synchronize()
        res[name] = args.spmv_reps
    a = torch.empty(1 << 27, dtype=torch.float64, device=dev)     # 1 GiB
    a.fill_(1.0)
    bcopy = torch.empty_like(a)
    for _ in range(3):
        bcopy.copy_(a)
    torch.cuda.synchronize()
    sys2.close()
    print(json.dumps({"spmv_launches_per_numbering": args.spmv_reps,
                      "algorithmic_bytes_per_spmv": int(spmv_bytes(N, nnzb, n)),
                      "copy_bytes_read": int(a.numel() * 8), "copy_bytes_written": int(a.numel() * 8)}))


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this solver path runs on a single MI355X "
              "(multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2403_07882_amd as P
    from workloads import pressure_velocity

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
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
    del s
    sysm = P.System(N, n, la, ua, diag, upper, lower)
    nnzb = sysm.info()["nnzb"]
    if args.spmv_only:
        spmv_only(args, P, torch, dev, sysm, N, n, nnzb, la, ua, diag, upper, lower)
        return
    common = dict(solver=P.SOLVER_BICGSTAB if args.solver == "bicgstab" else P.SOLVER_FGMRES,
                  precond=P.PREC_AMG, tol=1e-8, max_iter=500,
                  smoother=P.SMOOTH_DILU if args.smoother == "dilu" else P.SMOOTH_BJACOBI,
                  dilu_levels=args.dilu_levels, pre_sweeps=args.sweeps, post_sweeps=args.sweeps,
                  omega=args.omega, coarse_max=args.coarse_max, match_passes=args.passes,
                  row_split=args.row_split)
    opt_mixed = P.default_options(precision=P.PRECISION_MIXED, **common)
    opt_fp64 = P.default_options(precision=P.PRECISION_FP64, **common)

    L = P.lib()
    import ctypes as C
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def step(opt):
        # a1 pack -> a3 values -> setup -> solve -> a1 unpack
        L.cbs_pack_fields(N, n, C.c_void_p(b_fields.data_ptr()), C.c_void_p(b.data_ptr()), stream)
        sysm.update_values(diag, upper, lower)
        sysm.setup(opt)
        x.zero_()
        st = P.Stats()
        rc = L.cbs_solve(sysm.h, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), C.byref(st))
        if rc < 0:
            raise P.CbsError(rc, "cbs_solve")
        L.cbs_unpack_fields(N, n, C.c_void_p(x.data_ptr()), C.c_void_p(x_fields.data_ptr()), stream)
        return x, st.as_dict(), rc

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        _, st, _ = step(opt_mixed)
    torch.cuda.synchronize()
    log("timing %d steps (mixed)" % args.steps)
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        xs, st, _ = step(opt_mixed)
        stats.append(st)
    torch.cuda.synchronize()
    t_mixed = (time.perf_counter() - t0) / args.steps * 1e3
    if st["precision_fallback"]:
        log("WARNING: the mixed-precision hierarchy escalated to FP64")
    log("mixed: %.2f ms/step, iterations %d, relres %.3e, setup %.2f ms, solve %.2f ms"
        % (t_mixed, st["iterations"], st["rel_res_true"], st["t_setup_ms"], st["t_solve_ms"]))

    # plain FP64 GPU path on the same system
    t_fp64, st64 = float("nan"), {"iterations": -1}
    if not args.skip_fp64:
        for _ in range(max(1, args.warmup // 2)):
            step(opt_fp64)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k64 = max(1, args.steps // 2)
        for _ in range(k64):
            _, st64, _ = step(opt_fp64)
        torch.cuda.synchronize()
        t_fp64 = (time.perf_counter() - t0) / k64 * 1e3
        log("fp64: %.2f ms/step, iterations %d" % (t_fp64, st64["iterations"]))

    # dominant bandwidth kernel: FP64 block SpMV, timed with events on its
    # stream (torch's current stream, which the library was given).

    def time_spmv(system):
        xv = torch.randn(N * n, dtype=torch.float64, device=dev)
        yv = torch.empty_like(xv)
        for _ in range(5):
            L.cbs_spmv(system.h, C.c_void_p(xv.data_ptr()), C.c_void_p(yv.data_ptr()), 0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.spmv_reps):
            L.cbs_spmv(system.h, C.c_void_p(xv.data_ptr()), C.c_void_p(yv.data_ptr()), 0)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.spmv_reps

    byts = spmv_bytes(N, nnzb, n)
    spmv_user_ms = time_spmv(sysm)
    gbs_user = byts / (spmv_user_ms * 1e-3) / 1e9
    log("spmv fp64 (caller numbering): %.1f us, %.0f GB/s" % (spmv_user_ms * 1e3, gbs_user))
    # the same kernel on the solver's internal (aggregation-tree) numbering:
    # a system built from the renumbered LDU arrays
    sysm.setup(opt_mixed)
    order = sysm.get_level(0)["order"].long()
    pos = torch.empty_like(order)
    pos[order] = torch.arange(N, device=dev)
    la2 = pos[la.long()].int()
    ua2 = pos[ua.long()].int()
    sys2 = P.System(N, n, la2, ua2, diag[order], upper, lower)
    spmv_ms = time_spmv(sys2)
    sys2.close()
    del la2, ua2, order, pos
    gbs = byts / (spmv_ms * 1e-3) / 1e9
    log("spmv fp64 (internal numbering): %.1f us, %.0f GB/s" % (spmv_ms * 1e3, gbs))

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
                               "randomly renumbered (N=%d, F=%d, nnzb=%d); mixed AMG-BiCGStab to 1e-8"
                               % (nx, ny, nz, N, F, nnzb),
                   "step": "pack fields + update_values + setup + solve + unpack fields",
                   "solver": args.solver, "smoother": args.smoother, "dilu_levels": args.dilu_levels,
                   "sweeps": args.sweeps, "omega": args.omega, "coarse_max": args.coarse_max,
                   "match_passes": args.passes, "row_split": args.row_split},
        "iterations": st["iterations"],
        "precision_fallback": st["precision_fallback"],
        "rel_res_true": st["rel_res_true"],
        "levels": st["levels"],
        "op_complexity": round(st["op_complexity"], 3),
        "setup_ms": round(st["t_setup_ms"], 3),
        "solve_ms": round(st["t_solve_ms"], 3),
        "convert_ms": round(st["t_convert_ms"], 3),
        "fp64_ms_per_step": round(t_fp64, 3),
        "fp64_iterations": st64["iterations"],
        "mixed_vs_fp64_speedup": round(t_fp64 / t_mixed, 3) if t_fp64 == t_fp64 else None,
        "roofline": {"bound": "hbm", "kernel": "block SpMV FP64 (k_rows mode 0, n=4), internal numbering",
                     "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "traffic": SPMV_TRAFFIC_PU1M if (nx, ny, nz) == (100, 100, 100) else None,
                     "avg_launch_us": round(spmv_ms * 1e3, 2), "algorithmic_bytes": int(byts)},
        "spmv_caller_numbering": {"achieved_gbs": round(gbs_user, 1), "avg_launch_us": round(spmv_user_ms * 1e3, 2),
                                  "frac": round(gbs_user / HBM_PEAK_GBS, 4)},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline on %s" % (args.cpu_sample,))
        out["cpu_baseline"] = cpu_baseline(tuple(args.cpu_sample))
    print(json.dumps(out), flush=True)
    sysm.close()


if __name__ == "__main__":
    main()
