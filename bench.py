"""Benchmark: FAS solves of the nonlinear heterogeneous diffusion problem on
one MI355X.

A step is one complete FP64 FAS-Newton solve (x0 = 0 to relative residual
1e-8) of the 60x220x85 workload (1,122,000 cells, 4 levels of 4x4x4
aggregates, 3 local eigenvectors), with the problem data already resident in
device memory.  Setup (hierarchy construction) is timed separately.  Prints
one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FAS solves/s and cell-updates/s at rel. residual 1e-8; p50/p99 solve latency"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c1", "c2"])
    ap.add_argument("--seed", type=int, default=0, help="seed of the synthetic fields (the workload is seed 0)")
    ap.add_argument("--lin-rtol", type=float, default=1e-5)
    ap.add_argument("--lin-rtol-coarse", type=float, default=1e-2, help="<= 0: same as --lin-rtol")
    ap.add_argument("--lin-target", type=float, default=0.03, help="level-0 inexact-Newton forcing, 0 = off")
    ap.add_argument("--lin-max-it-coarse", type=int, default=10,
                    help="iteration limit of each coarse-level linear solve, PCG and its BiCGStab "
                         "fallback together (<= 0: same as level 0)")
    ap.add_argument("--newton-krylov", default="pcg", choices=["pcg", "bicgstab"],
                    help="pcg: PCG first with BiCGStab fallback on Newton systems")
    ap.add_argument("--coarsest-atol", type=float, default=1e-10,
                    help="absolute floor of the coarsest level's convergence test (Section 4: 1e-10); "
                         "the outer stop stays relative")
    ap.add_argument("--amg-reuse", type=int, default=-1,
                    help="linearisations that may reuse AMG values while the Krylov count stays low "
                         "(0 = off, < 0 = no limit)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparators", action="store_true")
    return ap.parse_args()


def percentile(v, q):
    v = sorted(v)
    if not v:
        return float("nan")
    k = (len(v) - 1) * q
    f, c = math.floor(k), math.ceil(k)
    return v[f] + (v[c] - v[f]) * (k - f)


def copy_rate(torch, nbytes: int = 1 << 30, reps: int = 5) -> dict:
    """Device-to-device copy of `nbytes` (larger than the 256 MB last-level
    cache) with torch's elementwise copy kernel: the measured HBM rate, and
    the kernel of known size that calibrates the FETCH_SIZE / WRITE_SIZE
    counters."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return {"bytes_read": nbytes, "bytes_written": nbytes, "avg_us": 1000.0 * ms,
            "GBps": 2.0 * nbytes / (ms * 1e-3) / 1e9}


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE /
    WRITE_SIZE counter summary of this workload (each counter scaled by
    what it reads for a 1 GiB copy), or None when there is no entry or the
    kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_c2_60x220x85.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    src = b"".join(open(os.path.join(ROOT, f), "rb").read() for f in t["sources"])
    if hashlib.sha256(src).hexdigest() != t["sources_sha256"] or kernel not in t["kernels"]:
        return None
    return t["kernels"][kernel]["bytes_per_launch"]


def cpu_baseline(n_full: int, vcycles_full: float) -> dict:
    """The CPU FP64 oracle timed on a bounded sample of the workload: the
    same recipe (log-normal top layers, channelised bottom layers, column
    wells, p = 0 on y = 0, kappa = exp(p), 4x4x4 aggregates, m = 3) on a
    16x32x16-cell grid, FAS-Newton with exact sparse solves to rtol 1e-8.
    Its cell-updates/s are converted to solves/s of the full workload with
    the GPU's V-cycle count and a cost linear in the number of cells."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from problems import c2_problem
    from oracle.coarsen import build_hierarchy
    from oracle.solvers import Opts, fas_solve
    from oracle.fv import linear_pressure
    shape = (16, 32, 16)
    # well rate of the sample by the workload's own rule: max |p| = 0.5 for kappa = 1
    p1 = linear_pressure(c2_problem(shape=shape, top_layers=7, permute=False, rate=1.0))
    sample = c2_problem(shape=shape, top_layers=7, permute=False, rate=0.5 / float(np.abs(p1).max()))
    t0 = time.perf_counter()
    h = build_hierarchy(sample, n_levels=3)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    x, st = fas_solve(h, Opts(newton=True, rtol=1e-8, atol=0.0, cap_c=sample.dp_cap_c))
    t_solve = time.perf_counter() - t0
    cu = sample.mesh.n_cells * st.iterations / t_solve
    blas = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    return {"value": cu / (n_full * vcycles_full), "unit": "solves/s", "cores": int(blas),
            "kind": "oracle",
            "sample": f"oracle FAS-Newton (exact sparse solves) on a 16x32x16 instance of the same recipe "
                      f"({sample.mesh.n_cells} cells, 3 levels): {st.iterations} V-cycles in {t_solve:.2f} s "
                      f"(setup {t_setup:.2f} s) = {cu:.4g} cell-updates/s, scaled by cells x V-cycles of the "
                      f"full workload; BLAS threads {blas} of {os.cpu_count()} host cores, SuperLU single-threaded",
            "cell_updates_per_s": cu, "converged": bool(st.converged)}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2005_01275_amd as pk
    from problems import c1_problem, c2_problem

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    copy = copy_rate(torch)
    prob = c2_problem(seed=args.seed) if args.workload == "c2" else c1_problem(seed=args.seed)
    n_cells = prob.mesh.n_cells
    stream = torch.cuda.current_stream()

    t0 = time.perf_counter()
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0

    cprob, keep = H._problem(prob, device=True)
    p = torch.zeros(n_cells, dtype=torch.float64, device="cuda")
    s = torch.zeros(prob.mesh.n_faces, dtype=torch.float64, device="cuda")
    cap = math.log(prob.dp_cap_c) / prob.alpha
    opts = pk.SolveOpts(smoother=pk.SPFAS_NEWTON, rtol=1e-8, atol=0.0, max_it=50, lin_rtol=args.lin_rtol,
                        lin_max_it=400, dp_cap=cap, lin_rtol_coarse=args.lin_rtol_coarse,
                        lin_target=args.lin_target, newton_pcg=int(args.newton_krylov == "pcg"),
                        amg_reuse=args.amg_reuse, lin_max_it_coarse=args.lin_max_it_coarse,
                        coarsest_atol=args.coarsest_atol)

    def solve():
        return H.fas_solve(prob, opts, device=True, cprob=cprob, out=(p, s), stream=stream.cuda_stream)

    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    lat, vcycles, lin = [], [], []
    H.profile_enable(True)
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        _, _, st = solve()
        lat.append(time.perf_counter() - a)
        vcycles.append(st["iterations"])
        lin.append(st["lin_iters"])
        assert st["converged"], st
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = H.profile_read()
    H.profile_enable(False)
    solves_per_s = args.steps / elapsed
    cell_updates = n_cells * sum(vcycles) / elapsed
    # dominant instrumented kernel: largest summed event time over the timed region
    dom = max(prof, key=lambda k: prof[k][1])
    nl, ms, by = prof[dom]
    achieved = (by / nl) / (ms / nl * 1e-3) / 1e9 if nl and ms > 0 else 0.0
    traffic = measured_traffic(dom) if args.workload == "c2" and args.seed == 0 else None
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                "frac": achieved / 8000.0, "traffic": traffic, "traffic_unit": "HBM bytes per launch", "launches": nl,
                "avg_us": 1000.0 * ms / max(nl, 1), "algo_bytes_per_launch": by / max(nl, 1),
                "frac_of_measured_copy": achieved / copy["GBps"]}
    kernels = {k: {"launches": v[0], "total_ms": v[1], "avg_us": 1000.0 * v[1] / max(v[0], 1),
                   "algo_GBps": (v[2] / v[1] * 1e-6) if v[1] > 0 else 0.0} for k, v in prof.items()}

    out = {
        "metric": METRIC,
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": prob.name + " FAS-Newton, 4 levels of 4x4x4 aggregates, m=3, rtol 1e-8",
                   "cells": n_cells, "levels": prob.n_levels, "smoother": "newton",
                   "lin_rtol": args.lin_rtol, "lin_rtol_coarse": args.lin_rtol_coarse or args.lin_rtol,
                   "lin_target": args.lin_target, "newton_krylov": args.newton_krylov, "amg_reuse": args.amg_reuse,
                   "lin_max_it_coarse": args.lin_max_it_coarse},
        "cell_updates_per_s": cell_updates,
        "latency_ms_p50": 1000.0 * percentile(lat, 0.5),
        "latency_ms_p99": 1000.0 * percentile(lat, 0.99),
        "vcycles": vcycles,
        "krylov_iters": lin,
        "setup_s": setup_s,
        "roofline": roofline,
        "kernels": kernels,
        "copy_1GiB": copy,
    }

    if not args.no_comparators:
        comp = {}
        for name, fn, sm in (("newton", H.newton_solve, pk.SPFAS_NEWTON), ("picard", H.picard_solve, pk.SPFAS_PICARD)):
            o = pk.SolveOpts(smoother=sm, rtol=1e-8, atol=0.0, max_it=200, lin_rtol=args.lin_rtol, lin_max_it=400,
                             dp_cap=cap, lin_target=args.lin_target, newton_pcg=int(args.newton_krylov == "pcg"),
                             amg_reuse=args.amg_reuse, lin_max_it_coarse=args.lin_max_it_coarse)
            torch.cuda.synchronize()
            a = time.perf_counter()
            _, _, st = fn(prob, o, device=True, cprob=cprob, out=(p, s), stream=stream.cuda_stream)
            torch.cuda.synchronize()
            comp[name] = {"time_s": time.perf_counter() - a, "iterations": st["iterations"],
                          "converged": st["converged"], "krylov_iters": st["lin_iters"]}
        out["gpu_single_level"] = comp
        # nonlinear cascadic multigrid (Newton smoothing): every level is solved
        # to its own tolerance, so the coarse linear solves go to 1e-6 without
        # an iteration limit (the FAS coarse options leave level 2 unconverged)
        o = pk.SolveOpts(smoother=pk.SPFAS_NEWTON, rtol=1e-8, atol=0.0, max_it=200, lin_rtol=args.lin_rtol,
                         lin_max_it=400, dp_cap=cap, lin_rtol_coarse=1e-6, lin_target=args.lin_target,
                         newton_pcg=int(args.newton_krylov == "pcg"), amg_reuse=args.amg_reuse,
                         lin_max_it_coarse=0)
        torch.cuda.synchronize()
        a = time.perf_counter()
        try:
            _, _, st = H.cascadic_solve(prob, o, device=True, cprob=cprob, out=(p, s), stream=stream.cuda_stream)
            torch.cuda.synchronize()
            out["gpu_cascadic"] = {"time_s": time.perf_counter() - a, "level_steps": st["level_steps"],
                                   "converged": st["converged"], "krylov_iters": st["lin_iters"]}
        except pk.SpfasError as e:   # a comparator's failure is reported, not fatal
            out["gpu_cascadic"] = {"error": str(e)}

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(n_cells, float(np.mean(vcycles)))

    print(json.dumps(out))


if __name__ == "__main__":
    main()
