"""Benchmark: FAS solves of the nonlinear heterogeneous diffusion problem on
one MI355X.

A step is one complete FP64 FAS-Newton solve (x0 = 0 to relative residual
1e-8) of the 60x220x85 workload (1,122,000 cells, 4 levels of 4x4x4
aggregates, 3 local eigenvectors), with the problem data already resident in
device memory.  Setup (hierarchy construction) is timed separately.  Prints
one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Beside the headline the line carries: the same solves in mixed precision
(FP32 level-0 linear solves inside the FP64 residual and update), the GPU
single-level Newton/Picard and cascadic comparators (medians after a
warm-up), seeds 1-4 of the workload recipe, the 32x32 workload (C1: us per
V-cycle), the unstructured configuration (Voronoi mesh, greedy aggregates,
eigenvector counts by threshold, mixed precision), a served stream (Poisson arrivals over several models through the
native serving runtime, p50/p99 latency) and a batched setup-and-solve of
independent problems with an autotuned number of solves in flight, and the
CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import dataclasses
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
    ap.add_argument("--no-extras", action="store_true",
                    help="headline only: no mixed-precision, seeds, C1, served or batched legs")
    ap.add_argument("--served-requests", type=int, default=200)
    ap.add_argument("--batch-problems", type=int, default=24)
    ap.add_argument("--c4", action="store_true",
                    help="also run the batched configuration at its full size (512 instances, about 1.0e8 cells; "
                         "several minutes)")
    return ap.parse_args()


_T0 = time.perf_counter()


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


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
    20x40x16-cell grid, FAS-Newton with exact sparse solves to rtol 1e-8.
    Its cell-updates/s are converted to solves/s of the full workload with
    the GPU's V-cycle count and a cost linear in the number of cells."""
    import numpy as np
    from threadpoolctl import threadpool_info
    from problems import c2_problem
    from oracle.coarsen import build_hierarchy
    from oracle.solvers import Opts, fas_solve
    from oracle.fv import linear_pressure
    shape = (20, 40, 16)
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
            "sample": f"oracle FAS-Newton (exact sparse solves) on a 20x40x16 instance of the same recipe "
                      f"({sample.mesh.n_cells} cells, 3 levels): {st.iterations} V-cycles in {t_solve:.2f} s "
                      f"(setup {t_setup:.2f} s) = {cu:.4g} cell-updates/s; the value is extrapolated to the "
                      f"1,122,000-cell workload linearly in cells x V-cycles (the oracle's sparse direct solves "
                      f"grow faster than that, so the extrapolation favours the CPU); BLAS threads {blas} of "
                      f"{os.cpu_count()} host cores, SuperLU single-threaded",
            "extrapolated": True, "sample_seconds": t_solve + t_setup,
            "cell_updates_per_s": cu, "converged": bool(st.converged)}


def timed_solves(torch, fn, n, warmup=1):
    """Runs fn() warmup + n times; returns (ms per call list, last stats)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ms, st = [], None
    for _ in range(n):
        a = time.perf_counter()
        _, _, st = fn()
        torch.cuda.synchronize()
        ms.append(1000.0 * (time.perf_counter() - a))
    return ms, st


def seeds_leg(torch, pk, c2_problem, opts, seeds=(1, 2, 3, 4), steps=2):
    """The same workload recipe with other seeds: ms per solve (median of
    `steps` after a warm-up), V-cycles, converged."""
    out = {}
    for sd in seeds:
        log(f"seed {sd}: problem and hierarchy")
        prob = c2_problem(seed=sd)
        H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
        cprob, keep = H._problem(prob, device=True)
        try:
            ms, st = timed_solves(torch, lambda: H.fas_solve(prob, opts, device=True, cprob=cprob), steps)
            out[str(sd)] = {"ms": float(percentile(ms, 0.5)), "vcycles": st["iterations"], "converged": st["converged"]}
        except pk.SpfasError as e:
            out[str(sd)] = {"error": str(e)}
        H.close()
        del H, keep
    return out


def c1_leg(torch, pk, c1_problem, steps=200):
    """The 32x32 workload: latency- and launch-bound, no HBM roofline."""
    log("c1: 32x32 solves")
    prob = c1_problem()
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    cprob, keep = H._problem(prob, device=True)
    o = pk.SolveOpts(smoother=pk.SPFAS_NEWTON, rtol=1e-8, atol=0.0, max_it=50, lin_rtol=1e-8, lin_max_it=400,
                     dp_cap=math.log(prob.dp_cap_c) / prob.alpha, newton_pcg=1, coarsest_atol=1e-10)
    ms, st = timed_solves(torch, lambda: H.fas_solve(prob, o, device=True, cprob=cprob), steps, warmup=10)
    t = sum(ms) / 1000.0
    H.close()
    return {"workload": prob.name + " FAS-Newton, 2 levels of 4x4 aggregates, m=2, rtol 1e-8",
            "solves_per_s": steps / t, "ms_per_solve_p50": percentile(ms, 0.5), "ms_per_solve_p99": percentile(ms, 0.99),
            "vcycles": st["iterations"], "us_per_vcycle": 1000.0 * percentile(ms, 0.5) / max(st["iterations"], 1),
            "krylov_iters": st["lin_iters"], "cell_updates_per_s": prob.mesh.n_cells * st["iterations"] * steps / t}


def unstructured_leg(torch, pk, steps=3):
    """The unstructured configuration at its full size: the bounded Voronoi
    mesh of 2,000,000 seeded points, ln k = 3G with correlation length 0.01,
    kappa = exp(2p), greedy aggregates of about 64 cells on 2 levels,
    eigenvectors per aggregate by the threshold 0.1 clamped to [2, 6],
    mixed-precision FAS-Newton to rtol 1e-8 beside the FP64 solve on the same
    hierarchy (which the parity tests tie to the oracle); the source rate is
    the oracle-calibrated one (alpha max |p_lin| = 0.5)."""
    import numpy as np
    from problems.grids import c3_problem
    from paper_2005_01275_amd import _native as N
    log("unstructured: Voronoi mesh of 2,000,000 points")
    t0 = time.perf_counter()
    prob = c3_problem()
    t_mesh = time.perf_counter() - t0
    log("unstructured: hierarchy (greedy aggregates, threshold counts)")
    t0 = time.perf_counter()
    H = pk.Hierarchy(prob.mesh, prob.n_levels, m=prob.m, agg_kind=N.SPFAS_AGG_GREEDY, greedy_size=prob.greedy_size,
                     eig_threshold=prob.eig_threshold, m_min=prob.m_min, greedy_size_coarse=prob.greedy_size_coarse)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    counts = []
    for l in range(prob.n_levels - 1):
        n_agg = H.level_sizes(l + 1)[0]
        counts.append(np.bincount(H.level_operator(l, N.SPFAS_OP_MCOUNT, n_agg).astype(int), minlength=7)[1:].tolist())
    cprob, keep = H._problem(prob, device=True)
    base = dict(smoother=pk.SPFAS_NEWTON, rtol=1e-8, atol=0.0, max_it=50, lin_rtol=1e-5, lin_max_it=400,
                lin_rtol_coarse=1e-2, lin_target=0.03, newton_pcg=1, amg_reuse=-1, lin_max_it_coarse=10,
                coarsest_atol=1e-10, dp_cap=math.log(prob.dp_cap_c) / prob.alpha)
    out = {"workload": "voronoi_2d_2000000, ln k = 3G, kappa = exp(2p), greedy aggregates of 64, 2 levels, "
                       "eigenvector counts by threshold 0.1 in [2, 6], FAS-Newton rtol 1e-8",
           "cells": prob.mesh.n_cells, "mesh_s": t_mesh, "setup_s": t_setup, "eig_counts_per_level": counts}
    res = {}
    for name, prec in (("mixed", pk.SPFAS_PREC_MIXED), ("fp64", pk.SPFAS_PREC_FP64)):
        o = pk.SolveOpts(precision=prec, **base)
        log(f"unstructured: {name} solves")
        try:
            ms, st = timed_solves(torch, lambda: H.fas_solve(prob, o, device=True, cprob=cprob), steps)
            p, s, _ = H.fas_solve(prob, o)
            res[name] = p
            out[name] = {"ms_per_solve_p50": percentile(ms, 0.5), "solves_per_s": 1000.0 / percentile(ms, 0.5),
                         "vcycles": st["iterations"], "krylov_iters": st["lin_iters"],
                         "refine_steps": st["refine_steps"], "converged": st["converged"]}
        except pk.SpfasError as e:
            out[name] = {"error": str(e)}
    if "mixed" in res and "fp64" in res:
        out["mixed_vs_fp64_max_rel_err"] = float(np.abs(res["mixed"] - res["fp64"]).max() /
                                                 np.abs(res["fp64"]).max())
    H.close()
    return out


def served_leg(pk, n_requests, seed=7, n_models=10, n_slots=6):
    """A served stream through the native runtime: n_models models of
    random size (2-D/3-D, 32^2..64^3 cells, their own k fields), requests
    with their own source scale arriving as a Poisson process at 0.7 of the
    closed-loop capacity measured first, mixed-precision FAS-Newton to rtol
    1e-8.  Beside it, the same requests solved one at a time in FP64 on
    cached hierarchies."""
    import dataclasses
    import threading
    import numpy as np
    from problems.grids import served_problem
    from paper_2005_01275_amd.serve import Server, ServerError
    rng = np.random.default_rng(seed)
    log("served: models")
    models = [served_problem(1000 + i) for i in range(n_models)]

    def opts(prec):
        return pk.SolveOpts(smoother=pk.SPFAS_NEWTON, rtol=1e-8, atol=0.0, max_it=60, lin_rtol=1e-5, lin_max_it=400,
                            lin_rtol_coarse=1e-2, lin_target=0.03, newton_pcg=1, amg_reuse=-1, lin_max_it_coarse=10,
                            coarsest_atol=1e-10, dp_cap=math.log(5.0), precision=prec)

    with Server(n_slots=n_slots) as S:
        ids = [S.add_model(m.mesh, m.n_levels, m.box, m.m) for m in models]
        # build the cached hierarchies; each model's source is scaled so that
        # the kappa = 1 (alpha = 0, linear) pressure has max |p| = 0.5, the
        # rule that keeps exp(p) problems solvable (a strong sink can leave
        # them without a root)
        log("served: building the cached hierarchies, source scales from linear solves")
        lin = [S.submit(ids[i], dataclasses.replace(m, alpha=0.0), opts(pk.SPFAS_PREC_FP64))
               for i, m in enumerate(models)]
        for i, t in enumerate(lin):
            pl = S.wait(t)[0]
            models[i] = dataclasses.replace(models[i], source=models[i].source * (0.5 / float(np.abs(pl).max())))
        reqs = []
        for r in range(n_requests):
            i = int(rng.integers(n_models))
            # per request: 0.3 .. 0.6 of the scaled source (stronger random
            # sinks leave some of these fields without a root)
            reqs.append((i, dataclasses.replace(models[i], source=models[i].source * float(0.3 + 0.3 * rng.random()))))
        # closed-loop capacity on one burst
        t0 = time.perf_counter()
        burst = [S.submit(ids[i], pr, opts(pk.SPFAS_PREC_MIXED)) for i, pr in reqs[:2 * n_slots]]
        for t in burst:
            S.wait(t)
        capacity = len(burst) / (time.perf_counter() - t0)

        def stream(rate, rq):
            """Poisson arrivals at `rate` of the requests rq: latencies
            (submission to completion), converged and failed counts, span."""
            arrivals = np.cumsum(rng.exponential(1.0 / rate, len(rq)))
            tickets = [None] * len(rq)
            start = time.perf_counter()

            def feeder():
                for k, (i, pr) in enumerate(rq):
                    d = arrivals[k] - (time.perf_counter() - start)
                    if d > 0:
                        time.sleep(d)
                    tickets[k] = S.submit(ids[i], pr, opts(pk.SPFAS_PREC_MIXED))

            th = threading.Thread(target=feeder)
            th.start()
            th.join()
            lat, ok, fail = [], 0, 0
            for t in tickets:
                try:
                    _, _, st, info = S.wait(t)
                    lat.append(info["total_ms"])
                    ok += int(st["converged"])
                except ServerError:
                    fail += 1
            return lat, ok, fail, time.perf_counter() - start

        rate = 0.7 * capacity
        log(f"served: capacity {capacity:.1f} solves/s, Poisson stream at {rate:.1f}/s")
        lat, ok, fail, span = stream(rate, reqs)
        cnt = S.counters()
        # the offered load swept around it (fewer requests per point)
        sweep = []
        for frac in (0.3, 0.5, 0.9, 1.1):
            log(f"served: rate sweep at {frac:.1f} x capacity")
            l2, ok2, f2, sp2 = stream(frac * capacity, reqs[:n_requests // 3])
            sweep.append({"fraction_of_capacity": frac, "arrival_rate": frac * capacity,
                          "solves_per_s": len(l2) / sp2, "latency_ms_p50": percentile(l2, 0.5),
                          "latency_ms_p99": percentile(l2, 0.99), "converged": ok2, "failed": f2})
    # the same requests one at a time, FP64, hierarchies cached
    log("served: the same requests one at a time in FP64")
    Hs = {}
    seq = []
    for i, pr in reqs:
        if i not in Hs:
            m = models[i]
            Hs[i] = pk.Hierarchy(m.mesh, m.n_levels, m.box, m.m)
            Hs[i].fas_solve(pr, opts(pk.SPFAS_PREC_FP64))
        a = time.perf_counter()
        Hs[i].fas_solve(pr, opts(pk.SPFAS_PREC_FP64))
        seq.append(1000.0 * (time.perf_counter() - a))
    for H in Hs.values():
        H.close()
    return {"workload": f"{n_requests} requests over {n_models} models (2-D/3-D, 32^2..64^3 cells log-uniform, "
                        f"ln k sigma 2), Poisson arrivals at 0.7 x the measured capacity, mixed-precision FAS-Newton "
                        f"rtol 1e-8, {n_slots} solves in flight",
            "cells": [m.mesh.n_cells for m in models], "capacity_solves_per_s": capacity, "arrival_rate": rate,
            "solves_per_s": len(lat) / span, "latency_ms_p50": percentile(lat, 0.5),
            "latency_ms_p99": percentile(lat, 0.99), "converged": ok, "failed": fail, "counters": cnt,
            "rate_sweep": sweep,
            "fp64_one_at_a_time": {"solves_per_s": 1000.0 * len(seq) / sum(seq),
                                   "service_ms_p50": percentile(seq, 0.5), "service_ms_p99": percentile(seq, 0.99)}}


def batched_leg(pk, n_problems, seed=11):
    """Independent problems (3-D cubes of 16^3..32^3 cells, their own k
    fields) set up and solved together through the native runtime, the
    number of solves in flight chosen by the autotuner on a sample; against
    the same problems one after the other (one in flight)."""
    import numpy as np
    from problems.grids import served_problem
    from paper_2005_01275_amd.batch import solve_batch, autotune_slots
    import dataclasses
    log("batched: problems")
    probs = [served_problem(seed * 1000 + i, n_min=16 ** 3, n_max=32 ** 3, dims=(3,)) for i in range(n_problems)]
    o = pk.SolveOpts(smoother=pk.SPFAS_NEWTON, rtol=1e-8, atol=0.0, max_it=60, lin_rtol=1e-5, lin_max_it=400,
                     lin_rtol_coarse=1e-2, lin_target=0.03, newton_pcg=1, amg_reuse=-1, lin_max_it_coarse=10,
                     coarsest_atol=1e-10, dp_cap=math.log(5.0), precision=pk.SPFAS_PREC_MIXED)
    # source scales from linear (alpha = 0) solves: max |p| = 0.25 for kappa = 1
    log("batched: source scales from linear solves")
    lin, _, _ = solve_batch([dataclasses.replace(pr, alpha=0.0) for pr in probs],
                            dataclasses.replace(o, precision=pk.SPFAS_PREC_FP64), 8)
    probs = [dataclasses.replace(pr, source=pr.source * (0.25 / float(np.abs(r[0]).max()))) for pr, r in zip(probs, lin)]
    log("batched: autotuning the solves in flight on 4 problems")
    best, table = autotune_slots(probs[:4], o, candidates=(1, 4, 8))
    log(f"batched: {best} in flight ({table}); the whole batch")
    res, sec, cnt = solve_batch(probs, o, best)
    log("batched: the whole batch one in flight")
    res1, sec1, _ = solve_batch(probs, o, 1)
    same = all(np.array_equal(a[0], b[0]) for a, b in zip(res, res1))
    cells = sum(p.mesh.n_cells for p in probs)
    return {"workload": f"{n_problems} independent 3-D problems of 16^3..32^3 cells ({cells} cells), setup and "
                        f"mixed-precision FAS-Newton solve each",
            "autotune_slots_s": {str(k): v for k, v in table.items()}, "slots": best,
            "problems_per_s": n_problems / sec, "seconds": sec, "one_in_flight_seconds": sec1,
            "speedup_vs_one_in_flight": sec1 / sec, "results_identical_to_one_in_flight": bool(same),
            "converged": sum(int(r[2]["converged"]) for r in res), "counters": cnt}


def c4_leg(pk, n_problems=512, slots=4, window=64):
    """The batched configuration at its full size: 512 independent boxes of
    16..96 cells per edge (about 1.0e8 cells), each with its own k field and
    box aggregates of 4..8 cells per edge.  The instances stream through the
    native runtime: each is generated on the host, registered, solved
    linearly (alpha = 0) to fix its source scale (max |p| = 0.25), then
    solved by mixed-precision FAS-Newton to rtol 1e-8; at most `window`
    instances are in the pipeline, and cached hierarchies are evicted when
    the device-memory budget is reached.  The wall time covers generation,
    every setup and both solves of every instance."""
    import collections
    import numpy as np
    from problems.grids import c4_problem
    from paper_2005_01275_amd.serve import Server, ServerError, FAS
    o = pk.SolveOpts(smoother=pk.SPFAS_NEWTON, rtol=1e-8, atol=0.0, max_it=60, lin_rtol=1e-5, lin_max_it=400,
                     lin_rtol_coarse=1e-2, lin_target=0.03, newton_pcg=1, amg_reuse=-1, lin_max_it_coarse=10,
                     coarsest_atol=1e-10, dp_cap=math.log(5.0), precision=pk.SPFAS_PREC_MIXED)
    lo = dataclasses.replace(o, precision=pk.SPFAS_PREC_FP64)
    lin_q, fas_q = collections.deque(), collections.deque()
    done, failed = [], []
    cells = 0
    t0 = time.perf_counter()
    with Server(n_slots=slots) as S:
        def finish_one():
            i, n, setup_ms, t = fas_q.popleft()
            try:
                _, _, st, info = S.wait(t)
                done.append((i, n, st["converged"], st["iterations"], setup_ms + info["setup_ms"], info["solve_ms"]))
            except ServerError as e:
                failed.append((i, str(e)))

        def scale_one():
            i, mid, pr, t = lin_q.popleft()
            try:
                p_lin, _, _, info = S.wait(t)
            except ServerError as e:
                failed.append((i, str(e)))
                return
            pr = dataclasses.replace(pr, source=pr.source * (0.25 / float(np.abs(p_lin).max())))
            fas_q.append((i, pr.mesh.n_cells, info["setup_ms"], S.submit(mid, pr, o, FAS)))

        for i in range(n_problems):
            pr = c4_problem(i)
            cells += pr.mesh.n_cells
            mid = S.add_model(pr.mesh, pr.n_levels, pr.box, pr.m)
            lin_q.append((i, mid, pr, S.submit(mid, dataclasses.replace(pr, alpha=0.0), lo, FAS)))
            while len(lin_q) > window // 2:
                scale_one()
            while len(fas_q) > window // 2:
                finish_one()
            if (i + 1) % 64 == 0:
                log(f"c4: {i + 1} instances generated and submitted, {len(done)} finished")
        while lin_q:
            scale_one()
        while fas_q:
            finish_one()
        cnt = S.counters()
    sec = time.perf_counter() - t0
    it = np.array([d[3] for d in done] or [0])
    return {"workload": f"{n_problems} independent 3-D boxes of 16..96 cells per edge ({cells} cells), ln k = 2G, "
                        "kappa = exp(p), box aggregates of 4..8 cells per edge, m = 3; linear solve for the source "
                        "scale, then mixed-precision FAS-Newton to rtol 1e-8",
            "cells": cells, "seconds": sec, "problems_per_s": n_problems / sec, "cells_per_s": cells / sec,
            "slots": slots, "converged": int(sum(d[2] for d in done)), "failed": failed[:8], "n_failed": len(failed),
            "vcycles_min_median_max": [int(it.min()), float(np.median(it)), int(it.max())],
            "setup_ms_sum": float(sum(d[4] for d in done)), "fas_solve_ms_sum": float(sum(d[5] for d in done)),
            "counters": cnt}


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
    log("workload and hierarchy")
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

    log("headline solves")
    for _ in range(args.warmup):
        solve()
    torch.cuda.synchronize()
    lat, vcycles, lin = [], [], []
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
    # the same number of solves again with HIP events around the instrumented
    # kernels (on the solver stream) for the per-kernel rooflines; the events
    # add gaps between launches, so the timed region above runs without them
    log("instrumented solves")
    H.profile_enable(True)
    torch.cuda.synchronize()
    t_prof = time.perf_counter()
    for _ in range(args.steps):
        solve()
    torch.cuda.synchronize()
    elapsed_prof = time.perf_counter() - t_prof
    prof = H.profile_read()
    H.profile_enable(False)
    solves_per_s = args.steps / elapsed
    cell_updates = n_cells * sum(vcycles) / elapsed
    # dominant instrumented kernel: largest summed event time over the
    # instrumented solves among the single kernels (the amg_tail_* entries are sums over
    # several levels' launches)
    dom = max((k for k in prof if not k.startswith("amg_tail")), key=lambda k: prof[k][1])
    nl, ms, by = prof[dom]
    achieved = (by / nl) / (ms / nl * 1e-3) / 1e9 if nl and ms > 0 else 0.0
    traffic = measured_traffic(dom) if args.workload == "c2" and args.seed == 0 else None
    roofline = {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": 8000.0, "unit": "GB/s",
                "frac": achieved / 8000.0, "traffic": traffic, "traffic_unit": "HBM bytes per launch", "launches": nl,
                "avg_us": 1000.0 * ms / max(nl, 1), "algo_bytes_per_launch": by / max(nl, 1),
                "frac_of_measured_copy": achieved / copy["GBps"]}
    kernels = {k: {"launches": v[0], "total_ms": v[1], "avg_us": 1000.0 * v[1] / max(v[0], 1),
                   "algo_GBps": (v[2] / v[1] * 1e-6) if v[1] > 0 else 0.0} for k, v in prof.items()}
    # every instrumented entry above 5 % of the instrumented solves, with its
    # roofline; the amg_tail_* entries sum the level-0 AMG's coarser levels
    # (per-launch data of a few MB, cache-resident, 3-9 us launches: latency
    # bound), the others are single finest-level kernels (HBM bound)
    rooflines = []
    for k, v in sorted(prof.items(), key=lambda kv: -kv[1][1]):
        nl_k, ms_k, by_k = v
        if not nl_k or ms_k < 0.05 * 1000.0 * elapsed_prof:
            continue
        ach = by_k / (ms_k * 1e-3) / 1e9
        rooflines.append({"kernel": k, "bound": "latency" if k.startswith("amg_tail") else "hbm", "achieved": ach,
                          "peak": 8000.0, "unit": "GB/s", "frac": ach / 8000.0,
                          "share_of_instrumented_solves": ms_k / (1000.0 * elapsed_prof), "launches": nl_k,
                          "avg_us": 1000.0 * ms_k / nl_k, "algo_bytes_per_launch": by_k / nl_k,
                          "traffic": measured_traffic(k) if args.workload == "c2" and args.seed == 0 else None})

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
                   "lin_max_it_coarse": args.lin_max_it_coarse, "coarsest_atol": args.coarsest_atol,
                   "preconditioner_storage": "level-0 classical AMG: FP16 cycle operators, FP32 cycle vectors; "
                                             "residual, Jacobian, transfers, Krylov vectors and dots FP64"},
        "cell_updates_per_s": cell_updates,
        "latency_ms_p50": 1000.0 * percentile(lat, 0.5),
        "latency_ms_p99": 1000.0 * percentile(lat, 0.99),
        "vcycles": vcycles,
        "krylov_iters": lin,
        "setup_s": setup_s,
        "roofline": roofline,
        "rooflines_above_5pct": rooflines,
        "kernels": kernels,
        "copy_1GiB": copy,
    }

    fas_ms = 1000.0 * percentile(lat, 0.5)
    out["ms_per_step_instrumented"] = 1000.0 * elapsed_prof / args.steps
    if not args.no_comparators:
        log("comparators")
        # each comparator after a warm-up, median of three runs
        comp = {}
        for name, fn, sm in (("newton", H.newton_solve, pk.SPFAS_NEWTON), ("picard", H.picard_solve, pk.SPFAS_PICARD)):
            o = pk.SolveOpts(smoother=sm, rtol=1e-8, atol=0.0, max_it=200, lin_rtol=args.lin_rtol, lin_max_it=400,
                             dp_cap=cap, lin_target=args.lin_target, newton_pcg=int(args.newton_krylov == "pcg"),
                             amg_reuse=args.amg_reuse, lin_max_it_coarse=args.lin_max_it_coarse)
            ms, st = timed_solves(torch, lambda: fn(prob, o, device=True, cprob=cprob, out=(p, s),
                                                    stream=stream.cuda_stream), 3)
            comp[name] = {"ms_median": percentile(ms, 0.5), "ms": ms, "iterations": st["iterations"],
                          "converged": st["converged"], "krylov_iters": st["lin_iters"],
                          "fas_speedup": percentile(ms, 0.5) / fas_ms}
        out["gpu_single_level"] = comp
        # nonlinear cascadic multigrid (Newton smoothing): every level is solved
        # to its own tolerance, so the coarse linear solves go to 1e-6 without
        # an iteration limit (the FAS coarse options leave level 2 unconverged)
        o = pk.SolveOpts(smoother=pk.SPFAS_NEWTON, rtol=1e-8, atol=0.0, max_it=200, lin_rtol=args.lin_rtol,
                         lin_max_it=400, dp_cap=cap, lin_rtol_coarse=1e-6, lin_target=args.lin_target,
                         newton_pcg=int(args.newton_krylov == "pcg"), amg_reuse=args.amg_reuse,
                         lin_max_it_coarse=0)
        try:
            ms, st = timed_solves(torch, lambda: H.cascadic_solve(prob, o, device=True, cprob=cprob, out=(p, s),
                                                                  stream=stream.cuda_stream), 3)
            out["gpu_cascadic"] = {"ms_median": percentile(ms, 0.5), "ms": ms, "level_steps": st["level_steps"],
                                   "converged": st["converged"], "krylov_iters": st["lin_iters"]}
        except pk.SpfasError as e:   # a comparator's failure is reported, not fatal
            out["gpu_cascadic"] = {"error": str(e)}

    if not args.no_extras:
        log("mixed precision")
        # mixed precision at equal accuracy (the FP64 residual decides the stop)
        mo = dataclasses.replace(opts, precision=pk.SPFAS_PREC_MIXED)
        ms, st = timed_solves(torch, lambda: H.fas_solve(prob, mo, device=True, cprob=cprob, out=(p, s),
                                                         stream=stream.cuda_stream), max(3, args.steps // 2))
        out["mixed"] = {"precision": "FP32 level-0 linear solves (S in row-sum form, right-hand side, Krylov "
                                     "vectors, AMG cycle input and output) refined against the FP64 system, inside "
                                     "the FP64 residual, Jacobian entries, back-substitution, Alg. 1 and update; "
                                     "coarse levels FP64",
                        "solves_per_s": 1000.0 / percentile(ms, 0.5), "ms_per_step_p50": percentile(ms, 0.5),
                        "vcycles": st["iterations"], "krylov_iters": st["lin_iters"],
                        "refine_steps": st["refine_steps"], "converged": st["converged"],
                        "speedup_vs_fp64": fas_ms / percentile(ms, 0.5)}
        del H, keep, p, s
        torch.cuda.empty_cache()
        sd = seeds_leg(torch, pk, c2_problem, opts)
        all_ms = [fas_ms] + [v["ms"] for v in sd.values() if "ms" in v]
        out["seeds"] = {"per_seed": dict({"0": {"ms": fas_ms, "vcycles": vcycles[0], "converged": True}}, **sd),
                        "mean_ms": float(np.mean(all_ms)), "max_ms": float(np.max(all_ms)),
                        "all_converged": all(v.get("converged", False) for v in sd.values())}
        torch.cuda.empty_cache()
        out["c1"] = c1_leg(torch, pk, c1_problem)
        torch.cuda.empty_cache()
        try:
            out["unstructured"] = unstructured_leg(torch, pk)
        except pk.SpfasError as e:   # reported, not fatal
            out["unstructured"] = {"error": str(e)}
        out["served"] = served_leg(pk, args.served_requests)
        out["batched"] = batched_leg(pk, args.batch_problems)
        if args.c4:
            log("c4: the batched configuration at full size")
            out["batched_c4"] = c4_leg(pk, slots=out["batched"].get("slots", 4))

    if not args.no_cpu_baseline:
        log("CPU oracle baseline")
        out["cpu_baseline"] = cpu_baseline(n_cells, float(np.mean(vcycles)))
    log("done")

    print(json.dumps(out))


if __name__ == "__main__":
    main()
