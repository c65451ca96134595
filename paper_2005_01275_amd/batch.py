"""Batched setup and solve of many independent problems on one GPU through
the native serving runtime (spfas_server_*), with a small autotuner for the
batch shape: the number of solves in flight.

Each problem gets its own hierarchy (built on the device when its first
request is admitted) and its solve runs on one of the server's worker
streams, so setups and solves of different problems overlap.  The autotuner
times the same sample of problems at several slot counts and keeps the
fastest.  Argument marshalling and timing only; all work is native."""
from __future__ import annotations

import time

from .serve import Server, FAS


def solve_batch(problems, opts, n_slots, hbm_budget=0, kind=FAS):
    """Sets up and solves every problem (``problems.Problem`` with its
    hierarchy configuration); returns (results, seconds, counters) with
    results[i] = (p, sigma, stats, info)."""
    t0 = time.perf_counter()
    with Server(n_slots=n_slots, hbm_budget=hbm_budget) as S:
        tickets = []
        for pr in problems:
            mid = S.add_model(pr.mesh, pr.n_levels, pr.box, pr.m)
            tickets.append(S.submit(mid, pr, opts, kind))
        res = [S.wait(t) for t in tickets]
        cnt = S.counters()
    return res, time.perf_counter() - t0, cnt


def autotune_slots(sample, opts, candidates=(1, 2, 4, 8), hbm_budget=0):
    """Times solve_batch on `sample` for every slot count; returns (best,
    {slots: seconds})."""
    table = {}
    for k in candidates:
        _, sec, _ = solve_batch(sample, opts, k, hbm_budget)
        table[k] = sec
    best = min(table, key=table.get)
    return best, table
