"""Serving runtime (GPU): requests of several models solved concurrently by
the native server give bit for bit the results of the same solves run alone
(isolation); admission by device-memory footprint evicts idle hierarchies
and stays within the budget; a model that cannot fit fails cleanly."""
import math

import numpy as np
import pytest

from problems import small_problem, c1_problem
from parity_util import assert_elementwise

pytestmark = pytest.mark.gpu


def models():
    return [
        c1_problem(),
        small_problem((24, 16), seed=2, box=(4, 4), m=3, n_levels=3, g_d_scale=0.3, g_n_scale=0.2,
                      dirichlet=((0, 0), (1, 1)), permute=True, alpha=1.5, src_scale=2.0),
        small_problem((10, 8, 6), seed=3, box=(2, 2, 2), m=3, n_levels=3, anisotropic=True, permute=True, alpha=2.0),
        small_problem((40, 40), seed=4, box=(4, 4), m=2, n_levels=3, alpha=1.0, src_scale=3.0),
    ]


def opts(prob):
    import paper_2005_01275_amd as pk
    return pk.SolveOpts(smoother=pk.SPFAS_NEWTON, rtol=1e-10, atol=0.0, max_it=100, lin_rtol=1e-8, lin_max_it=1000,
                        dp_cap=math.log(prob.dp_cap_c) / prob.alpha, newton_pcg=1, amg_reuse=-1)


def with_source(prob, seed):
    """The same model with another source density (another request)."""
    import dataclasses
    rng = np.random.default_rng(seed)
    src = prob.source * (0.5 + rng.random())
    return dataclasses.replace(prob, source=src)


def alone(prob):
    import paper_2005_01275_amd as pk
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    out = H.fas_solve(prob, opts(prob))
    H.close()
    return out


def test_results_in_the_mix_equal_alone():
    from paper_2005_01275_amd.serve import Server
    ms = models()
    reqs = []
    for k in range(3):
        for i, prob in enumerate(ms):
            reqs.append((i, with_source(prob, 10 * i + k)))
    ref = [alone(pr) for _, pr in reqs]
    with Server(n_slots=4) as S:
        ids = [S.add_model(pr.mesh, pr.n_levels, pr.box, pr.m) for pr in ms]
        tickets = [S.submit(ids[i], pr, opts(pr)) for i, pr in reqs]
        got = [S.wait(t) for t in tickets]
        c = S.counters()
    assert c["completed"] == len(reqs) and c["setups"] == len(ms) and c["cache_hits"] == len(reqs) - len(ms)
    for (p_ref, s_ref, st_ref), (p, s, st, info) in zip(ref, got):
        assert st["converged"] and st["iterations"] == st_ref["iterations"]
        np.testing.assert_array_equal(p, p_ref)
        np.testing.assert_array_equal(s, s_ref)
    # a served result meets the stopping rule under the oracle's residual
    from oracle.fv import FineSystem
    i, pr = reqs[5]
    fs = FineSystem(pr)
    p, s = got[5][0], got[5][1]
    rs, rp = fs.residual(s[fs.fm.flux_face], p)
    r0 = np.linalg.norm(np.concatenate([fs.g, fs.f]))
    assert np.linalg.norm(np.concatenate([rs, rp])) <= 1.01e-10 * r0


def test_admission_by_footprint_evicts_idle_hierarchies():
    import paper_2005_01275_amd as pk
    from paper_2005_01275_amd.serve import Server
    ms = models()
    held, peak = [], []
    for pr in ms:
        H = pk.Hierarchy(pr.mesh, pr.n_levels, pr.box, pr.m)
        H.fas_solve(pr, opts(pr))
        b, pk_ = H.device_bytes()
        held.append(b)
        peak.append(pk_)
        H.close()
    # a build reserves the larger of the model's measured peak (setup scratch
    # included) and the sizes-based estimate the server starts from; a cached
    # idle hierarchy reserves what it holds.  The budget admits any one build
    # but not a build beside every other hierarchy cached, so builds evict.
    est = [3072 * pr.mesh.n_cells + 1024 * pr.mesh.n_faces + (16 << 20) for pr in ms]
    need = max(max(peak), max(est))
    budget = need + min(held) // 2
    assert budget < need + sum(held) - max(held)
    ref = [alone(pr) for pr in ms]
    with Server(n_slots=3, hbm_budget=budget) as S:
        ids = [S.add_model(pr.mesh, pr.n_levels, pr.box, pr.m) for pr in ms]
        tickets = []
        for k in range(3):
            for i, pr in enumerate(ms):
                tickets.append((i, S.submit(ids[i], pr, opts(pr))))
        got = [(i, S.wait(t)) for i, t in tickets]
        c = S.counters()
    assert c["evictions"] > 0 and c["peak_bytes"] <= budget and c["completed"] == len(tickets)
    for i, (p, s, st, info) in got:
        assert st["converged"]
        np.testing.assert_array_equal(p, ref[i][0])
        np.testing.assert_array_equal(s, ref[i][1])


def test_model_above_the_budget_fails_cleanly():
    from paper_2005_01275_amd.serve import Server, ServerError
    pr = models()[1]
    with Server(n_slots=2, hbm_budget=1 << 20) as S:
        mid = S.add_model(pr.mesh, pr.n_levels, pr.box, pr.m)
        t = S.submit(mid, pr, opts(pr))
        with pytest.raises(ServerError, match="budget"):
            S.wait(t)
