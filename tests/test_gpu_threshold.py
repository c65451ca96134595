"""Eigenvector count per aggregate by eigenvalue threshold (GPU): the counts
the device setup chooses equal the oracle's aggregate by aggregate, the
hierarchies built on them agree (eigenvalues, P_sigma, M, D), and FAS on
them reaches the oracle's root; one V-cycle map on a threshold hierarchy
matches the oracle's.  Each case first checks that no eigenvalue lies within
1e-8 (relative to the aggregate's largest) of the threshold, where the count
would be decided by rounding."""
import math

import numpy as np
import pytest

from problems import small_problem
from problems.grids import voronoi_problem
from oracle.coarsen import build_hierarchy
from oracle.fv import full_flux
from oracle.levels import residual
from oracle.solvers import Opts, nonlinear_mg, result_solve
from parity_util import assert_elementwise, max_rel_err

pytestmark = pytest.mark.gpu

THR, M_MAX, M_MIN = 0.1, 6, 2


def voronoi(**kw):
    from oracle.fv import linear_pressure
    prob = voronoi_problem(**kw)
    rate = 0.5 / (kw["alpha"] * np.abs(linear_pressure(prob)).max())
    return voronoi_problem(**kw, rate=rate)


CASES = {
    "voronoi": lambda: (voronoi(n_points=2000, seed=1, n_levels=3, m=M_MAX, alpha=2.0, sigma=1.0,
                                eig_threshold=THR, m_min=M_MIN), 64),
    "box-2d": lambda: (small_problem((12, 12), seed=8, sigma=1.5, box=(4, 4), m=M_MAX, n_levels=3, alpha=1.0,
                                     src_scale=3.0, permute=True), 0),
    "box-3d": lambda: (small_problem((8, 8, 4), seed=9, sigma=1.0, box=(2, 2, 2), m=M_MAX, n_levels=3, alpha=1.5,
                                     src_scale=2.0, anisotropic=True), 0),
}


def hierarchies(case):
    import paper_2005_01275_amd as pk
    from paper_2005_01275_amd import _native as N
    prob, target = CASES[case]()
    h = build_hierarchy(prob, greedy_size=target, eig_threshold=THR, m_min=M_MIN)
    for tr in h.transfers:
        for ad in tr.aggs:
            lam = ad.lam
            if lam.size > 1:
                gap = np.min(np.abs(lam - THR * lam[-1])) / lam[-1]
                assert gap > 1e-8, f"{case}: an eigenvalue at the threshold ({gap:.1e})"
    kw = dict(agg_kind=N.SPFAS_AGG_GREEDY, greedy_size=target) if target else {}
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, M_MAX, eig_threshold=THR, m_min=M_MIN, **kw)
    return prob, h, H


@pytest.mark.parametrize("case", list(CASES))
def test_threshold_counts_and_hierarchy(case):
    from paper_2005_01275_amd import _native as N
    print("case", case, flush=True)
    prob, h, H = hierarchies(case)
    varied = False
    for l, tr in enumerate(h.transfers):
        clev = h.levels[l + 1]
        ms = np.array([ad.P.shape[1] for ad in tr.aggs])
        varied = varied or ms.min() < ms.max()
        got = H.level_operator(l, N.SPFAS_OP_MCOUNT, clev.n_cells)
        np.testing.assert_array_equal(got, ms)
        assert H.level_sizes(l + 1) == (clev.n_cells, clev.n_p, clev.n_flux)
        g = H.level_operator(l, N.SPFAS_OP_EIGVALS, int(ms.sum()))
        for ad, m, seg in zip(tr.aggs, ms, np.split(g, np.cumsum(ms)[:-1])):
            np.testing.assert_allclose(seg, ad.lam[:m], rtol=0.0, atol=1e-12 * abs(ad.lam[-1]))
        Ps = tr.P_sig.toarray()
        assert max_rel_err(H.level_operator(l, N.SPFAS_OP_PSIGMA, Ps.size).reshape(Ps.shape), Ps) <= 1e-10
        M = np.concatenate([m.ravel() for m in clev.M_loc])
        assert max_rel_err(H.level_operator(l, N.SPFAS_OP_MLOC, M.size), M) <= 1e-10
        D = np.concatenate([d.ravel() for d in clev.D_loc])
        assert max_rel_err(H.level_operator(l, N.SPFAS_OP_DLOC, D.size), D) <= 1e-10
    if case != "voronoi":   # the Voronoi aggregates of about 64 cells all keep the upper clamp 6
        assert varied, "the case should have counts that differ between aggregates"


@pytest.mark.parametrize("case", list(CASES))
def test_threshold_fas_root_and_vcycle(case):
    import paper_2005_01275_amd as pk
    print("case", case, flush=True)
    prob, h, H = hierarchies(case)
    xs = result_solve(h)
    nf = h.levels[0].n_flux
    p_star, s_star = xs[nf:], full_flux(prob, h.finemap, xs[:nf])
    cap = math.log(prob.dp_cap_c) / prob.alpha
    for sm in (pk.SPFAS_NEWTON, pk.SPFAS_PICARD):
        o = pk.SolveOpts(smoother=sm, rtol=1e-13, atol=0.0, max_it=200, lin_rtol=1e-13, lin_max_it=4000, dp_cap=cap)
        p, s, st = H.fas_solve(prob, o)
        assert st["converged"], (sm, st)
        assert_elementwise(p, p_star, 1e-10, f"{case} {sm} p")
        assert_elementwise(s, s_star, 1e-10, f"{case} {sm} sigma")
    # one V-cycle from zero with near-exact inner solves
    lev = h.levels[0]
    x0 = np.zeros(lev.n)
    r0 = np.linalg.norm(residual(lev, x0, h.b0, h.alpha))
    oo = Opts(newton=True, rtol=1e-8, atol=0.0, cap_c=prob.dp_cap_c)
    x1 = nonlinear_mg(h, 0, x0, h.b0, oo, stop_tol=oo.rtol * r0)
    so = pk.SolveOpts(smoother=pk.SPFAS_NEWTON, rtol=1e-8, atol=0.0, max_it=1, lin_rtol=1e-14, lin_max_it=4000,
                      dp_cap=cap)
    p, s, st = H.fas_solve(prob, so)
    assert st["iterations"] == 1
    assert_elementwise(p, x1[nf:], 1e-10, "one V-cycle p")
    assert_elementwise(s, full_flux(prob, h.finemap, x1[:nf]), 1e-10, "one V-cycle sigma")
