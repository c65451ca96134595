"""Nonlinear solves of the HIP library against the oracle (GPU): converged
FAS and single-level Picard/Newton solutions against the oracle's root x*,
one V-cycle map against the oracle's V-cycle, and the operational stopping
rule checked with the oracle's residual.  Solutions are compared element by
element: max|x - x*| <= 1e-10 max|x*| for p and for sigma."""
import math

import numpy as np
import pytest

from problems import small_problem, c1_problem
from oracle.coarsen import build_hierarchy
from oracle.fv import full_flux, FineSystem
from oracle.solvers import Opts, result_solve, nonlinear_mg, cap_value
from parity_util import assert_elementwise

pytestmark = pytest.mark.gpu

CASES = [
    dict(shape=(8, 8), box=(4, 4), m=2, n_levels=2, seed=1, alpha=1.0, src_scale=3.0),
    dict(shape=(12, 8), box=(4, 4), m=3, n_levels=3, seed=2, g_d_scale=0.3, g_n_scale=0.2,
         dirichlet=((0, 0), (1, 1)), permute=True, alpha=1.5, src_scale=2.0),
    dict(shape=(6, 4, 4), box=(2, 2, 2), m=3, n_levels=3, seed=3, anisotropic=True, permute=True, alpha=2.0),
]


def problem(kw):
    return c1_problem() if kw == "c1" else small_problem(**kw)


def oracle_root(prob):
    h = build_hierarchy(prob)
    xs = result_solve(h)
    nf = h.levels[0].n_flux
    return h, xs[nf:], full_flux(prob, h.finemap, xs[:nf])


def opts(smoother, prob, rtol=1e-12, lin=1e-13, max_it=200):
    import paper_2005_01275_amd as pk
    return pk.SolveOpts(smoother=smoother, rtol=rtol, atol=0.0, max_it=max_it, lin_rtol=lin, lin_max_it=2000,
                        dp_cap=cap_value(prob.alpha, prob.dp_cap_c) if prob.alpha > 0 else 0.0)


@pytest.mark.parametrize("kw", CASES + ["c1"])
def test_converged_solutions(kw):
    import paper_2005_01275_amd as pk
    print("case", kw, flush=True)
    prob = problem(kw)
    h, p_star, s_star = oracle_root(prob)
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    runs = [("fas-newton", H.fas_solve, pk.SPFAS_NEWTON), ("fas-picard", H.fas_solve, pk.SPFAS_PICARD),
            ("newton", H.newton_solve, pk.SPFAS_NEWTON), ("picard", H.picard_solve, pk.SPFAS_PICARD)]
    for name, fn, sm in runs:
        print(" run", name, flush=True)
        p, s, st = fn(prob, opts(sm, prob))
        assert st["converged"], (name, st)
        assert_elementwise(p, p_star, 1e-10, f"{name} p")
        assert_elementwise(s, s_star, 1e-10, f"{name} sigma")


@pytest.mark.parametrize("kw", CASES[:2] + ["c1"])
@pytest.mark.parametrize("newton", [True, False])
def test_one_vcycle_map(kw, newton):
    """One V-cycle from x0 = 0 with (nearly) exact inner solves equals the
    oracle's V-cycle (Alg. 2 with exact sparse solves)."""
    import paper_2005_01275_amd as pk
    print("case", kw, newton, flush=True)
    prob = problem(kw)
    h = build_hierarchy(prob)
    o = Opts(newton=newton, rtol=1e-8, atol=0.0, cap_c=prob.dp_cap_c)
    lev = h.levels[0]
    x0 = np.zeros(lev.n)
    from oracle.levels import residual
    r0 = np.linalg.norm(residual(lev, x0, h.b0, h.alpha))
    x1 = nonlinear_mg(h, 0, x0, h.b0, o, stop_tol=o.rtol * r0)
    nf = lev.n_flux
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    so = opts(pk.SPFAS_NEWTON if newton else pk.SPFAS_PICARD, prob, rtol=1e-8, lin=1e-14, max_it=1)
    p, s, st = H.fas_solve(prob, so)
    assert st["iterations"] == 1
    ref_p = x1[nf:]
    ref_s = full_flux(prob, h.finemap, x1[:nf])
    assert_elementwise(p, ref_p, 1e-10, "one V-cycle p")
    assert_elementwise(s, ref_s, 1e-10, "one V-cycle sigma")


@pytest.mark.parametrize("smoother", ["newton", "picard"])
def test_operational_rtol_c1(smoother):
    """Runs at rtol 1e-8 meet the stopping rule when their state is
    re-evaluated with the oracle's residual."""
    import paper_2005_01275_amd as pk
    prob = c1_problem()
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    sm = pk.SPFAS_NEWTON if smoother == "newton" else pk.SPFAS_PICARD
    o = pk.SolveOpts(smoother=sm, rtol=1e-8, atol=0.0, dp_cap=math.log(5.0))
    fs = FineSystem(prob)
    ff = fs.fm.flux_face
    r0 = np.linalg.norm(np.concatenate(fs.residual(np.zeros(ff.size), np.zeros(prob.mesh.n_cells))))
    for fn in (H.fas_solve, H.newton_solve if sm == pk.SPFAS_NEWTON else H.picard_solve):
        p, s, st = fn(prob, o)
        assert st["converged"]
        rs, rp = fs.residual(s[ff], p)
        assert np.linalg.norm(np.concatenate([rs, rp])) <= 1.01e-8 * r0


@pytest.mark.parametrize("kw", CASES + ["c1"])
def test_newton_pcg_converged_and_vcycle(kw):
    """Newton systems solved by PCG first (BiCGStab fallback) reach the same
    root x* and, with near-exact inner solves, the same one-V-cycle map."""
    import paper_2005_01275_amd as pk
    print("case", kw, flush=True)
    prob = problem(kw)
    h, p_star, s_star = oracle_root(prob)
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    for fn in (H.fas_solve, H.newton_solve):
        o = opts(pk.SPFAS_NEWTON, prob)
        o.newton_pcg = 1
        p, s, st = fn(prob, o)
        assert st["converged"], st
        assert_elementwise(p, p_star, 1e-10, "pcg p")
        assert_elementwise(s, s_star, 1e-10, "pcg sigma")
    o = Opts(newton=True, rtol=1e-8, atol=0.0, cap_c=prob.dp_cap_c)
    lev = h.levels[0]
    x0 = np.zeros(lev.n)
    from oracle.levels import residual
    r0 = np.linalg.norm(residual(lev, x0, h.b0, h.alpha))
    x1 = nonlinear_mg(h, 0, x0, h.b0, o, stop_tol=o.rtol * r0)
    so = opts(pk.SPFAS_NEWTON, prob, rtol=1e-8, lin=1e-14, max_it=1)
    so.newton_pcg = 1
    p, s, st = H.fas_solve(prob, so)
    ref_p = x1[lev.n_flux:]
    assert_elementwise(p, ref_p, 1e-10, "pcg one V-cycle p")
    assert_elementwise(s, full_flux(prob, h.finemap, x1[:lev.n_flux]), 1e-10, "pcg one V-cycle sigma")


@pytest.mark.parametrize("kw", CASES + ["c1"])
def test_amg_reuse_reaches_the_same_root(kw):
    """Keeping the AMG values across linearisations (amg_reuse) and capping
    the coarse-level Krylov iterations only change the inner iteration:
    FAS-Newton and FAS-Picard still reach the oracle's root x*."""
    import paper_2005_01275_amd as pk
    print("case", kw, flush=True)
    prob = problem(kw)
    h, p_star, s_star = oracle_root(prob)
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    for sm in (pk.SPFAS_NEWTON, pk.SPFAS_PICARD):
        for reuse, cap in ((-1, 0), (2, 0), (-1, 10)):
            o = opts(sm, prob)
            o.newton_pcg = 1
            o.amg_reuse = reuse
            o.lin_max_it_coarse = cap   # 10: coarse Krylov solves stop early, the FAS cycle still converges
            p, s, st = H.fas_solve(prob, o)
            assert st["converged"], (sm, reuse, cap, st)
            assert_elementwise(p, p_star, 1e-10, f"reuse {sm} {reuse} {cap} p")
            assert_elementwise(s, s_star, 1e-10, f"reuse {sm} {reuse} {cap} sigma")


EDGE = [
    # more levels than the lattice coarsens: the last levels hold one aggregate each
    dict(shape=(4, 4), seed=0, box=(2, 2), m=2, n_levels=5),
    # m = 1: piecewise-constant coarse pressure
    dict(shape=(8, 8), seed=1, box=(4, 4), m=1, n_levels=2),
    # alpha = 0: the linear problem
    dict(shape=(6, 6), seed=2, box=(3, 3), m=1, n_levels=3, alpha=0.0),
    # a single level: FAS reduces to the smoother iterated on level 0
    dict(shape=(5, 3), seed=3, box=(2, 2), m=2, n_levels=1),
    # ragged 3-D boxes with a remainder layer
    dict(shape=(5, 4, 3), seed=4, box=(2, 2, 2), m=2, n_levels=2, permute=True, anisotropic=True),
]


@pytest.mark.parametrize("kw", EDGE)
def test_edge_cases_reach_the_root(kw):
    import paper_2005_01275_amd as pk
    print("case", kw, flush=True)
    prob = small_problem(**kw)
    h, p_star, s_star = oracle_root(prob)
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    for fn, sm in ((H.fas_solve, pk.SPFAS_NEWTON), (H.fas_solve, pk.SPFAS_PICARD), (H.newton_solve, pk.SPFAS_NEWTON)):
        p, s, st = fn(prob, opts(sm, prob, rtol=1e-13))
        assert st["converged"], st
        assert_elementwise(p, p_star, 1e-10, "edge p")
        assert_elementwise(s, s_star, 1e-10, "edge sigma")
    if prob.alpha == 0.0:
        # the linear limit: the reduced cell system solved by a library routine
        from oracle.fv import linear_pressure
        p_lin = linear_pressure(prob)
        assert_elementwise(p, p_lin, 1e-10, "linear limit p")


def test_warm_start_at_the_root_takes_no_cycle():
    import paper_2005_01275_amd as pk
    prob = small_problem((8, 8), seed=5, box=(4, 4), m=2, n_levels=2, src_scale=2.0)
    h, p_star, s_star = oracle_root(prob)
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    o = opts(pk.SPFAS_NEWTON, prob, rtol=1e-8)
    o.atol = 1e-12
    p, s, st = H.fas_solve(prob, o, p0=p_star, sigma0=s_star)
    assert st["converged"] and st["iterations"] == 0, st
    np.testing.assert_array_equal(p, p_star)
