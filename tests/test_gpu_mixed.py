"""Mixed precision (GPU): FP32 level-0 linear solves, refined against the
FP64 linear system, inside the FP64 residual and update.  Each smoothing
step corrects the FP64 defect, so the solve reaches the FP64 root: solved
to rtol 1e-12 the state agrees with the oracle's root element by element to
1e-8 (the gate for mixed-precision results; the error is printed), and at
the operational rtol 1e-8 the state meets the stopping rule under the
oracle's residual.  Cases: C1, a small 3-D problem, the 262,144-cell case
whose level-0 system takes the SELL-64 path (FP32 SELL values), and two
ln k = 3G cases where the refinement has to run."""
import math

import numpy as np
import pytest

from problems import small_problem, c1_problem
from oracle.coarsen import build_hierarchy
from oracle.fv import full_flux, FineSystem
from oracle.solvers import result_solve
from parity_util import assert_elementwise, max_rel_err

pytestmark = pytest.mark.gpu

CASES = {
    "c1": lambda: c1_problem(),
    "small3d": lambda: small_problem((10, 8, 6), seed=3, box=(2, 2, 2), m=3, n_levels=3, anisotropic=True,
                                     permute=True, alpha=2.0),
}


def root(prob):
    h = build_hierarchy(prob, n_levels=1)
    xs = result_solve(h)
    nf = h.levels[0].n_flux
    return xs[nf:], full_flux(prob, h.finemap, xs[:nf])


def opts(prob, sm, rtol, **kw):
    import paper_2005_01275_amd as pk
    d = dict(smoother=sm, rtol=rtol, atol=0.0, max_it=200, lin_rtol=1e-6, lin_max_it=2000, newton_pcg=1,
             dp_cap=math.log(prob.dp_cap_c) / prob.alpha, precision=pk.SPFAS_PREC_MIXED)
    d.update(kw)
    return pk.SolveOpts(**d)


@pytest.mark.parametrize("case", list(CASES))
def test_mixed_reaches_the_fp64_root(case):
    import paper_2005_01275_amd as pk
    prob = CASES[case]()
    p_star, s_star = root(prob)
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    for name, fn, sm in (("fas-newton", H.fas_solve, pk.SPFAS_NEWTON), ("fas-picard", H.fas_solve, pk.SPFAS_PICARD),
                         ("newton", H.newton_solve, pk.SPFAS_NEWTON)):
        p, s, st = fn(prob, opts(prob, sm, 1e-12))
        assert st["converged"], (name, st)
        print(case, name, "max rel error vs the FP64 root: p %.2e sigma %.2e" % (max_rel_err(p, p_star),
                                                                               max_rel_err(s, s_star)))
        assert_elementwise(p, p_star, 1e-8, f"{case} {name} p")
        assert_elementwise(s, s_star, 1e-8, f"{case} {name} sigma")


@pytest.mark.parametrize("case", list(CASES))
def test_mixed_operational_rtol(case):
    import paper_2005_01275_amd as pk
    prob = CASES[case]()
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    fs = FineSystem(prob)
    r0 = np.linalg.norm(np.concatenate([fs.g, fs.f]))
    for sm in (pk.SPFAS_NEWTON, pk.SPFAS_PICARD):
        p, s, st = H.fas_solve(prob, opts(prob, sm, 1e-8, lin_rtol=1e-5))
        assert st["converged"], st
        rs, rp = fs.residual(s[fs.fm.flux_face], p)
        assert np.linalg.norm(np.concatenate([rs, rp])) <= 1.01e-8 * r0


def test_mixed_sell_path_at_262144_cells():
    import json
    import os
    import paper_2005_01275_amd as pk
    from oracle.fv import fine_level
    from oracle.levels import M_of
    here = os.path.dirname(os.path.abspath(__file__))
    meta = json.load(open(os.path.join(here, "golden", "root_512x512_p.json")))
    recipe = {k: tuple(v) if isinstance(v, list) else v for k, v in meta["recipe"].items()}
    prob = small_problem(**recipe)
    p_star = np.load(os.path.join(here, "golden", "root_512x512_p.npy"))
    lev, b0, fm = fine_level(prob)
    s_star = full_flux(prob, fm, -(lev.D.T @ p_star - b0[:lev.n_flux]) / M_of(lev, p_star, prob.alpha).diagonal())
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    p, s, st = H.fas_solve(prob, opts(prob, pk.SPFAS_NEWTON, 1e-12), device=True)
    assert st["converged"], st
    p, s = p.cpu().numpy(), s.cpu().numpy()
    print("512x512 mixed: max rel error p %.2e sigma %.2e" % (max_rel_err(p, p_star), max_rel_err(s, s_star)))
    assert_elementwise(p, p_star, 1e-8, "p")
    assert_elementwise(s, s_star, 1e-8, "sigma")
    # the benchmark's inner options at rtol 1e-8
    o = opts(prob, pk.SPFAS_NEWTON, 1e-8, lin_rtol=1e-5, lin_max_it=400, lin_rtol_coarse=1e-2, lin_target=0.03,
             amg_reuse=-1, lin_max_it_coarse=10, coarsest_atol=1e-10)
    p, s, st = H.fas_solve(prob, o)
    assert st["converged"], st
    fs = FineSystem(prob)
    rs, rp = fs.residual(s[fs.fm.flux_face], p)
    assert np.linalg.norm(np.concatenate([rs, rp])) <= 1.01e-8 * np.linalg.norm(np.concatenate([fs.g, fs.f]))


def high_contrast(case):
    """ln k = 3G, kappa = exp(2p), the source pair scaled by the oracle's
    linear (kappa = 1) solve to alpha max |p_lin| = 0.5."""
    import dataclasses
    from problems.grids import Problem, cartesian_mesh, gaussian_field, voronoi_problem, _flat
    from oracle.fv import linear_pressure
    if case == "grid512":   # 262,144 cells: the SELL-64 level-0 path (FP32 rows in row-sum form)
        rng = np.random.default_rng(11)
        n = 512
        k = np.exp(3.0 * _flat(gaussian_field((n, n), 5.0, rng)))
        mesh = cartesian_mesh((n, n), (1.0 / n, 1.0 / n), k, dirichlet=((0, 0),))
        src = np.zeros(n * n)
        src[n // 2 + n * (n // 2)] = 1.0
        src[n * n - 1] = -1.0
        prob = Problem(mesh=mesh, alpha=2.0, source=src, g_dirichlet=np.zeros(mesh.n_faces),
                       g_neumann=np.zeros(mesh.n_faces), name="grid512_3g", box=(4, 4), m=3, n_levels=3)
    else:                   # 20,000 Voronoi cells: the DIA+CSR level-0 path
        prob = voronoi_problem(n_points=20000, seed=3, sigma=3.0, corr_len=0.01, alpha=2.0, n_levels=2,
                               greedy_size=64, m=6, eig_threshold=0.1, m_min=2)
    rate = 0.5 / (prob.alpha * np.abs(linear_pressure(prob)).max())
    return dataclasses.replace(prob, source=prob.source * rate)


@pytest.mark.parametrize("case", ["grid512", "voronoi20k"])
def test_mixed_refinement_on_high_contrast(case):
    """On ln k = 3G the FP32 level-0 solutions alone leave FP64 residuals far
    above the inner tolerance (FP32 vectors cannot hold a more accurate
    solution); the refinement against the FP64 system runs (refine_steps >
    0), mixed FAS-Newton takes no more V-cycles than FP64, meets the stopping
    rule under the oracle's residual and agrees with the FP64 result."""
    import paper_2005_01275_amd as pk
    from paper_2005_01275_amd import _native as N
    print("case", case, flush=True)
    prob = high_contrast(case)
    if prob.greedy_size:
        H = pk.Hierarchy(prob.mesh, prob.n_levels, m=prob.m, agg_kind=N.SPFAS_AGG_GREEDY,
                         greedy_size=prob.greedy_size, eig_threshold=prob.eig_threshold, m_min=prob.m_min)
    else:
        H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    res = {}
    for name, prec in (("fp64", pk.SPFAS_PREC_FP64), ("mixed", pk.SPFAS_PREC_MIXED)):
        o = opts(prob, pk.SPFAS_NEWTON, 1e-8, lin_rtol=1e-5, lin_max_it=400, lin_rtol_coarse=1e-2, lin_target=0.03,
                 amg_reuse=-1, lin_max_it_coarse=10, coarsest_atol=1e-10, max_it=60, precision=prec)
        p, s, st = H.fas_solve(prob, o)
        print(case, name, {k: st[k] for k in ("iterations", "lin_iters", "refine_steps", "converged")}, flush=True)
        assert st["converged"], (name, st)
        res[name] = (p, s, st)
    H.close()
    pm, sm, stm = res["mixed"]
    p64, s64, st64 = res["fp64"]
    assert stm["refine_steps"] > 0
    assert st64["refine_steps"] == 0
    assert stm["iterations"] <= st64["iterations"]
    fs = FineSystem(prob)
    rs, rp = fs.residual(sm[fs.fm.flux_face], pm)
    assert np.linalg.norm(np.concatenate([rs, rp])) <= 1.01e-8 * np.linalg.norm(np.concatenate([fs.g, fs.f]))
    print(case, "mixed vs fp64: p %.2e sigma %.2e" % (max_rel_err(pm, p64), max_rel_err(sm, s64)))
    assert_elementwise(pm, p64, 1e-8, f"{case} p")
    assert_elementwise(sm, s64, 1e-8, f"{case} sigma")
