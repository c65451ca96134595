"""Root parity at 262,144 cells (GPU): a 512 x 512 problem large enough for
the library's SELL-64 level-0 paths, 3 levels of 4 x 4 boxes, m = 2.  The
oracle's root x* (result oracle: damped Newton with exact sparse solves) is
stored by tests/golden/make_root_512.py; sigma* follows from p* face by face
since the flux rows of the residual vanish at the root.  The GPU solves to
rtol 1e-13 and every entry of p and sigma must lie within 1e-10 of the
largest entry of p* and sigma*."""
import hashlib
import json
import math
import os

import numpy as np
import pytest

from problems import small_problem
from parity_util import assert_elementwise

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def case():
    import paper_2005_01275_amd as pk
    from oracle.fv import fine_level, full_flux
    from oracle.levels import M_of
    meta = json.load(open(os.path.join(HERE, "golden", "root_512x512_p.json")))
    recipe = {k: tuple(v) if isinstance(v, list) else v for k, v in meta["recipe"].items()}
    prob = small_problem(**recipe)
    p_star = np.load(os.path.join(HERE, "golden", "root_512x512_p.npy"))
    assert hashlib.sha256(p_star.tobytes()).hexdigest() == meta["sha256"]
    lev, b0, fm = fine_level(prob)
    g = -b0[:lev.n_flux]
    s_dofs = -(lev.D.T @ p_star + g) / M_of(lev, p_star, prob.alpha).diagonal()
    s_star = full_flux(prob, fm, s_dofs)
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    return prob, H, p_star, s_star


def test_512_root_fixture_is_the_root(case):
    """The stored p* with its sigma* has a relative residual at rounding
    level under the oracle's face-by-face residual."""
    from oracle.fv import FineSystem
    prob, _, p_star, s_star = case
    fs = FineSystem(prob)
    rs, rp = fs.residual(s_star[fs.fm.flux_face], p_star)
    assert np.linalg.norm(np.concatenate([rs, rp])) <= 1e-12 * np.linalg.norm(fs.f)


@pytest.mark.parametrize("name", ["fas-newton", "fas-newton-pcg", "fas-picard", "newton"])
def test_512_root_parity(case, name):
    import paper_2005_01275_amd as pk
    prob, H, p_star, s_star = case
    print("case 512x512", name, flush=True)
    o = pk.SolveOpts(smoother=pk.SPFAS_PICARD if name == "fas-picard" else pk.SPFAS_NEWTON, rtol=1e-13, atol=0.0,
                     max_it=200, lin_rtol=1e-13, lin_max_it=4000,
                     dp_cap=math.log(prob.dp_cap_c) / prob.alpha)
    if name == "fas-newton-pcg":
        o.newton_pcg = 1
    fn = H.newton_solve if name == "newton" else H.fas_solve
    p, s, st = fn(prob, o, device=True)
    assert st["converged"], st
    assert_elementwise(p.cpu().numpy(), p_star, 1e-10, f"{name} p")
    assert_elementwise(s.cpu().numpy(), s_star, 1e-10, f"{name} sigma")


def test_512_bench_options_meet_rtol(case):
    """The inner-solver options of the benchmark at rtol 1e-8: the state
    meets the stopping rule under the oracle's residual."""
    import paper_2005_01275_amd as pk
    from oracle.fv import FineSystem
    prob, H, p_star, _ = case
    o = pk.SolveOpts(smoother=pk.SPFAS_NEWTON, rtol=1e-8, atol=0.0, max_it=50, lin_rtol=1e-5, lin_max_it=400,
                     lin_rtol_coarse=1e-2, lin_target=0.03, newton_pcg=1, amg_reuse=-1, lin_max_it_coarse=10,
                     coarsest_atol=1e-10, dp_cap=math.log(prob.dp_cap_c) / prob.alpha)
    p, s, st = H.fas_solve(prob, o)
    assert st["converged"], st
    fs = FineSystem(prob)
    r0 = np.linalg.norm(np.concatenate([fs.g, fs.f]))
    rs, rp = fs.residual(s[fs.fm.flux_face], p)
    assert np.linalg.norm(np.concatenate([rs, rp])) <= 1.01e-8 * r0
