"""No solve reads device memory before writing it (GPU): the same solves
run in a child process where every new floating-point device buffer starts
as NaN (SPFAS_POISON=1) give bit for bit the states of this process, on the
PCG, BiCGStab and Picard paths, small problems and the 262,144-cell case
with the SELL-64 level-0 paths and the benchmark's inner options.  (A PCG
first iteration once computed 0 * p on a never-written p.)"""
import math
import os
import subprocess
import sys

import numpy as np
import pytest

from problems import small_problem, c1_problem

pytestmark = pytest.mark.gpu


def cases():
    return {
        "c1": c1_problem(),
        "b": small_problem((24, 16), seed=2, box=(4, 4), m=3, n_levels=3, g_d_scale=0.3, g_n_scale=0.2,
                           dirichlet=((0, 0), (1, 1)), permute=True, alpha=1.5, src_scale=2.0),
        "big": small_problem((512, 512), seed=11, box=(4, 4), m=2, n_levels=3, permute=True, src_scale=200.0,
                             g_d_scale=0.3),
    }


def run_all():
    import paper_2005_01275_amd as pk
    out = {}
    for name, prob in cases().items():
        H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
        cap = math.log(prob.dp_cap_c) / prob.alpha
        variants = {"pcg": dict(smoother=pk.SPFAS_NEWTON, newton_pcg=1),
                    "bicgstab": dict(smoother=pk.SPFAS_NEWTON, newton_pcg=0),
                    "picard": dict(smoother=pk.SPFAS_PICARD)}
        if name == "big":
            variants = {"bench": dict(smoother=pk.SPFAS_NEWTON, newton_pcg=1, lin_rtol_coarse=1e-2, lin_target=0.03,
                                      lin_max_it_coarse=10)}
        for v, kw in variants.items():
            base = dict(rtol=1e-10 if name != "big" else 1e-8, atol=0.0, max_it=100,
                        lin_rtol=1e-8 if name != "big" else 1e-5, lin_max_it=1000, dp_cap=cap, amg_reuse=-1)
            base.update(kw)
            p, s, st = H.fas_solve(prob, pk.SolveOpts(**base))
            out[f"{name}_{v}"] = (p, s, st["iterations"])
        H.close()
    return out


def test_poisoned_buffers_change_nothing(tmp_path):
    ref = run_all()
    env = dict(os.environ, SPFAS_POISON="1")
    here = os.path.dirname(os.path.abspath(__file__))
    r = subprocess.run([sys.executable, os.path.join(here, "poison_child.py"), str(tmp_path)], env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    for name, (p, s, it) in ref.items():
        assert np.isfinite(p).all()
        np.testing.assert_array_equal(np.load(tmp_path / f"{name}_p.npy"), p, err_msg=name)
        np.testing.assert_array_equal(np.load(tmp_path / f"{name}_s.npy"), s, err_msg=name)
