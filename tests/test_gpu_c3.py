"""The unstructured workload at its full size (GPU): the Voronoi mesh of
2,000,000 seeded points, ln k = 3G, kappa = exp(2p), greedy aggregates of
about 64 cells on 2 levels, 2-6 eigenvectors per aggregate by the threshold
0.1.  The oracle's greedy aggregation and dense eigensolves do not finish at
this size, so the test checks what holds at any size: the aggregation is a
partition into connected aggregates with the fragments merged, the counts
lie in [2, 6] and size the coarse level, and FP64 and mixed-precision
FAS-Newton with the benchmark's inner options meet rtol 1e-8 under the
oracle's residual and agree element by element to 1e-8.  The smaller
Voronoi cases of test_gpu_unstructured and test_gpu_threshold hold the same
code to the oracle aggregate by aggregate."""
import math

import numpy as np
import pytest

from oracle.fv import FineSystem
from parity_util import assert_elementwise, max_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3():
    import paper_2005_01275_amd as pk
    from paper_2005_01275_amd import _native as N
    from problems.grids import c3_problem
    print("case c3: Voronoi mesh of 2,000,000 points", flush=True)
    prob = c3_problem()
    print("case c3: hierarchy", flush=True)
    H = pk.Hierarchy(prob.mesh, prob.n_levels, m=prob.m, agg_kind=N.SPFAS_AGG_GREEDY,
                     greedy_size=prob.greedy_size, eig_threshold=prob.eig_threshold, m_min=prob.m_min,
                     greedy_size_coarse=prob.greedy_size_coarse)
    yield prob, H
    H.close()


def test_c3_aggregation_and_counts(c3):
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    from paper_2005_01275_amd import _native as N
    prob, H = c3
    mesh = prob.mesh
    agg = np.asarray(H.aggregation(0), dtype=np.int64)
    n_agg = int(agg.max()) + 1
    assert agg.min() == 0 and np.unique(agg).size == n_agg
    size = np.bincount(agg, minlength=n_agg)
    # BFS growth stops at 64; merged fragments add fewer than 32 cells each
    assert size.min() >= 32, size.min()
    fc = mesh.face_cells
    inner = fc[:, 1] >= 0
    K, L = fc[inner, 0], fc[inner, 1]
    same = agg[K] == agg[L]
    g = sp.coo_matrix((np.ones(same.sum()), (K[same], L[same])), shape=(mesh.n_cells, mesh.n_cells))
    n_comp, _ = connected_components(g, directed=False)
    assert n_comp == n_agg, "every aggregate is connected"
    counts = H.level_operator(0, N.SPFAS_OP_MCOUNT, n_agg).astype(np.int64)
    assert counts.min() >= 2 and counts.max() <= 6
    nc, np_c, _ = H.level_sizes(1)
    assert nc == n_agg and np_c == counts.sum()
    print("c3: %d aggregates of %d-%d cells, counts %s" % (n_agg, size.min(), size.max(),
                                                          np.bincount(counts, minlength=7)[2:].tolist()))
    if prob.n_levels < 3:
        return
    # level 1 -> 2: aggregates of about greedy_size_coarse coarse cells, fragments below half merged
    agg1 = np.asarray(H.aggregation(1), dtype=np.int64)
    assert agg1.size == n_agg
    n_agg1 = int(agg1.max()) + 1
    assert agg1.min() == 0 and np.unique(agg1).size == n_agg1
    assert 2 * np.bincount(agg1, minlength=n_agg1).min() >= (prob.greedy_size_coarse or prob.greedy_size)
    counts1 = H.level_operator(1, N.SPFAS_OP_MCOUNT, n_agg1).astype(np.int64)
    assert counts1.min() >= 2 and counts1.max() <= 6
    assert H.level_sizes(2)[:2] == (n_agg1, counts1.sum())


def test_c3_fp64_and_mixed_meet_the_oracle_residual(c3):
    import paper_2005_01275_amd as pk
    prob, H = c3
    fs = FineSystem(prob)
    r0 = np.linalg.norm(np.concatenate([fs.g, fs.f]))
    res = {}
    for name, prec in (("fp64", pk.SPFAS_PREC_FP64), ("mixed", pk.SPFAS_PREC_MIXED)):
        print("case c3", name, flush=True)
        o = pk.SolveOpts(smoother=pk.SPFAS_NEWTON, rtol=1e-8, atol=0.0, max_it=50, lin_rtol=1e-5, lin_max_it=400,
                         lin_rtol_coarse=1e-2, lin_target=0.03, newton_pcg=1, amg_reuse=-1, lin_max_it_coarse=10,
                         coarsest_atol=1e-10, dp_cap=math.log(prob.dp_cap_c) / prob.alpha, precision=prec)
        p, s, st = H.fas_solve(prob, o)
        assert st["converged"], (name, st)
        rs, rp = fs.residual(s[fs.fm.flux_face], p)
        r = np.linalg.norm(np.concatenate([rs, rp]))
        print("c3 %s: %d V-cycles, %d Krylov, oracle residual %.2e of r0" % (name, st["iterations"],
                                                                             st["lin_iters"], r / r0))
        assert r <= 1.01e-8 * r0
        res[name] = (p, s)
    print("c3 mixed vs fp64: p %.2e sigma %.2e" % (max_rel_err(res["mixed"][0], res["fp64"][0]),
                                                   max_rel_err(res["mixed"][1], res["fp64"][1])))
    assert_elementwise(res["mixed"][0], res["fp64"][0], 1e-8, "c3 p")
    assert_elementwise(res["mixed"][1], res["fp64"][1], 1e-8, "c3 sigma")
