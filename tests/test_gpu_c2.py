"""Full-size 60x220x85 workload, with plain inner solves and with the
inner-solver options bench.py times (GPU): the returned state meets the
stopping rule when re-evaluated with the oracle's residual, the level-0
aggregation matches the oracle bit for bit, and sampled aggregates of the
hierarchy match the oracle's local computations."""
import math

import numpy as np
import pytest

from problems import c2_problem
from oracle.fv import FineSystem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2():
    import paper_2005_01275_amd as pk
    prob = c2_problem()
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    return prob, H


# the inner-solver options bench.py times (level-0 tolerance 1e-5 with
# forcing 0.03, coarse tolerance 1e-2 with at most 10 iterations, PCG first
# on Newton systems, AMG values reused)
BENCH_INNER = dict(lin_rtol=1e-5, lin_max_it=400, lin_rtol_coarse=1e-2, lin_target=0.03, newton_pcg=1,
                   amg_reuse=-1, lin_max_it_coarse=10, coarsest_atol=1e-10)


@pytest.mark.parametrize("inner", ["plain", "bench"])
def test_c2_fas_newton_meets_rtol(c2, inner):
    import paper_2005_01275_amd as pk
    prob, H = c2
    print(f"case c2 fas-newton {inner}", flush=True)
    kw = dict(lin_rtol=1e-4, lin_max_it=400) if inner == "plain" else BENCH_INNER
    o = pk.SolveOpts(smoother=pk.SPFAS_NEWTON, rtol=1e-8, atol=0.0, max_it=50,
                     dp_cap=math.log(prob.dp_cap_c) / prob.alpha, **kw)
    p, s, st = H.fas_solve(prob, o)
    assert st["converged"], st
    fs = FineSystem(prob)
    ff = fs.fm.flux_face
    r0 = np.linalg.norm(fs.f)
    rs, rp = fs.residual(s[ff], p)
    rel = np.linalg.norm(np.concatenate([rs, rp])) / r0
    assert rel <= 1.01e-8, rel
    # flux conservation at the solution: all injected fluid leaves through the Dirichlet faces
    dirf = ~fs.inner
    assert abs(s[ff][dirf].sum() - fs.f.sum()) <= 1e-6 * np.abs(fs.f).sum()


# the cascadic solve needs every coarse level solved to its own tolerance
# (Section 4.2), which the FAS coarse options (1e-2, at most 10 Krylov
# iterations) do not reach on level 2: the benchmark runs it with coarse
# linear solves to 1e-6 and no coarse iteration limit
CASCADIC_INNER = dict(BENCH_INNER, lin_rtol_coarse=1e-6, lin_max_it_coarse=0)


def test_c2_cascadic_meets_rtol(c2):
    """The nonlinear cascadic solve bench.py reports beside FAS-Newton: every
    level converges to its own tolerance and the fine state meets the
    stopping rule under the oracle's residual."""
    import paper_2005_01275_amd as pk
    prob, H = c2
    print("case c2 cascadic", flush=True)
    o = pk.SolveOpts(smoother=pk.SPFAS_NEWTON, rtol=1e-8, atol=0.0, max_it=200,
                     dp_cap=math.log(prob.dp_cap_c) / prob.alpha, **CASCADIC_INNER)
    p, s, st = H.cascadic_solve(prob, o)
    assert st["converged"] and len(st["level_steps"]) == prob.n_levels, st
    assert max(st["level_steps"]) < 200, st
    fs = FineSystem(prob)
    ff = fs.fm.flux_face
    rs, rp = fs.residual(s[ff], p)
    rel = np.linalg.norm(np.concatenate([rs, rp])) / np.linalg.norm(fs.f)
    assert rel <= 1.01e-8, rel


def test_c2_aggregation_bit_exact(c2):
    """The device-built hierarchy's level-0 aggregation and renumbering equal
    the oracle's box rule on the lattice recovered from the centroids."""
    from oracle.fv import lattice_from_centroids
    from oracle.coarsen import box_aggregate
    prob, H = c2
    shape, index = lattice_from_centroids(prob.mesh.cell_centroid)
    agg, cshape = box_aggregate(shape, index, prob.box)
    assert cshape == (15, 55, 21)
    np.testing.assert_array_equal(H.aggregation(0), agg)
    c, _ = H.permutation(0)
    # cells contiguous per aggregate, ascending id inside each one
    np.testing.assert_array_equal(c, np.lexsort((np.arange(agg.size), agg)))


def test_c2_aggregates_sampled(c2):
    """Sampled level-0 aggregates: the m = 3 smallest eigenvalues of each
    local Laplacian (static matrices, eq. local-eigenvalue-problem) against a
    dense eigen-solve of the weighted graph Laplacian of the same cells."""
    from paper_2005_01275_amd import _native as N
    prob, H = c2
    n_agg = 17325
    m = prob.m
    lam_gpu = H.level_operator(0, N.SPFAS_OP_EIGVALS, n_agg * m)
    agg = H.aggregation(0)
    rng = np.random.default_rng(0)
    sample = rng.choice(n_agg, 6, replace=False)
    fs = FineSystem(prob)
    for A in sample:
        cells = np.sort(np.nonzero(agg == A)[0])
        inside = np.isin(fs.K, cells) & np.isin(np.where(fs.inner, fs.L, -1), cells)
        pos = {c: i for i, c in enumerate(cells)}
        n = cells.size
        # weighted graph Laplacian of the aggregate with harmonic transmissibilities (kappa = 1)
        Lm = np.zeros((n, n))
        for f in np.nonzero(inside)[0]:
            w = 1.0 / (1.0 / fs.TK[f] + 1.0 / fs.TL[f])
            i, j = pos[fs.K[f]], pos[fs.L[f]]
            Lm[i, i] += w; Lm[j, j] += w; Lm[i, j] -= w; Lm[j, i] -= w
        lam = np.linalg.eigvalsh(Lm)
        np.testing.assert_allclose(lam_gpu[m * A:m * (A + 1)], lam[:m], atol=1e-10 * lam[-1])


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_c2_other_seeds_converge_at_bench_options(seed):
    """Seeds 1-4 of the same recipe (their own fields and permutations)
    with the benchmark's inner options: each converges and meets rtol 1e-8
    under the oracle's residual."""
    import paper_2005_01275_amd as pk
    print(f"case c2 seed {seed}", flush=True)
    prob = c2_problem(seed=seed)
    H = pk.Hierarchy(prob.mesh, prob.n_levels, prob.box, prob.m)
    o = pk.SolveOpts(smoother=pk.SPFAS_NEWTON, rtol=1e-8, atol=0.0, max_it=50,
                     dp_cap=math.log(prob.dp_cap_c) / prob.alpha, **BENCH_INNER)
    p, s, st = H.fas_solve(prob, o)
    H.close()
    assert st["converged"], st
    fs = FineSystem(prob)
    rs, rp = fs.residual(s[fs.fm.flux_face], p)
    rel = np.linalg.norm(np.concatenate([rs, rp])) / np.linalg.norm(fs.f)
    assert rel <= 1.01e-8, rel
