"""Aggregation kinds other than boxes (CPU): the oracle's greedy graph
aggregation pinned on hand-worked cases and invariants, the library's
greedy aggregation and renumbering bit for bit against the oracle's on
Cartesian and Voronoi meshes (host_only handles), a USER aggregation equal
to the box rule giving the same hierarchy topology as BOX, and malformed
USER aggregations rejected."""
import numpy as np
import pytest

from problems import small_problem
from problems.grids import voronoi_problem
from oracle.fv import fine_level
from oracle.coarsen import greedy_aggregate, build_hierarchy, box_aggregate, renumber


def level0(prob):
    return fine_level(prob)[0]


def test_greedy_hand_chain():
    # a 9-cell chain, target 4: {0..3}, {4..7}, {8}; the single cell (below
    # 4/2) joins its only neighbour aggregate
    lev = level0(small_problem((9, 1), seed=0))
    np.testing.assert_array_equal(greedy_aggregate(lev, 4), [0, 0, 0, 0, 1, 1, 1, 1, 1])
    # 11 cells: the last aggregate has 3 >= 4/2 cells and stays
    lev = level0(small_problem((11, 1), seed=0))
    np.testing.assert_array_equal(greedy_aggregate(lev, 4), [0, 0, 0, 0, 1, 1, 1, 1, 2, 2, 2])


def test_greedy_hand_grid():
    # 4x4 grid, cell id i + 4 j, target 4, worked by hand: seed 0 takes 1 and
    # 4 then 2; seed 3 takes 7, then 6 and 11; seed 5 takes 9, then 8 and 10;
    # seed 12 takes 13, 14, 15
    lev = level0(small_problem((4, 4), seed=0))
    want = [0, 0, 0, 1, 0, 2, 1, 1, 2, 2, 2, 1, 3, 3, 3, 3]
    np.testing.assert_array_equal(greedy_aggregate(lev, 4), want)


def test_greedy_fragment_joins_the_neighbour_with_most_faces():
    # 5x2 grid, target 8: seed 0 grows over 8 cells ({0,1,5,2,6,3,7,4}), the
    # left-over cell 9 shares one face with that aggregate and joins it
    lev = level0(small_problem((5, 2), seed=0))
    np.testing.assert_array_equal(greedy_aggregate(lev, 8), np.zeros(10, dtype=np.int64))
    # 3x3 grid, target 3: seed 0 takes 1 and 3; seed 2 takes 5, then 4;
    # seed 6 takes 7, then 8: no fragments
    lev = level0(small_problem((3, 3), seed=0))
    np.testing.assert_array_equal(greedy_aggregate(lev, 3), [0, 0, 1, 0, 1, 1, 2, 2, 2])


def _connected(lev, agg):
    fc = lev.flux_cells
    ok = True
    for A in np.unique(agg):
        cells = set(np.nonzero(agg == A)[0].tolist())
        start = next(iter(cells))
        seen, stack = {start}, [start]
        while stack:
            u = stack.pop()
            for j in lev.cell_flux[u]:
                a, b = int(fc[j, 0]), int(fc[j, 1])
                if b < 0:
                    continue
                v = b if a == u else a
                if v in cells and v not in seen:
                    seen.add(v)
                    stack.append(v)
        ok &= seen == cells
    return ok


def test_greedy_invariants_on_a_voronoi_mesh():
    prob = voronoi_problem(1500, seed=3)
    lev = level0(prob)
    agg = greedy_aggregate(lev, 64)
    sizes = np.bincount(agg)
    assert sizes.sum() == lev.n_cells and sizes.min() >= 32
    assert np.array_equal(np.unique(agg), np.arange(agg.max() + 1))
    assert _connected(lev, agg)


def host_handle(prob, n_levels, **kw):
    import paper_2005_01275_amd as pk
    return pk.Hierarchy(prob.mesh, n_levels, m=prob.m, host_only=True, **kw)


@pytest.mark.parametrize("case", ["voronoi", "cart2d", "cart3d"])
def test_greedy_bit_exact(case):
    from paper_2005_01275_amd import _native as N
    if case == "voronoi":
        prob, target, L = voronoi_problem(2000, seed=1, n_levels=3), 64, 3
    elif case == "cart2d":
        prob, target, L = small_problem((12, 10), seed=2, m=2, n_levels=3, permute=True), 8, 3
    else:
        prob, target, L = small_problem((6, 5, 4), seed=3, m=2, n_levels=3, permute=True), 6, 3
    h = build_hierarchy(prob, n_levels=L, greedy_size=target)
    H = host_handle(prob, L, agg_kind=N.SPFAS_AGG_GREEDY, greedy_size=target)
    for l, tr in enumerate(h.transfers):
        np.testing.assert_array_equal(H.aggregation(l), tr.agg)
        c, f = H.permutation(l)
        np.testing.assert_array_equal(c, tr.cell_order)
        np.testing.assert_array_equal(f, tr.flux_order)
        clev = h.levels[l + 1]
        assert H.level_sizes(l + 1) == (clev.n_cells, clev.n_p, clev.n_flux)


def test_greedy_bit_exact_on_the_threaded_host_path():
    """40,000 Voronoi cells: above the size from which the library's host
    steps (neighbour lists, renumbering keys and bucket sorts) run on
    several threads; level-0 aggregation and renumbering against the
    oracle's, bit for bit."""
    from paper_2005_01275_amd import _native as N
    prob = voronoi_problem(40000, seed=5, n_levels=2)
    lev = level0(prob)
    agg = greedy_aggregate(lev, 64)
    co, fo = renumber(lev, agg)
    H = host_handle(prob, 2, agg_kind=N.SPFAS_AGG_GREEDY, greedy_size=64)
    np.testing.assert_array_equal(H.aggregation(0), agg)
    c, f = H.permutation(0)
    np.testing.assert_array_equal(c, co)
    np.testing.assert_array_equal(f, fo)


def test_user_aggregation_equal_to_boxes_gives_the_box_topology():
    from paper_2005_01275_amd import _native as N
    prob = small_problem((9, 7), seed=2, box=(4, 3), m=3, n_levels=3, dirichlet=((0, 0), (1, 1)), permute=True)
    h = build_hierarchy(prob)
    user = np.concatenate([tr.agg for tr in h.transfers])
    Hb = host_handle(prob, 3, box=prob.box)
    Hu = host_handle(prob, 3, agg_kind=N.SPFAS_AGG_USER, user_agg=user)
    for l in range(2):
        np.testing.assert_array_equal(Hu.aggregation(l), Hb.aggregation(l))
        for a, b in zip(Hu.permutation(l), Hb.permutation(l)):
            np.testing.assert_array_equal(a, b)
        assert Hu.level_sizes(l + 1) == Hb.level_sizes(l + 1)


def test_malformed_user_aggregation_rejected():
    import paper_2005_01275_amd as pk
    from paper_2005_01275_amd import _native as N
    prob = small_problem((4, 4), seed=0, m=1)
    good0 = np.array([0, 0, 1, 1] * 2 + [2, 2, 3, 3] * 2)
    good1 = np.array([0, 0, 0, 0])
    cases = [
        (np.concatenate([good0, good1])[:-1], "shorter"),                   # too short
        (np.concatenate([np.where(good0 == 3, 4, good0), [0] * 5]), "unused"),  # id 3 unused
        (np.concatenate([np.array([0, 1, 0, 1] * 4), [0, 0]]), "connected"),  # checkerboard columns
        (np.concatenate([-good0, good1]), "negative"),
    ]
    for ua, what in cases:
        with pytest.raises(pk.SpfasError, match=what):
            host_handle(prob, 3, agg_kind=N.SPFAS_AGG_USER, user_agg=ua)
    H = host_handle(prob, 3, agg_kind=N.SPFAS_AGG_USER, user_agg=np.concatenate([good0, good1]))
    assert H.level_sizes(1)[0] == 4 and H.level_sizes(2)[0] == 1
