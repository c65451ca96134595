"""Pins of the oracle's hierarchy (Section 3.1, Appendix A, Prop. 1,
Appendix B) and of the FAS cycle against properties the paper states or the
mathematics fixes (CPU only)."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from problems import small_problem, c1_problem
from oracle.coarsen import box_blocks, box_aggregate, renumber, build_hierarchy
from oracle.levels import residual, apply_A, M_of, pwc, jacobian, kinv, INTERIOR, BUBBLE, DIRICHLET
from oracle.solvers import (Opts, nonlinear_mg, result_solve, fas_solve, backtracking,
                            cap_scale, cap_value)


def test_box_blocks_rule():
    # remainder with fewer than half a box merges into the previous box
    assert [box_blocks(n, 4) for n in (85, 15, 14, 5, 2, 1, 16, 60, 220, 55, 21)] == \
        [21, 4, 4, 1, 1, 1, 4, 15, 55, 14, 5]


def test_box_aggregate_hand():
    shape = (7, 5)
    idx = np.arange(35)
    agg, cshape = box_aggregate(shape, idx, (4, 2))
    assert cshape == (2, 3)
    i, j = idx % 7, idx // 7
    bx = np.minimum(i // 4, 1)
    by = np.minimum(j // 2, 2)
    np.testing.assert_array_equal(agg, bx + 2 * by)


def test_renumber_groups():
    prob = small_problem((8, 6), seed=1, box=(4, 3), m=2, n_levels=3, dirichlet=((0, 0), (1, 1)))
    h = build_hierarchy(prob)
    for l, tr in enumerate(h.transfers):
        lev = h.levels[l]
        agg = tr.agg
        co, fo = tr.cell_order, tr.flux_order
        assert sorted(co) == list(range(lev.n_cells))
        assert sorted(fo) == list(range(lev.n_flux))
        a = agg[co]
        assert np.all(np.diff(a) >= 0)
        for A in np.unique(a):
            seg = co[a == A]
            assert np.all(np.diff(seg) > 0)
        # flux groups: inside-aggregate, then interfaces, then Dirichlet
        kind = lev.flux_kind[fo]
        c1 = lev.flux_cells[fo, 0]
        c2 = lev.flux_cells[fo, 1]
        a1 = agg[c1]
        a2 = np.where(c2 >= 0, agg[np.maximum(c2, 0)], -1)
        g = np.where((kind == BUBBLE) | ((kind == INTERIOR) & (a1 == a2)), 0,
                     np.where(kind == INTERIOR, 1, 2))
        assert np.all(np.diff(g) >= 0)


def hier(prob):
    return build_hierarchy(prob)


CASES = [
    dict(shape=(8, 8), box=(4, 4), m=2, n_levels=3, seed=1),
    dict(shape=(8, 4, 4), box=(2, 2, 2), m=3, n_levels=3, seed=2, anisotropic=True),
    dict(shape=(10, 7), box=(4, 3), m=3, n_levels=3, seed=3, dirichlet=((0, 0), (1, 1))),
]


@pytest.fixture(scope="module", params=range(len(CASES)))
def case(request):
    kw = dict(CASES[request.param])
    prob = small_problem(**kw)
    return prob, hier(prob)


def test_eigen_invariants(case):
    prob, h = case
    for l, tr in enumerate(h.transfers):
        lev = h.levels[l]
        for ad in tr.aggs:
            lam = ad.lam
            assert abs(lam[0]) <= 1e-11 * max(1.0, abs(lam[-1]))
            v0 = ad.V[:, 0]
            one = lev.ones[ad.pd]
            cosang = abs(v0 @ one) / (np.linalg.norm(one) * np.linalg.norm(v0))
            assert cosang == pytest.approx(1.0, abs=1e-10)
            if ad.pd.size > 1:
                assert lam[1] > 1e-10 * lam[-1]           # connected aggregate
            P = ad.P
            np.testing.assert_allclose(P.T @ P, np.eye(P.shape[1]), atol=1e-13)
            np.testing.assert_allclose(P[:, 0], one / np.linalg.norm(one), atol=1e-15)


def test_uniform_box_eigenvalues_closed_form():
    """Uniform k: the aggregate Laplacian is a weighted grid graph, whose
    spectrum is the Kronecker sum of path-graph spectra 2 w (1 - cos(i pi / n))."""
    for shape, box, spacing in [((8, 8), (4, 4), (0.5, 0.25)), ((4, 6, 4), (4, 3, 2), (1.0, 0.5, 0.2))]:
        prob = small_problem(shape, seed=0, sigma=0.0, box=box, m=2, n_levels=2, spacing=spacing)
        h = hier(prob)
        dim = len(shape)
        h_ = np.array(spacing)
        area = np.prod(h_) / h_
        w = area / h_   # harmonic mean of two equal half-transmissibilities |eps| k/(h/2), k = 1
        grids = np.meshgrid(*[2 * w[a] * (1 - np.cos(np.arange(box[a]) * math.pi / box[a]))
                              for a in range(dim)], indexing="ij")
        ref = np.sort(sum(g.ravel() for g in grids))
        for ad in h.transfers[0].aggs:
            np.testing.assert_allclose(ad.lam, ref, rtol=1e-11, atol=1e-11 * ref[-1])


def test_projection_identities(case):
    """Q P = I (Section 3.1) and the commutativity D^{l+1} Q_sigma = Q_p D^l."""
    prob, h = case
    for l, tr in enumerate(h.transfers):
        lev, clev = h.levels[l], h.levels[l + 1]
        I_s = (tr.Q_sig @ tr.P_sig).toarray()
        np.testing.assert_allclose(I_s, np.eye(clev.n_flux), atol=1e-11)
        I_p = (tr.Q_p @ tr.P_p).toarray()
        np.testing.assert_allclose(I_p, np.eye(clev.n_p), atol=1e-13)
        lhs = (clev.D @ tr.Q_sig).toarray()
        rhs = (tr.Q_p @ lev.D).toarray()
        np.testing.assert_allclose(lhs, rhs, atol=1e-10 * np.abs(rhs).max())
        # Pi = P Q is a projection
        rng = np.random.default_rng(0)
        x = rng.standard_normal(lev.n)
        y = tr.P(tr.Q(x, lev.n_flux), clev.n_flux)
        z = tr.P(tr.Q(y, lev.n_flux), clev.n_flux)
        np.testing.assert_allclose(z, y, atol=1e-10 * np.abs(y).max())


def test_coarse_divergence_galerkin_and_structure(case):
    """D^{l+1} assembled from local blocks equals P_p^T D^l P_sigma; row PV
    holds c_{A,F} on interfaces and 0 on bubbles; the NPV rows are the
    identity on the aggregate's own bubbles."""
    prob, h = case
    for l, tr in enumerate(h.transfers):
        lev, clev = h.levels[l], h.levels[l + 1]
        G = (tr.P_p.T @ lev.D @ tr.P_sig).toarray()
        np.testing.assert_allclose(clev.D.toarray(), G, atol=1e-11 * np.abs(G).max())
        for A in range(clev.n_cells):
            Dl = clev.D_loc[A]
            lf = clev.cell_flux[A]
            kinds = clev.flux_kind[lf]
            bub = kinds == BUBBLE
            np.testing.assert_allclose(Dl[0, bub], 0.0, atol=1e-12)
            assert np.all(np.abs(Dl[0, ~bub]) > 1e-12)
            np.testing.assert_allclose(Dl[1:, ~bub], 0.0, atol=1e-11)
            np.testing.assert_allclose(Dl[1:, bub], np.eye(int(bub.sum())), atol=1e-11)
        # 1^l lies in the kernel of D^T on interior (non-Dirichlet) unknowns
        t = lev.D.T @ lev.ones
        np.testing.assert_allclose(t[lev.flux_kind != DIRICHLET], 0.0, atol=1e-12)


def test_pv_traces_unit_flux(case):
    prob, h = case
    for l, tr in enumerate(h.transfers):
        lev = h.levels[l]
        for (A, B), t in zip(tr.coarse_faces, tr.traces):
            ad = tr.aggs[A]
            F = ad.faces[B] if B >= 0 else ad.dir_dofs
            pos = [list(ad.dofs).index(j) for j in F]
            outflow = -(lev.ones[ad.pd] @ ad.D[:, pos] @ t)
            assert outflow == pytest.approx(1.0, abs=1e-12)


def test_prop1_local_assembly_equals_galerkin(case):
    """Prop. 1: the coarse M assembled from static local matrices scaled by
    1/kappa of the aggregate pressure equals P_sigma^T M^l P_sigma with M^l
    evaluated at that piecewise-constant pressure (proof in Appendix C)."""
    prob, h = case
    rng = np.random.default_rng(5)
    a = prob.alpha
    for l, tr in enumerate(h.transfers):
        lev, clev = h.levels[l], h.levels[l + 1]
        pc = 0.5 * rng.standard_normal(clev.n_p)
        pbar = pwc(clev, pc)                       # one value per aggregate
        s_fine = np.repeat(0.0, lev.n_cells)
        s_fine = kinv(pbar[tr.agg], a)             # every level-l cell of A sees kappa(pbar_A)
        Mf = (lev.W.T @ lev.Mhat @ sp.diags(lev.Wsp @ s_fine) @ lev.W)
        G = (tr.P_sig.T @ Mf @ tr.P_sig).toarray()
        Mloc = M_of(clev, pc, a).toarray()
        np.testing.assert_allclose(Mloc, G, atol=1e-11 * np.abs(G).max())


def test_linear_limit_galerkin():
    """alpha = 0: A^{l+1} = P^T A^l P exactly (eq. coarse-saddle)."""
    prob = small_problem((8, 8), seed=4, alpha=0.0, box=(4, 4), m=3, n_levels=3)
    h = hier(prob)
    rng = np.random.default_rng(2)
    for l, tr in enumerate(h.transfers):
        lev, clev = h.levels[l], h.levels[l + 1]
        xc = rng.standard_normal(clev.n)
        lhs = apply_A(clev, xc, 0.0)
        rhs = tr.R(apply_A(lev, tr.P(xc, clev.n_flux), 0.0), lev.n_flux)
        np.testing.assert_allclose(lhs, rhs, atol=1e-11 * np.abs(rhs).max())


def test_pwc_projector(case):
    """Appendix B: Pi~(1^l) = 1 on every cell, and a level-0 pressure that is
    constant on each coarse cell is returned unchanged by Pi~ Q."""
    prob, h = case
    for l in range(1, len(h.levels)):
        lev = h.levels[l]
        np.testing.assert_allclose(pwc(lev, lev.ones), 1.0, atol=1e-13)
    rng = np.random.default_rng(3)
    fine_cells = np.arange(h.levels[0].n_cells)
    owner = fine_cells.copy()
    for l, tr in enumerate(h.transfers):
        owner = tr.agg[owner]
        vals = rng.standard_normal(h.levels[l + 1].n_cells)
        p = vals[owner]
        for t in h.transfers[:l + 1]:
            p = t.Q_p @ p
        np.testing.assert_allclose(pwc(h.levels[l + 1], p), vals, atol=1e-12)


@pytest.mark.parametrize("newton", [True, False])
def test_coarse_jacobian_finite_differences(case, newton):
    """Prop. 3 on coarse levels: J matches central finite differences."""
    prob, h = case
    rng = np.random.default_rng(7)
    for l in range(1, len(h.levels)):
        lev = h.levels[l]
        x = 0.2 * rng.standard_normal(lev.n)
        b = rng.standard_normal(lev.n)
        J = jacobian(lev, x, prob.alpha, True).toarray()
        eps = 1e-6
        Jfd = np.zeros_like(J)
        for j in range(lev.n):
            e = np.zeros(lev.n)
            e[j] = eps
            Jfd[:, j] = (residual(lev, x + e, b, prob.alpha) - residual(lev, x - e, b, prob.alpha)) / (2 * eps)
        np.testing.assert_allclose(J, Jfd, atol=1e-7 * np.abs(J).max())


def test_fas_fixed_point(case):
    """r(x*) = 0 gives b^{l+1} = A^{l+1}(Q x*), so the V-cycle leaves x* in place."""
    prob, h = case
    xs = result_solve(h)
    for newton in (True, False):
        y = nonlinear_mg(h, 0, xs.copy(), h.b0, Opts(newton=newton))
        assert np.linalg.norm(y - xs) <= 1e-11 * np.linalg.norm(xs)


def test_fas_converges_to_root(case):
    prob, h = case
    xs = result_solve(h)
    for newton in (True, False):
        x, st = fas_solve(h, Opts(newton=newton, rtol=1e-13, atol=0.0, max_it=60))
        assert st.converged
        assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


# ------------------------------------------------------------- Alg. 1, cap

def scripted(table):
    """Residual norm as a function of the step fraction (x is a scalar s)."""
    return lambda y: table[round(float(y), 12)]


def test_backtracking_transcription():
    # accept the full step when it reduces the residual
    t = {0.0: 1.0, 1.0: 0.5}
    x, s, n = backtracking(scripted(t), 0.0, 1.0, 4, 0.9)
    assert (s, n) == (1.0, 0)
    # halve while the residual grows and halving keeps paying off
    t = {0.0: 1.0, 1.0: 4.0, 0.5: 2.0, 0.25: 0.9}
    x, s, n = backtracking(scripted(t), 0.0, 1.0, 4, 0.9)
    assert (s, n) == (0.25, 2)
    # stop when halving gains less than the factor theta: keep the larger step
    t = {0.0: 1.0, 1.0: 2.0, 0.5: 1.95}
    x, s, n = backtracking(scripted(t), 0.0, 1.0, 4, 0.9)
    assert (s, n) == (1.0, 0)
    # at most n_max halvings, even if the residual is still larger
    t = {0.0: 1.0, 1.0: 64.0, 0.5: 32.0, 0.25: 16.0, 0.125: 8.0, 0.0625: 4.0, 0.03125: 2.0}
    x, s, n = backtracking(scripted(t), 0.0, 1.0, 4, 0.9)
    assert (s, n) == (0.0625, 4)


def test_backtracking_non_finite_trials():
    inf, nan = math.inf, math.nan
    # an overflowing full step is halved like a very large residual
    t = {0.0: 1.0, 1.0: inf, 0.5: nan, 0.25: 0.8}
    x, s, n = backtracking(scripted(t), 0.0, 1.0, 4, 0.9)
    assert (s, n) == (0.25, 2)
    # every trial overflows: the step is rejected and x is returned unchanged
    t = {0.0: 1.0, 1.0: inf, 0.5: inf, 0.25: nan, 0.125: inf, 0.0625: inf}
    x, s, n = backtracking(scripted(t), 0.0, 1.0, 4, 0.9)
    assert (s, n) == (0.0, 4) and float(x) == 0.0
    # a finite but larger residual is still preferred to an overflow
    t = {0.0: 1.0, 1.0: inf, 0.5: 3.0, 0.25: 2.9}
    x, s, n = backtracking(scripted(t), 0.0, 1.0, 4, 0.9)
    assert (s, n) == (0.5, 1)


def test_cap():
    cap = cap_value(1.0, 5.0)
    assert cap == pytest.approx(math.log(5.0))
    assert cap_scale(np.array([0.1, -0.2]), cap) == 1.0
    assert cap_scale(np.array([0.1, -2 * cap]), cap) == pytest.approx(0.5)
    assert math.isinf(cap_value(0.0, 5.0))
    assert cap_value(2.0, 1.5) == pytest.approx(math.log(1.5) / 2.0)


# ------------------------------------------------------------- eigenvector count by threshold

def test_eig_count_hand_cases():
    from oracle.coarsen import eig_count
    lam = np.array([0.0, 0.05, 0.09, 0.1, 0.5, 1.0])
    assert eig_count(lam, 6, 0.1) == 4          # 0, 0.05, 0.09, 0.1 <= 0.1 * 1.0
    assert eig_count(lam, 3, 0.1) == 3          # upper clamp m
    assert eig_count(np.array([0.0, 0.5, 1.0]), 6, 0.1) == 2     # lower clamp m_min
    assert eig_count(np.array([0.0, 0.5, 1.0]), 6, 0.1, m_min=1) == 1
    assert eig_count(np.array([0.0]), 6, 0.1) == 1               # at most the unknowns of the aggregate
    assert eig_count(lam, 5, 0.0) == 5          # threshold off: the uniform count
    assert eig_count(np.r_[np.linspace(0.0, 0.01, 9), 1.0], 6, 0.1) == 6          # 9 below: upper clamp


def test_threshold_count_on_uniform_boxes_closed_form():
    """Uniform k: the eigenvalues of each box are the Kronecker sums of the
    path-graph spectra, so the count kept by the threshold rule is known in
    closed form; every aggregate of the hierarchy keeps exactly that many,
    and the coarse level has that many pressure unknowns per cell."""
    for shape, box, spacing, thr in [((8, 8), (4, 4), (0.5, 0.25), 0.1), ((8, 8), (4, 4), (0.5, 0.25), 0.15),
                                     ((8, 8), (4, 4), (0.25, 0.25), 0.3), ((4, 6, 4), (4, 3, 2), (1.0, 0.5, 0.2), 0.1),
                                     ((4, 6, 4), (4, 3, 2), (1.0, 0.5, 0.2), 0.06)]:
        prob = small_problem(shape, seed=0, sigma=0.0, box=box, m=6, n_levels=2, spacing=spacing)
        h = build_hierarchy(prob, eig_threshold=thr, m_min=2)
        dim = len(shape)
        h_ = np.array(spacing)
        w = (np.prod(h_) / h_) / h_
        grids = np.meshgrid(*[2 * w[a] * (1 - np.cos(np.arange(box[a]) * math.pi / box[a]))
                              for a in range(dim)], indexing="ij")
        ref = np.sort(sum(g.ravel() for g in grids))
        want = min(max(int(np.sum(ref <= thr * ref[-1] * (1 + 1e-12))), 2), 6)
        counts = np.diff(h.levels[1].pdof_ptr)
        assert np.all(counts == want), (shape, thr, counts, want)


def test_threshold_hierarchy_invariants_and_root():
    """Heterogeneous k, counts varying per aggregate: Q_p P_p = I, the
    commuting property, and FAS reaching the same root as with a fixed m."""
    prob = small_problem((12, 12), seed=8, sigma=1.5, box=(4, 4), m=6, n_levels=3, alpha=1.0, src_scale=3.0)
    h = build_hierarchy(prob, eig_threshold=0.1, m_min=2)
    counts = np.diff(h.levels[1].pdof_ptr)
    assert counts.min() >= 2 and counts.max() <= 6 and counts.min() < counts.max()
    for l, tr in enumerate(h.transfers):
        lev, clev = h.levels[l], h.levels[l + 1]
        np.testing.assert_allclose((tr.Q_p @ tr.P_p).toarray(), np.eye(clev.n_p), atol=1e-12)
        np.testing.assert_allclose((tr.Q_sig @ tr.P_sig).toarray(), np.eye(clev.n_flux), atol=1e-11)
        rhs = (tr.Q_p @ lev.D).toarray()
        np.testing.assert_allclose((clev.D @ tr.Q_sig).toarray(), rhs, atol=1e-10 * np.abs(rhs).max())
    xs = result_solve(h)
    x, st = fas_solve(h, Opts(newton=True, rtol=1e-13, atol=0.0, max_it=60))
    assert st.converged
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
