"""Pins of the oracle's kappa families (CPU): the Richards-type conductivity
of Example 3 (eq. permeability_function_richards) evaluated at the shifted
pressure p - z, and the shift's coarse-level form (volume-weighted mean of
the level-0 field over each coarse cell)."""
import dataclasses

import numpy as np
import pytest
import scipy.optimize as so

from problems.grids import Problem, cartesian_mesh, richards_problem, small_problem
from oracle.coarsen import build_hierarchy
from oracle.fv import linear_pressure
from oracle.levels import Kappa, jacobian, residual
from oracle.solvers import Opts, fas_solve, single_level_solve, cap_value


def test_kappa_closed_forms():
    k = Kappa("richards", a=124.6, beta=1.77)
    psi = np.array([-300.0, -2.0, 0.0, 0.5, 40.0])
    np.testing.assert_array_equal(k.kinv(np.array([0.0])), [1.0])
    # 1/kappa = (a + |psi|^beta) / a, written out per value
    for v in psi:
        assert k.kinv(np.array([v]))[0] == pytest.approx((124.6 + abs(v) ** 1.77) / 124.6, rel=1e-15)
    # derivative against central differences
    for v in [-300.0, -2.0, 0.5, 40.0]:
        h = 1e-6 * max(1.0, abs(v))
        fd = (k.kinv(np.array([v + h]))[0] - k.kinv(np.array([v - h]))[0]) / (2 * h)
        assert k.dkinv(np.array([v]))[0] == pytest.approx(fd, rel=1e-7)
    e = Kappa("exp", alpha=1.3)
    np.testing.assert_allclose(e.kinv(psi[:3]), np.exp(-1.3 * psi[:3]), rtol=1e-15)
    np.testing.assert_allclose(e.dkinv(psi[:3]), -1.3 * np.exp(-1.3 * psi[:3]), rtol=1e-15)
    assert cap_value(k, 5.0) == np.inf and cap_value(e, 5.0) == pytest.approx(np.log(5.0) / 1.3)


def test_richards_chain_brute_force():
    """n x 1 column along x with the shift z = x (the height), p = 0 at x = 0
    and inflow Q at x = L: every face carries the same flux, so p follows
    cell by cell from scalar root finding on the TPFA flux with
    kappa(p_i - z_i) (eq. TPFA_flux)."""
    n = 12
    rng = np.random.default_rng(4)
    k = np.exp(0.5 * rng.standard_normal(n))
    h = 1.0 / n
    mesh = cartesian_mesh((n, 1), (h, 1.0), k, dirichlet=((0, 0),))
    gn = np.zeros(mesh.n_faces)
    right = np.nonzero((mesh.face_bc == 2) & (mesh.face_normal[:, 0] > 0.5))[0]
    Q = 0.3
    gn[right] = Q
    a, beta = 0.5, 2.0
    z = mesh.cell_centroid[:, 0].copy()
    prob = Problem(mesh=mesh, alpha=0.0, source=np.zeros(n), g_dirichlet=np.zeros(mesh.n_faces),
                   g_neumann=gn, box=(4, 1), m=2, n_levels=2, kappa_kind="richards", kappa_a=a,
                   kappa_beta=beta, shift=z)
    kap = lambda s, i: a / (a + abs(s - z[i]) ** beta)
    Tb = 1.0 * k / (h / 2)
    p = np.zeros(n)
    p[0] = so.brentq(lambda s: kap(s, 0) * Tb[0] * s - Q, 0.0, 2.0, xtol=1e-15, rtol=1e-15)
    for i in range(n - 1):
        def flux(s, i=i):
            u1, u2 = kap(p[i], i) * Tb[i], kap(s, i + 1) * Tb[i + 1]
            return 1.0 / (1.0 / u1 + 1.0 / u2) * (p[i] - s) + Q
        p[i + 1] = so.brentq(flux, p[i], p[i] + 1.0, xtol=1e-15, rtol=1e-15)
    hier = build_hierarchy(prob)
    for solver in ("single", "fas"):
        for newton in (True, False):
            opts = Opts(newton=newton, rtol=1e-13, atol=0.0, max_it=200)
            x, st = (single_level_solve if solver == "single" else fas_solve)(hier, opts)
            assert st.converged, (solver, newton)
            np.testing.assert_allclose(x[hier.levels[0].n_flux:], p, rtol=1e-9, atol=1e-12)


def test_constant_shift_is_a_rescaled_k0():
    """exp(alpha (p - z0)) = exp(-alpha z0) exp(alpha p): a constant shift
    is the same problem as K0 scaled by exp(-alpha z0) without shift, on
    every level (the coarse shift of a constant field is that constant)."""
    base = small_problem((8, 8), seed=6, alpha=1.2, box=(4, 4), m=2, n_levels=3, src_scale=2.0)
    z0 = 0.7
    shifted = dataclasses.replace(base, kappa_kind="exp", shift=np.full(base.mesh.n_cells, z0))
    scaled = dataclasses.replace(base, mesh=dataclasses.replace(base.mesh, cell_k0=base.mesh.cell_k0 *
                                                                np.exp(-1.2 * z0)))
    hs, hk = build_hierarchy(shifted), build_hierarchy(scaled)
    for lev in hs.levels[1:]:
        np.testing.assert_allclose(lev.shift, z0, rtol=1e-14)
    o = Opts(newton=True, rtol=1e-13, atol=0.0, max_it=60)
    xs, st1 = fas_solve(hs, o)
    xk, st2 = fas_solve(hk, o)
    assert st1.converged and st2.converged
    np.testing.assert_allclose(xs, xk, atol=1e-10 * np.abs(xk).max())


def test_coarse_shift_is_the_volume_mean():
    """The shift of a coarse cell is the volume-weighted mean of the level-0
    field over the level-0 cells it contains (computed here from the
    aggregation maps and the level-0 volumes only)."""
    prob = richards_problem(shape=(16, 8), size=(160.0, 80.0), box=(2, 2), n_levels=3, permute=True)
    h = build_hierarchy(prob)
    owner = np.arange(prob.mesh.n_cells)
    vol0 = prob.mesh.cell_volume
    for l, tr in enumerate(h.transfers):
        owner = tr.agg[owner]
        nc = h.levels[l + 1].n_cells
        want = np.bincount(owner, vol0 * prob.shift, nc) / np.bincount(owner, vol0, nc)
        np.testing.assert_allclose(h.levels[l + 1].shift, want, rtol=1e-13)


@pytest.mark.parametrize("medium", ["loam", "sand"])
def test_jacobian_finite_differences_richards(medium):
    """Props. 2-3 with the Richards family and a non-constant shift: the
    Newton Jacobian matches central finite differences on every level."""
    prob = richards_problem(shape=(8, 8), size=(80.0, 80.0), medium=medium, box=(2, 2), n_levels=3, m=3,
                            sigma=0.5, seed=3)
    h = build_hierarchy(prob)
    rng = np.random.default_rng(7)
    for l, lev in enumerate(h.levels):
        # states near the shift so that |psi| stays in the range of the problem
        x = 0.2 * rng.standard_normal(lev.n)
        zc = lev.shift if lev.shift is not None else 0.0
        if l == 0:
            x[lev.n_flux:] += zc - 5.0
        b = rng.standard_normal(lev.n)
        J = jacobian(lev, x, h.alpha, True).toarray()
        Jfd = np.zeros_like(J)
        for j in range(lev.n):
            e = np.zeros(lev.n)
            eps = 1e-6 * max(1.0, abs(x[j]))
            e[j] = eps
            Jfd[:, j] = (residual(lev, x + e, b, h.alpha) - residual(lev, x - e, b, h.alpha)) / (2 * eps)
        np.testing.assert_allclose(J, Jfd, atol=1e-6 * np.abs(J).max())


def test_richards_large_a_is_the_linear_problem():
    """a -> infinity gives kappa = 1: the root is the sparse-direct solution
    of the linear cell system (a library routine)."""
    prob = dataclasses.replace(richards_problem(shape=(12, 8), size=(120.0, 80.0), box=(4, 4), sigma=1.0),
                               kappa_a=1e30)
    h = build_hierarchy(prob)
    x, st = fas_solve(h, Opts(newton=True, rtol=1e-13, atol=0.0, max_it=20))
    assert st.converged and len(st.residuals) <= 3
    p = x[h.levels[0].n_flux:]
    np.testing.assert_allclose(p, linear_pressure(prob), atol=1e-9 * np.abs(p).max())


def test_richards_media_behaviour():
    """Example 3's observation on this stand-in section: on loam Picard,
    Newton and both FAS variants converge, FAS-Newton in fewer outer
    iterations than single-level Newton; on sand (n_max = 10) Newton and
    FAS-Newton converge while FAS-Picard does not."""
    loam = build_hierarchy(richards_problem(medium="loam"))
    its = {}
    for name, fn, newton in [("newton", single_level_solve, True), ("fas-newton", fas_solve, True),
                             ("fas-picard", fas_solve, False)]:
        x, st = fn(loam, Opts(newton=newton, max_it=100))
        assert st.converged, name
        its[name] = st.iterations
    assert its["fas-newton"] < its["newton"]
    sand = build_hierarchy(richards_problem(medium="sand"))
    for name, fn, newton, ok in [("newton", single_level_solve, True, True), ("fas-newton", fas_solve, True, True),
                                 ("fas-picard", fas_solve, False, False)]:
        x, st = fn(sand, Opts(newton=newton, max_it=60, bt_nmax=10))
        assert st.converged == ok, name
