"""Pins of the oracle's fine level and single-level solvers against facts the
paper and the mathematics fix (CPU only)."""
import os

import numpy as np
import pytest
import scipy.optimize as so
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from problems import cartesian_mesh, Problem, small_problem, c1_problem
from oracle.fv import fine_level, half_transmissibilities, FineSystem
from oracle.levels import residual, jacobian, split
from oracle.coarsen import build_hierarchy
from oracle.solvers import Opts, single_level_solve, fas_solve, result_solve


def two_cell_problem():
    mesh = cartesian_mesh((2, 1), (1.0, 1.0), np.array([2.0, 8.0]), dirichlet=((0, 0),))
    gd = np.zeros(mesh.n_faces)
    gn = np.zeros(mesh.n_faces)
    gd[mesh.face_bc == 1] = 1.0
    # Neumann face on x = 2 (cell 1, outward normal +x)
    right = np.nonzero((mesh.face_bc == 2) & (mesh.face_normal[:, 0] > 0.5))[0]
    assert right.size == 1
    gn[right] = 0.5
    return Problem(mesh=mesh, alpha=0.5, source=np.array([0.25, -0.5]), g_dirichlet=gd,
                   g_neumann=gn, box=(2, 1), m=1, n_levels=1)


def test_two_cell_hand_values(golden_dir):
    vals = {}
    with open(os.path.join(golden_dir, "two_cell_residual.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    prob = two_cell_problem()
    TK, TL = half_transmissibilities(prob.mesh)
    assert TK[0] == pytest.approx(vals["Tb_interior_K"], rel=1e-15)
    assert TL[0] == pytest.approx(vals["Tb_interior_L"], rel=1e-15)
    dir_face = np.nonzero(prob.mesh.face_bc == 1)[0][0]
    assert TK[dir_face] == pytest.approx(vals["Tb_dirichlet"], rel=1e-15)
    lev, b0, fm = fine_level(prob)
    assert lev.n_flux == 2 and lev.n_p == 2
    x = np.array([0.3, -0.2, 0.4, -0.6])
    r = residual(lev, x, b0, prob.alpha)
    ref = [vals["r_sigma_interior"], vals["r_sigma_dirichlet"], vals["r_p0"], vals["r_p1"]]
    np.testing.assert_allclose(r, ref, rtol=1e-14, atol=1e-15)
    # the face-by-face transcription gives the same numbers
    fs = FineSystem(prob)
    rs, rp = fs.residual(x[:2], x[2:])
    np.testing.assert_allclose(np.concatenate([rs, rp]), ref, rtol=1e-14, atol=1e-15)


def cartesian_tb(prob):
    """Textbook half-transmissibility of an axis-aligned Cartesian mesh with
    diagonal K0: |eps| k_axis / (h_axis / 2)."""
    m = prob.mesh
    fc = m.face_cells
    axis = np.argmax(np.abs(m.face_normal), axis=1)
    h = np.array([np.ptp(np.unique(m.cell_centroid[:, a])) / max(1, np.unique(m.cell_centroid[:, a]).size - 1)
                  if np.unique(m.cell_centroid[:, a]).size > 1 else 2 * m.cell_centroid[0, a]
                  for a in range(m.dim)])
    kK = m.cell_k0[fc[:, 0], axis, axis]
    TK = m.face_area * kK / (h[axis] / 2)
    kL = np.where(fc[:, 1] >= 0, m.cell_k0[np.maximum(fc[:, 1], 0), axis, axis], 0.0)
    TL = m.face_area * kL / (h[axis] / 2)
    return TK, TL


@pytest.mark.parametrize("shape,aniso", [((5, 4), False), ((3, 4, 3), True), ((6, 3), True)])
def test_half_transmissibility_cartesian(shape, aniso):
    prob = small_problem(shape, seed=3, anisotropic=aniso, spacing=tuple(0.3 + 0.2 * i for i in range(len(shape))))
    TK, TL = half_transmissibilities(prob.mesh)
    tk, tl = cartesian_tb(prob)
    np.testing.assert_allclose(TK, tk, rtol=1e-13)
    np.testing.assert_allclose(TL, tl, rtol=1e-13)


def manufactured(prob, p_star, rng):
    """Discrete manufactured solution: sigma* from the TPFA flux with the
    harmonic transmissibility (eq. TPFA_flux), f := -D sigma* so that the
    mixed residual vanishes at (sigma*, p*)."""
    m = prob.mesh
    TK, TL = cartesian_tb(prob)
    fc = m.face_cells.astype(np.int64)
    a = prob.alpha
    kap = np.exp(a * p_star)
    gd = np.where(m.face_bc == 1, rng.standard_normal(m.n_faces) * 0.3, 0.0)
    gn = np.where(m.face_bc == 2, rng.standard_normal(m.n_faces) * 0.2, 0.0)
    sig = np.zeros(m.n_faces)
    inner = m.face_bc == 0
    K, L = fc[:, 0], fc[:, 1]
    UK = kap[K] * TK
    UL = np.where(inner, kap[np.maximum(L, 0)] * np.where(inner, TL, 1.0), 1.0)
    ups = 1.0 / (1.0 / UK + 1.0 / UL)
    sig[inner] = ups[inner] * (p_star[K[inner]] - p_star[L[inner]])
    d = m.face_bc == 1
    sig[d] = UK[d] * (p_star[K[d]] - gd[d])
    nn = m.face_bc == 2
    sig[nn] = -m.face_area[nn] * gn[nn]
    outflow = np.zeros(m.n_cells)
    np.add.at(outflow, K, sig)
    np.add.at(outflow, L[inner], -sig[inner])
    src = outflow / m.cell_volume          # eq. mass_balance_FV
    return Problem(mesh=m, alpha=a, source=src, g_dirichlet=gd, g_neumann=gn), sig


@pytest.mark.parametrize("shape,alpha", [((6, 5), 1.0), ((4, 3, 3), 2.0), ((8, 2), 0.5)])
def test_manufactured_solution_zero_residual(shape, alpha):
    rng = np.random.default_rng(11)
    base = small_problem(shape, seed=5, alpha=alpha, anisotropic=True,
                         dirichlet=((0, 0), (1, 1)))
    c = base.mesh.cell_centroid
    p_star = 0.3 * np.sin(2.0 * c[:, 0]) + 0.2 * np.cos(3.0 * c[:, 1])
    prob, sig_all = manufactured(base, p_star, rng)
    lev, b0, fm = fine_level(prob)
    x = np.concatenate([sig_all[fm.flux_face], p_star])
    r = residual(lev, x, b0, prob.alpha)
    scale = np.abs(b0).max() + np.abs(sig_all).max()
    assert np.abs(r).max() <= 1e-13 * scale
    # the solvers find it from x0 = 0
    h = build_hierarchy(prob, n_levels=1)
    xs, st = single_level_solve(h, Opts(newton=True, rtol=1e-13, atol=0.0, max_it=60))
    assert st.converged
    np.testing.assert_allclose(xs[lev.n_flux:], p_star, atol=1e-10)
    np.testing.assert_allclose(xs[:lev.n_flux], sig_all[fm.flux_face], atol=1e-10 * np.abs(sig_all).max())


def test_conservation_identity():
    """Sum over cells of r_p = sum of f - Dirichlet outflow, at any state
    (interior fluxes cancel in D); at the solution all the source leaves
    through the Dirichlet faces."""
    prob = small_problem((7, 6), seed=2, g_n_scale=0.4, g_d_scale=0.5)
    lev, b0, fm = fine_level(prob)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(lev.n)
    r = residual(lev, x, b0, prob.alpha)
    sig, p = split(lev, x)
    f = -b0[lev.n_flux:]
    dirf = lev.flux_kind == 1
    assert r[lev.n_flux:].sum() == pytest.approx(f.sum() - sig[dirf].sum(), abs=1e-12)
    h = build_hierarchy(prob, n_levels=1)
    xs = result_solve(h)
    sig_s = xs[:lev.n_flux]
    assert sig_s[dirf].sum() == pytest.approx(f.sum(), rel=1e-10, abs=1e-12)


def test_one_dimensional_chain_brute_force():
    """n x 1 channel, p = 0 at x = 0, inflow Q per unit area at x = L, no
    source: every face carries the same flux, so p follows cell by cell from
    scalar root finding on the TPFA flux (eq. TPFA_flux)."""
    n = 12
    rng = np.random.default_rng(4)
    k = np.exp(rng.standard_normal(n))
    h = 1.0 / n
    mesh = cartesian_mesh((n, 1), (h, 1.0), k, dirichlet=((0, 0),))
    gn = np.zeros(mesh.n_faces)
    right = np.nonzero((mesh.face_bc == 2) & (mesh.face_normal[:, 0] > 0.5))[0]
    Q = 0.8
    gn[right] = Q
    alpha = 1.3
    prob = Problem(mesh=mesh, alpha=alpha, source=np.zeros(n), g_dirichlet=np.zeros(mesh.n_faces),
                   g_neumann=gn, box=(4, 1), m=2, n_levels=2)
    kap = lambda p: np.exp(alpha * p)
    Tb = 1.0 * k / (h / 2)     # |eps| = 1 (unit height)
    p = np.zeros(n)
    # Dirichlet face: kappa(p0) Tb0 (p0 - 0) = Q (outflow through x = 0)
    p[0] = so.brentq(lambda s: kap(s) * Tb[0] * s - Q, 0.0, 50.0, xtol=1e-15, rtol=1e-15)
    for i in range(n - 1):
        def flux(s, i=i):
            u1, u2 = kap(p[i]) * Tb[i], kap(s) * Tb[i + 1]
            return 1.0 / (1.0 / u1 + 1.0 / u2) * (p[i] - s) + Q   # sigma_{i->i+1} = -Q
        p[i + 1] = so.brentq(flux, p[i], p[i] + 50.0, xtol=1e-15, rtol=1e-15)
    hier = build_hierarchy(prob)
    for solver in ("single", "fas"):
        for newton in (True, False):
            opts = Opts(newton=newton, rtol=1e-13, atol=0.0, max_it=200)
            x, st = (single_level_solve if solver == "single" else fas_solve)(hier, opts)
            assert st.converged, (solver, newton)
            np.testing.assert_allclose(x[hier.levels[0].n_flux:], p, rtol=1e-9, atol=1e-12)


def primal_residual(prob, p):
    """Cell-centred primal form: net outflow - (|tau| f + Neumann inflow),
    outflow through interior faces Upsilon_KL (p_K - p_L) with the harmonic
    mean of the kappa-scaled half transmissibilities and through Dirichlet
    faces kappa(p_K) Tb_K (p_K - g_D) (eqs. TPFA_flux, mass_balance_FV)."""
    m = prob.mesh
    TK, TL = cartesian_tb(prob)
    fc = m.face_cells.astype(np.int64)
    kap = np.exp(prob.alpha * p)
    out = np.zeros(m.n_cells)
    for f in range(m.n_faces):
        K, L = fc[f]
        if m.face_bc[f] == 0:
            u = 1.0 / (1.0 / (kap[K] * TK[f]) + 1.0 / (kap[L] * TL[f]))
            out[K] += u * (p[K] - p[L])
            out[L] -= u * (p[K] - p[L])
        elif m.face_bc[f] == 1:
            out[K] += kap[K] * TK[f] * (p[K] - prob.g_dirichlet[f])
        else:
            out[K] -= m.face_area[f] * prob.g_neumann[f]
    return out - m.cell_volume * prob.source


@pytest.mark.parametrize("shape,alpha,lin", [((4, 4), 1.0, False), ((3, 3, 2), 1.5, False),
                                             ((5, 4), 0.0, True)])
def test_primal_brute_force(shape, alpha, lin):
    """The mixed-form root equals the root of the primal TPFA equations
    found by a general-purpose root finder (alpha = 0: a sparse direct solve
    of the linear primal system)."""
    prob = small_problem(shape, seed=8, alpha=alpha, g_d_scale=0.3, g_n_scale=0.2, src_scale=2.0)
    hier = build_hierarchy(prob, n_levels=1)
    x = result_solve(hier)
    p_mixed = x[hier.levels[0].n_flux:]
    if lin:
        n = prob.mesh.n_cells
        r0 = primal_residual(prob, np.zeros(n))
        A = np.stack([primal_residual(prob, np.eye(n)[i]) - r0 for i in range(n)], axis=1)
        p_ref = spla.spsolve(sp.csr_matrix(A), -r0)
    else:
        sol = so.root(lambda p: primal_residual(prob, p), np.zeros(prob.mesh.n_cells), method="hybr",
                      options={"xtol": 1e-14})
        assert sol.success
        p_ref = sol.x
    np.testing.assert_allclose(p_mixed, p_ref, rtol=1e-9, atol=1e-11)


@pytest.mark.parametrize("newton", [True, False])
def test_jacobian_finite_differences_fine(newton):
    """Prop. 3 on level 0: analytic Newton Jacobian equals central finite
    differences of the residual; Picard drops exactly the kappa derivative."""
    prob = small_problem((4, 3), seed=9, alpha=1.7)
    lev, b0, fm = fine_level(prob)
    rng = np.random.default_rng(1)
    x = 0.3 * rng.standard_normal(lev.n)
    J = jacobian(lev, x, prob.alpha, True).toarray()
    eps = 1e-6
    Jfd = np.zeros_like(J)
    for j in range(lev.n):
        e = np.zeros(lev.n)
        e[j] = eps
        Jfd[:, j] = (residual(lev, x + e, b0, prob.alpha) - residual(lev, x - e, b0, prob.alpha)) / (2 * eps)
    np.testing.assert_allclose(J, Jfd, atol=1e-7 * np.abs(J).max())
    if not newton:
        JP = jacobian(lev, x, prob.alpha, False).toarray()
        nf = lev.n_flux
        np.testing.assert_allclose(JP[:, :nf], J[:, :nf])
        np.testing.assert_allclose(JP[nf:], J[nf:])
        np.testing.assert_allclose(JP[:nf, nf:], lev.D.T.toarray())


def test_c1_fas_matches_result_oracle():
    prob = c1_problem()
    h = build_hierarchy(prob)
    xs = result_solve(h)
    for newton in (True, False):
        x, st = fas_solve(h, Opts(newton=newton, rtol=1e-13, atol=0.0, max_it=100))
        assert st.converged
        assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_reduced_linear_form():
    """alpha = 0: the mixed-form root equals the reduced cell system of the
    remark after eq. FV_matrix, D M^{-1} D^T p = f - D M^{-1} g (with g_D != 0,
    which fixes the sign of the g term)."""
    from oracle.fv import linear_pressure
    prob = small_problem((7, 5), seed=3, alpha=0.0, g_d_scale=0.5, g_n_scale=0.3)
    h = build_hierarchy(prob, n_levels=1)
    x = result_solve(h)
    np.testing.assert_allclose(x[h.levels[0].n_flux:], linear_pressure(prob), atol=1e-12)


def test_c2_rate_constant_matches_calibration(golden_dir):
    """The stored well rate of the 60x220x85 workload is the one written by
    tests/golden/calibrate_c2_rate.py (which calls only the oracle)."""
    import json
    from problems.grids import C2_WELL_RATE
    with open(os.path.join(golden_dir, "c2_rate.json")) as fh:
        rec = json.load(fh)
    assert C2_WELL_RATE == pytest.approx(rec["rate"], rel=1e-12)
    assert rec["max_abs_p_at_rate_1"] * rec["rate"] == pytest.approx(0.5, rel=1e-12)
