"""Oracle pins for nonlinear cascadic multigrid (Section 4.2, Table 4),
checked against what the method reduces to or must satisfy: with one level
it is single-level Newton; on the linear problem (alpha = 0) each level is
solved by one exact Newton step and the fine state is the direct solution
of the fine linear system; the coarse right-hand sides R b^l are the FAS
right-hand sides at the zero state (A^l(0) = 0 on every level); and on a
nonlinear problem the result meets the stopping rule at the root x*."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

from problems import small_problem
from oracle.coarsen import build_hierarchy
from oracle.levels import residual, apply_A, jacobian
from oracle.solvers import Opts, cascadic_solve, single_level_solve, result_solve, norm


def test_cascadic_one_level_is_single_level_newton():
    prob = small_problem((6, 5), seed=4, box=(3, 5), m=2, n_levels=1, alpha=1.5, src_scale=2.0)
    h = build_hierarchy(prob)
    o = Opts(newton=True, rtol=1e-10, atol=0.0, cap_c=prob.dp_cap_c)
    xc, stc = cascadic_solve(h, o)
    xs, sts = single_level_solve(h, o)
    assert stc.level_steps == [sts.iterations]
    assert np.array_equal(xc, xs)


def test_cascadic_linear_problem_one_step_per_level():
    prob = small_problem((9, 6), seed=2, box=(3, 3), m=2, n_levels=3, alpha=0.0, g_d_scale=0.3)
    h = build_hierarchy(prob)
    o = Opts(newton=True, rtol=1e-10, atol=0.0, cap_c=prob.dp_cap_c)
    x, st = cascadic_solve(h, o)
    assert st.converged and st.level_steps == [1, 1, 1], st
    lev = h.levels[0]
    # direct solve of the linear fine system A x = b0 (kappa = 1)
    J = jacobian(lev, np.zeros(lev.n), 0.0, True)
    x_lin = spla.spsolve(J.tocsc(), h.b0)
    assert np.allclose(x, x_lin, rtol=1e-9, atol=1e-12 * np.abs(x_lin).max())
    # every level solved its own linear problem with the restricted right-hand side R b^{l-1}
    b = h.b0
    for l in range(1, len(h.levels)):
        tr, fine = h.transfers[l - 1], h.levels[l - 1]
        b = np.concatenate([tr.P_sig.T @ b[:fine.n_flux], tr.P_p.T @ b[fine.n_flux:]])
        lev = h.levels[l]
        Jl = jacobian(lev, np.zeros(lev.n), 0.0, True)
        xl = spla.spsolve(Jl.tocsc(), b)
        assert np.allclose(st.level_x[l], xl, rtol=1e-9, atol=1e-12 * np.abs(xl).max())


def test_cascadic_coarse_rhs_is_the_fas_rhs_at_zero():
    prob = small_problem((12, 8), seed=2, box=(4, 4), m=3, n_levels=3, alpha=1.5, g_d_scale=0.3, g_n_scale=0.2,
                         dirichlet=((0, 0), (1, 1)))
    h = build_hierarchy(prob)
    b = h.b0
    for l in range(len(h.levels) - 1):
        lev, clev, tr = h.levels[l], h.levels[l + 1], h.transfers[l]
        assert np.array_equal(apply_A(lev, np.zeros(lev.n), h.alpha), np.zeros(lev.n))
        r0 = residual(lev, np.zeros(lev.n), b, h.alpha)
        assert np.array_equal(r0, -b)
        xc = tr.Q(np.zeros(lev.n), lev.n_flux)
        b_fas = apply_A(clev, xc, h.alpha) - tr.R(r0, lev.n_flux)
        b_next = tr.R(b, lev.n_flux)
        assert np.allclose(b_fas, b_next, rtol=0.0, atol=1e-15 * max(1.0, np.abs(b_next).max()))
        b = b_next


@pytest.mark.parametrize("newton", [True, False])
def test_cascadic_reaches_the_root(newton):
    prob = small_problem((12, 8), seed=2, box=(4, 4), m=3, n_levels=3, alpha=1.5, src_scale=2.0, g_d_scale=0.3,
                         g_n_scale=0.2, dirichlet=((0, 0), (1, 1)))
    h = build_hierarchy(prob)
    o = Opts(newton=newton, rtol=1e-10, atol=0.0, cap_c=prob.dp_cap_c, max_it=200)
    x, st = cascadic_solve(h, o)
    assert st.converged and all(st.level_converged), st
    assert norm(residual(h.levels[0], x, h.b0, h.alpha)) <= 1e-10 * norm(h.b0)
    xs = result_solve(h)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    # the fine level starts from the prolongated coarse solution: fewer steps than from zero
    _, sts = single_level_solve(h, o)
    assert st.level_steps[0] <= sts.iterations
