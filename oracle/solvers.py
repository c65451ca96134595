"""Nonlinear solvers (oracle; test infrastructure only).

* ``backtracking``  -- Alg. 1 (n_max = 4, theta = 0.9 in Section 4).
* ``cap``           -- the exponential-kappa step limit of Section 4.1: if
                       max|dp| > ln(c)/alpha the whole step is scaled so that
                       max|dp| = ln(c)/alpha; applied before Alg. 1 at every
                       smoothing step.  On a coarse level the quantity kappa
                       sees is the aggregate-average pressure, so the cap is
                       read as acting on Pi~ dp there (on level 0 Pi~ = I).
* ``smooth``        -- one Picard or Newton step with an exact linear solve
                       (Section 3.3), then the cap, then Alg. 1.
* ``nonlinear_mg``  -- the FAS V-cycle of Alg. 2 with coarse right-hand side
                       b^{l+1} = A^{l+1}(Q x) - R(A^l(x) - b^l) (eq.
                       coarse_level_residual); the coarsest level takes at
                       most 10 smoothing steps, stopping early on convergence
                       (Section 4).  A step that Alg. 1 rejected (s = 0: the
                       chosen trial was not finite) leaves the state as it
                       was, so every further step would repeat it; the loop
                       stops there too.  A step that Alg. 1 accepted while
                       it raised the residual does not stop the loop.
* ``cascadic_solve`` -- nonlinear cascadic multigrid (Section 4.2, Table 4):
                       the right-hand side restricted level by level
                       (b^{l+1} = R b^l), the coarsest problem solved from
                       zero with smoothing steps until it converges, its
                       solution prolongated (P) as the initial guess of the
                       next finer level, and so on up to level 0.  Reading:
                       each level stops on the same rule as the fine level,
                       relative to the residual of the zero state
                       (||r^l(0)|| = ||b^l||), and takes at most max_it steps;
                       like the coarsest level of the V-cycle, a level also
                       stops after a step that Alg. 1 rejected (s = 0, state
                       unchanged).
* ``fas_solve`` / ``single_level_solve`` -- outer loops with the stopping rule
  of Section 4: relative residual below rtol or absolute below atol (2-norm
  of the whole residual vector; relative to the residual of the initial
  guess x0 = 0).  A V-cycle may stop right after the fine pre-smoothing when
  that already meets the rule (footnote of Table 1).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List

import numpy as np
import scipy.sparse.linalg as spla

from .levels import residual, jacobian, pwc, apply_A, Kappa


@dataclasses.dataclass
class Opts:
    newton: bool = True
    rtol: float = 1e-8
    atol: float = 1e-10
    max_it: int = 100
    bt_nmax: int = 4
    bt_theta: float = 0.9
    cap_c: float = 5.0            # max |dp| <= ln(cap_c)/alpha; <= 1 disables
    coarsest_max: int = 10
    coarsest_atol: float = None   # absolute floor of the coarsest level's test; None: atol


@dataclasses.dataclass
class Stats:
    iterations: int = 0
    residuals: List[float] = dataclasses.field(default_factory=list)
    stopped_after_presmooth: bool = False
    bt_steps: int = 0
    converged: bool = False


def norm(v):
    return float(np.sqrt(np.dot(v, v)))


def backtracking(rnorm_of, x, dx, nmax, theta, r_x=None):
    """Alg. 1: halve s while ||r(x + s dx)|| > ||r(x)|| and fewer than n_max
    halvings were taken; stop halving when the halved step would not reduce
    the residual by more than the factor theta.  Returns (x_new, s, halvings).

    The paper does not consider trial points where kappa overflows.  Reading
    taken here: a non-finite trial residual counts as +infinity (so the
    comparisons above stay well defined), and when the trial finally chosen
    is still non-finite the step is rejected (s = 0, x unchanged)."""
    def rn(y):
        v = float(rnorm_of(y))
        return v if math.isfinite(v) else math.inf

    rx = rn(x) if r_x is None else r_x
    s = 1.0
    n = 0
    r_s = rn(x + s * dx)
    while r_s > rx and n < nmax:
        r_half = rn(x + 0.5 * s * dx)
        if r_half > theta * r_s:
            break
        s *= 0.5
        n += 1
        r_s = r_half
    if r_s == math.inf:
        return np.copy(x), 0.0, n
    return x + s * dx, s, n


def cap_scale(dpbar: np.ndarray, cap: float) -> float:
    """Scale factor that limits max|dp| to cap (1 if already within)."""
    if not np.isfinite(cap) or dpbar.size == 0:
        return 1.0
    mx = float(np.max(np.abs(dpbar)))
    return cap / mx if mx > cap else 1.0


def cap_value(alpha, c: float) -> float:
    """ln(c)/alpha for kappa = exp(alpha p) (Section 4.1); other kappa
    families take no cap (Example 3 uses Alg. 1 alone)."""
    if isinstance(alpha, Kappa):
        if alpha.kind != "exp":
            return math.inf
        alpha = alpha.alpha
    if alpha <= 0 or c <= 1:
        return math.inf
    return math.log(c) / alpha


def smooth_step(level, x, b, alpha, opts: Opts, stats: Stats = None):
    """One Picard or Newton step on a level (Section 3.3).  Picard solves
    [M(Pi~p) D^T; D 0] x_P = b and steps along x_P - x, which is the same as
    solving that matrix against -r(x); Newton solves J dx = -r(x).
    Returns (x_new, s): s is the step length Alg. 1 chose, 0 when it
    rejected the step (x_new is then x)."""
    r = residual(level, x, b, alpha)
    J = jacobian(level, x, alpha, opts.newton)
    dx = spla.spsolve(J, -r)
    cap = cap_value(alpha, opts.cap_c)
    dx = dx * cap_scale(pwc(level, dx[level.n_flux:]), cap)
    rn = lambda y: norm(residual(level, y, b, alpha))
    xn, s, n = backtracking(rn, x, dx, opts.bt_nmax, opts.bt_theta, r_x=norm(r))
    if stats is not None:
        stats.bt_steps += n
    return xn, s


def smooth(level, x, b, alpha, opts: Opts, stats: Stats = None):
    """``smooth_step`` without the step length."""
    return smooth_step(level, x, b, alpha, opts, stats)[0]


def coarsest_solve(level, x, b, alpha, opts: Opts, stats=None):
    """Section 4: at most ``coarsest_max`` smoothing steps, fewer when the
    level residual meets rtol (relative to its value on entry) or the
    absolute tolerance (the paper's pair: relative 1e-8 or absolute 1e-10;
    ``coarsest_atol`` when set, else atol).  The loop also ends after a step
    Alg. 1 rejected (s = 0): the state is then unchanged and the next step
    would be the same one."""
    r = norm(residual(level, x, b, alpha))
    atol = opts.atol if opts.coarsest_atol is None else opts.coarsest_atol
    tol = max(opts.rtol * r, atol)
    for _ in range(opts.coarsest_max):
        if r <= tol:
            break
        x, s = smooth_step(level, x, b, alpha, opts, stats)
        if s == 0.0:
            break
        r = norm(residual(level, x, b, alpha))
    return x


def nonlinear_mg(h, l, x, b, opts: Opts, stats: Stats = None, stop_tol=None):
    """Alg. 2.  ``stop_tol`` (level 0 only) returns right after
    pre-smoothing when the fine residual already meets the stopping rule."""
    lev = h.levels[l]
    a = h.alpha
    if l == len(h.levels) - 1:
        return coarsest_solve(lev, x, b, a, opts, stats)
    x = smooth(lev, x, b, a, opts, stats)
    r = residual(lev, x, b, a)
    if stop_tol is not None and norm(r) <= stop_tol:
        if stats is not None:
            stats.stopped_after_presmooth = True
        return x
    tr = h.transfers[l]
    clev = h.levels[l + 1]
    xc = tr.Q(x, lev.n_flux)
    bc = apply_A(clev, xc, a) - tr.R(r, lev.n_flux)
    yc = nonlinear_mg(h, l + 1, xc, bc, opts, stats)
    dx = tr.P(yc - xc, clev.n_flux)
    rn = lambda y: norm(residual(lev, y, b, a))
    x, _, n = backtracking(rn, x, dx, opts.bt_nmax, opts.bt_theta, r_x=norm(r))
    if stats is not None:
        stats.bt_steps += n
    x = smooth(lev, x, b, a, opts, stats)
    return x


def fas_solve(h, opts: Opts, x0=None):
    lev = h.levels[0]
    x = np.zeros(lev.n) if x0 is None else x0.copy()
    st = Stats()
    r0 = norm(residual(lev, x, h.b0, h.alpha))
    tol = max(opts.rtol * r0, opts.atol)
    st.residuals.append(r0)
    for _ in range(opts.max_it):
        if st.residuals[-1] <= tol:
            st.converged = True
            break
        st.stopped_after_presmooth = False
        x = nonlinear_mg(h, 0, x, h.b0, opts, st, stop_tol=tol)
        st.iterations += 1
        st.residuals.append(norm(residual(lev, x, h.b0, h.alpha)))
    else:
        st.converged = st.residuals[-1] <= tol
    return x, st


def single_level_solve(h, opts: Opts, x0=None):
    """Single-level Picard or Newton (Section 2.2), same cap and Alg. 1."""
    lev = h.levels[0]
    x = np.zeros(lev.n) if x0 is None else x0.copy()
    st = Stats()
    r0 = norm(residual(lev, x, h.b0, h.alpha))
    tol = max(opts.rtol * r0, opts.atol)
    st.residuals.append(r0)
    for _ in range(opts.max_it):
        if st.residuals[-1] <= tol:
            st.converged = True
            break
        x = smooth(lev, x, h.b0, h.alpha, opts, st)
        st.iterations += 1
        st.residuals.append(norm(residual(lev, x, h.b0, h.alpha)))
    else:
        st.converged = st.residuals[-1] <= tol
    return x, st


@dataclasses.dataclass
class CascadicStats:
    level_steps: List[int] = dataclasses.field(default_factory=list)   # per level, finest first
    level_converged: List[bool] = dataclasses.field(default_factory=list)
    level_x: List[np.ndarray] = dataclasses.field(default_factory=list)   # final state of each level
    bt_steps: int = 0
    r0: float = 0.0
    r_final: float = 0.0
    converged: bool = False


def cascadic_solve(h, opts: Opts):
    """Nonlinear cascadic multigrid from the zero state; returns the fine
    state and per-level step counts (finest level first)."""
    L = len(h.levels)
    a = h.alpha
    rhs = [h.b0]
    for l in range(L - 1):
        rhs.append(h.transfers[l].R(rhs[l], h.levels[l].n_flux))
    st = CascadicStats(level_steps=[0] * L, level_converged=[False] * L, level_x=[None] * L)
    x = np.zeros(h.levels[L - 1].n)
    for l in range(L - 1, -1, -1):
        lev = h.levels[l]
        if l < L - 1:
            x = h.transfers[l].P(x, h.levels[l + 1].n_flux)
        tol = max(opts.rtol * norm(rhs[l]), opts.atol)
        r = norm(residual(lev, x, rhs[l], a))
        if l == 0:
            st.r0 = norm(rhs[0])
        for _ in range(opts.max_it):
            if r <= tol:
                break
            x, s = smooth_step(lev, x, rhs[l], a, opts, st)
            st.level_steps[l] += 1
            if s == 0.0:
                break
            r = norm(residual(lev, x, rhs[l], a))
        st.level_converged[l] = r <= tol
        st.level_x[l] = x.copy()
    st.r_final = r
    st.converged = st.level_converged[0]
    return x, st


def result_solve(h, x0=None, max_it=200):
    """The root x* of r^0 (eq. nonlinear_system_residual_form): damped Newton
    with exact solves, iterated until the residual stops decreasing below
    1e-13 of its initial value."""
    opts = Opts(newton=True, rtol=1e-14, atol=0.0, max_it=max_it)
    lev = h.levels[0]
    x = np.zeros(lev.n) if x0 is None else x0.copy()
    r0 = norm(residual(lev, x, h.b0, h.alpha))
    best = r0
    stall = 0
    for _ in range(max_it):
        x = smooth(lev, x, h.b0, h.alpha, opts)
        rn = norm(residual(lev, x, h.b0, h.alpha))
        if rn <= 1e-15 * r0:
            break
        if rn > 0.5 * best and best <= 1e-12 * r0:
            stall += 1
            if stall >= 2:
                break
        best = min(best, rn)
    return x
