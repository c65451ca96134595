"""Oracle pins for the control flow of the nonlinear solvers, on scripted
residual sequences (no linear algebra involved): the coarsest-level loop of
Section 4 (at most 10 smoothing steps, stopping early on convergence
relative to its entry residual or on atol, and after a step Alg. 1
rejected), the early return of Alg. 2 right after the fine pre-smoothing
(footnote of Table 1), the cascadic per-level loop, and the eigenvector sign
rule of the hierarchy (first entry above 1e-8 of the largest made
positive).

The scripted level is a counter: the state x is an integer, the residual of
state k is a prescribed number, and a smoothing step maps k to k + 1 with a
prescribed step length (0 = rejected by Alg. 1, state unchanged)."""
import numpy as np
import pytest

import oracle.solvers as S
from oracle.coarsen import sign_fix


class Script:
    """Residual norms r[k] of the states k = 0, 1, ...; step lengths s[k] of
    the step taken from state k."""

    def __init__(self, r, s=None):
        self.r = list(r)
        self.s = list(s) if s is not None else [1.0] * len(self.r)
        self.steps = 0

    def residual(self, level, x, b, alpha):
        return np.array([self.r[int(x)]])

    def smooth_step(self, level, x, b, alpha, opts, stats=None):
        self.steps += 1
        k = int(x)
        s = self.s[k]
        return (k if s == 0.0 else k + 1), s


@pytest.fixture
def script(monkeypatch):
    def make(r, s=None):
        sc = Script(r, s)
        monkeypatch.setattr(S, "residual", sc.residual)
        monkeypatch.setattr(S, "smooth_step", sc.smooth_step)
        return sc
    return make


def run_coarsest(sc, rtol=1e-8, atol=0.0, cmax=10, catol=None):
    o = S.Opts(rtol=rtol, atol=atol, coarsest_max=cmax, coarsest_atol=catol)
    x = S.coarsest_solve(None, 0, None, 1.0, o)
    return int(x), sc.steps


def test_coarsest_cap_of_ten_steps(script):
    # slow decrease that never meets 1e-8 of the entry residual: exactly 10 steps
    sc = script([10.0 ** (-0.1 * k) for k in range(20)])
    assert run_coarsest(sc) == (10, 10)
    sc = script([10.0 ** (-0.1 * k) for k in range(20)])
    assert run_coarsest(sc, cmax=3) == (3, 3)
    sc = script([1.0])
    assert run_coarsest(sc, cmax=0) == (0, 0)


def test_coarsest_tolerance_is_relative_to_the_entry_residual(script):
    # entry 100: the rule is r <= 1e-6; state 3 meets it exactly (<=), state 2 does not
    sc = script([100.0, 1.0, 1.01e-6, 1e-6, 1e-9, 1e-12])
    assert run_coarsest(sc) == (3, 3)
    # the same sequence scaled to entry 1: it needs r <= 1e-8
    sc = script([1.0, 1e-2, 1.01e-8, 1e-8, 1e-11])
    assert run_coarsest(sc) == (3, 3)
    # an entry already below atol takes no step
    sc = script([1e-11, 1.0])
    assert run_coarsest(sc, atol=1e-10) == (0, 0)
    # atol above rtol * entry decides
    sc = script([1.0, 1e-3, 5e-5, 1e-9])
    assert run_coarsest(sc, atol=1e-4) == (2, 2)
    # the coarsest level's own absolute floor replaces atol when given
    sc = script([1.0, 1e-3, 5e-5, 1e-9])
    assert run_coarsest(sc, atol=0.0, catol=1e-4) == (2, 2)
    sc = script([1.0, 1e-3, 5e-5, 1e-9])
    assert run_coarsest(sc, atol=1e-4, catol=0.0) == (3, 3)


def test_coarsest_stops_on_a_rejected_step(script):
    # the third step is rejected (s = 0): the state stays 2 and the loop ends
    sc = script([1.0, 0.5, 0.25, 0.1], s=[1.0, 0.5, 0.0, 1.0])
    assert run_coarsest(sc) == (2, 3)
    # rejected at once
    sc = script([1.0, 0.5], s=[0.0, 1.0])
    assert run_coarsest(sc) == (0, 1)


def test_coarsest_keeps_going_after_an_accepted_rise(script):
    # Alg. 1 may accept a step that raises the residual (after n_max halvings,
    # or when a halving gains less than theta); the loop must continue
    sc = script([1.0, 3.0, 2.0, 1e-9], s=[0.0625, 0.5, 1.0, 1.0])
    assert run_coarsest(sc) == (3, 3)
    # a rounding-level plateau above the tolerance runs to the cap
    sc = script([1.0, 1e-7] + [1.2e-7, 1e-7] * 10)
    assert run_coarsest(sc) == (10, 10)


class _NoTransfers:
    """Hierarchy stand-in whose transfers must not be touched."""

    def __init__(self):
        self.levels = [type("L", (), {"n_flux": 0})(), object()]
        self.alpha = 1.0

    @property
    def transfers(self):
        raise AssertionError("coarse correction entered")


def test_vcycle_returns_after_presmoothing_when_converged(monkeypatch):
    calls = []

    def smooth(lev, x, b, a, opts, stats=None):
        calls.append(x)
        return x + 1

    monkeypatch.setattr(S, "smooth", smooth)
    monkeypatch.setattr(S, "residual", lambda lev, x, b, a: np.array([[5.0, 1e-9, 2e-9][int(x)]]))
    h = _NoTransfers()
    st = S.Stats()
    x = S.nonlinear_mg(h, 0, 0, None, S.Opts(), st, stop_tol=1e-9)
    assert x == 1 and calls == [0] and st.stopped_after_presmooth
    # above the threshold the V-cycle goes on to the coarse correction
    st = S.Stats()
    with pytest.raises(AssertionError, match="coarse correction entered"):
        S.nonlinear_mg(h, 0, 0, None, S.Opts(), st, stop_tol=0.99e-9)
    assert not st.stopped_after_presmooth
    # without a threshold (coarse levels) it never returns early
    with pytest.raises(AssertionError, match="coarse correction entered"):
        S.nonlinear_mg(h, 0, 0, None, S.Opts(), S.Stats(), stop_tol=None)


def test_outer_loop_counts_a_presmoothing_stop_as_a_cycle(monkeypatch):
    seq = {0: 1.0, 1: 1e-3, 2: 1e-9}

    def mg(h, l, x, b, opts, stats=None, stop_tol=None):
        if int(x[0]) + 1 == 2 and stats is not None:
            stats.stopped_after_presmooth = True
        return x + 1

    monkeypatch.setattr(S, "nonlinear_mg", mg)
    monkeypatch.setattr(S, "residual", lambda lev, x, b, a: np.array([seq[int(x[0])]]))
    h = type("H", (), {})()
    h.levels = [type("L", (), {"n": 1})()]
    h.b0, h.alpha = None, 1.0
    x, st = S.fas_solve(h, S.Opts(rtol=1e-8, atol=0.0))
    assert int(x[0]) == 2 and st.iterations == 2 and st.converged and st.stopped_after_presmooth
    assert st.residuals == [1.0, 1e-3, 1e-9]


def test_sign_fix_hand_cases():
    # the first entry above 1e-8 max|v| is the third (the second, 1e-10, is below)
    v = np.array([0.0, -1e-10, -0.5, 0.3, 0.8])
    np.testing.assert_array_equal(sign_fix(v), -v)
    # already positive there: unchanged
    w = np.array([0.0, 1e-10, 0.5, -0.3, -0.8])
    np.testing.assert_array_equal(sign_fix(w), w)
    # an entry just above the threshold decides
    u = np.array([-2e-8, 0.5, -1.0])
    np.testing.assert_array_equal(sign_fix(u), -u)
    u = np.array([-0.5e-8, 0.5, -1.0])
    np.testing.assert_array_equal(sign_fix(u), u)
    # idempotent and sign-invariant
    rng = np.random.default_rng(3)
    for _ in range(20):
        z = rng.standard_normal(7)
        z[rng.integers(0, 7, 2)] = 0.0
        assert np.array_equal(sign_fix(sign_fix(z)), sign_fix(z))
        assert np.array_equal(sign_fix(-z), sign_fix(z))


def test_cascadic_levels_stop_on_tolerance_rejection_or_max_it(monkeypatch):
    # per level: residual of state k, and step lengths; the zero state of
    # level l has residual ||b^l||
    r = {2: [1.0, 3.0, 1e-9], 1: [2.0, 1e-3, 1e-3], 0: [4.0, 1e-2, 5e-9]}
    s = {2: [1.0, 1.0, 1.0], 1: [1.0, 0.0, 1.0], 0: [1.0, 1.0, 1.0]}

    class Lev:
        def __init__(self, l):
            self.l, self.n, self.n_flux = l, 1, 0

    levels = [Lev(0), Lev(1), Lev(2)]

    class Tr:
        def R(self, v, nf):
            return v

        def P(self, x, nf):
            return np.zeros(1)   # every finer level starts from its own state 0

    h = type("H", (), {})()
    h.levels, h.transfers, h.alpha = levels, [Tr(), Tr()], 1.0
    h.b0 = None   # ||b^l|| = 1 on every level (see norm below)

    def residual(lev, x, b, a):
        return np.array([r[lev.l][int(x[0])]])

    def smooth_step(lev, x, b, a, opts, stats=None):
        k = int(x[0])
        return np.array([float(k if s[lev.l][k] == 0.0 else k + 1)]), s[lev.l][k]

    monkeypatch.setattr(S, "residual", residual)
    monkeypatch.setattr(S, "smooth_step", smooth_step)
    monkeypatch.setattr(S, "norm", lambda v: float(abs(v[0])) if v is not None else 1.0)
    x, st = S.cascadic_solve(h, S.Opts(rtol=1e-8, atol=0.0, max_it=5))
    # level 2 (coarsest): the accepted rise 1 -> 3 does not stop it, then converged
    # level 1: the second step is rejected, the level hands its state up unconverged
    # level 0: converged after two steps
    assert st.level_steps == [2, 2, 2], st.level_steps
    assert st.level_converged == [True, False, True]
    assert st.converged and int(x[0]) == 2
    # max_it bounds every level: with one step allowed, level 2 stops unconverged at state 1
    x, st = S.cascadic_solve(h, S.Opts(rtol=1e-8, atol=0.0, max_it=1))
    assert st.level_steps == [1, 1, 1] and st.level_converged == [False, False, False]
