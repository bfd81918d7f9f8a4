"""Pins of the oracle's RKC integrator (Sec. II, ref. [9]) — CPU only.

The stage recurrence is checked against the closed form of the Chebyshev
polynomials (T_j(x) = cos(j arccos x) or cosh(j arccosh x)), which the
oracle never evaluates, and against exactness/order properties of a
second-order Runge-Kutta method.
"""

import numpy as np
import pytest

from oracle import rkc


def cheb_closed(j, x):
    x = np.asarray(x, dtype=float)
    out = np.empty_like(x)
    inside = np.abs(x) <= 1
    out[inside] = np.cos(j * np.arccos(x[inside]))
    hi = x > 1
    out[hi] = np.cosh(j * np.arccosh(x[hi]))
    lo = x < -1
    out[lo] = (-1) ** j * np.cosh(j * np.arccosh(-x[lo]))
    return out


@pytest.mark.parametrize("s", [2, 3, 5, 8, 12, 16])
def test_stage_values_follow_chebyshev_closed_form(s):
    """y' = lam y: stage j equals P_j(z) y0, P_j(z) = a_j + b_j T_j(w0 + w1 z)."""
    co = rkc.coefficients(s)
    for z in [-co.beta, -0.9 * co.beta, -0.37 * co.beta, -1.0, -0.05, 0.0, 0.3]:
        lam, tau = z / 0.01, 0.01
        st = []
        rkc.step(lambda t, y: lam * y, 0.0, np.array([1.0]), tau, co, st)
        for j in range(1, s + 1):
            Yj = st[j][1][0]
            expect = co.a[j] + co.b[j] * cheb_closed(j, np.array([co.w0 + co.w1 * z]))[0]
            assert Yj == pytest.approx(expect, rel=1e-11, abs=1e-12), (s, z, j)


@pytest.mark.parametrize("s", [2, 4, 8, 12, 16])
def test_second_order_and_stability_interval(s):
    co = rkc.coefficients(s)
    assert co.c[s] == pytest.approx(1.0, rel=1e-14)

    def Ps(z):
        return rkc.step(lambda t, y: (z / 0.1) * y, 0.0, np.array([1.0]), 0.1, co)[0]

    # P_s(z) = 1 + z + z^2/2 + O(z^3): the z^3 remainder must scale like z^3
    r1 = Ps(1e-2) - (1 + 1e-2 + 0.5e-4)
    r2 = Ps(5e-3) - (1 + 5e-3 + 0.5 * 25e-6)
    assert abs(r1) < 1e-5 and abs(r2) < 1e-6
    if s == 2:  # P_2 is quadratic: exactly the Taylor polynomial
        assert abs(r1) < 1e-15 and abs(r2) < 1e-15
    else:
        assert r1 / r2 == pytest.approx(8.0, rel=0.05)
    # damped: |P_s| <= 1 on [-beta, 0]; grows beyond the boundary
    zs = np.linspace(-co.beta, 0.0, 301)
    assert max(abs(Ps(z)) for z in zs) <= 1.0 + 1e-12
    assert abs(Ps(-1.1 * co.beta)) > 1.0
    if s >= 8:
        assert 0.64 <= co.beta / s ** 2 <= 0.67


@pytest.mark.parametrize("s", [2, 5, 16])
def test_stage_times(s):
    """F = 1: Y_j = c_j tau exactly; F = t: Y_s = t0 tau + tau^2/2 (2nd order)."""
    co = rkc.coefficients(s)
    tau, t0 = 0.3, 1.7
    st = []
    rkc.step(lambda t, y: np.ones_like(y), t0, np.zeros(1), tau, co, st)
    for j in range(s):
        assert st[j][0] == pytest.approx(t0 + co.c[j] * tau, rel=1e-15)
        assert st[j][1][0] == pytest.approx(co.c[j] * tau, rel=1e-12, abs=1e-15)
    y = rkc.step(lambda t, y: np.full_like(y, t), t0, np.zeros(1), tau, co)
    assert y[0] == pytest.approx(t0 * tau + tau ** 2 / 2, rel=1e-12)


@pytest.mark.parametrize("s", [3, 8])
def test_order_two_on_nonautonomous_problem(s):
    """y' = cos(t) y, y(0) = 1 has y = exp(sin t): global error ~ tau^2."""
    co = rkc.coefficients(s)
    errs = []
    for steps in (20, 40, 80):
        tau = 2.0 / steps
        y = np.array([1.0])
        for n in range(steps):
            y = rkc.step(lambda t, yy: np.cos(t) * yy, n * tau, y, tau, co)
        errs.append(abs(y[0] - np.exp(np.sin(2.0))))
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.1)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.1)


def test_needs_two_stages():
    with pytest.raises(ValueError):
        rkc.coefficients(1)


# ------------------------------------------------------------- adaptive RKC
def test_error_estimate_vanishes_where_rkc_is_exact():
    """y' = a + b t has a quadratic solution, which a second-order method
    reproduces exactly; ref. [9]'s estimate is then zero (to rounding)."""
    a, b = 0.7, -3.1
    F = lambda t, y: np.full_like(y, a + b * t)  # noqa: E731
    for s in (2, 5, 12):
        co = rkc.coefficients(s)
        t0, tau = 0.3, 0.05
        y0 = np.array([1.2])
        y1 = rkc.step(F, t0, y0, tau, co)
        exact = y0 + a * tau + 0.5 * b * ((t0 + tau) ** 2 - t0 ** 2)
        assert y1[0] == pytest.approx(exact[0], rel=1e-14)
        est = rkc.error_estimate(y0, y1, F(t0, y0), F(t0 + tau, y1), tau)
        assert abs(est[0]) < 1e-14


@pytest.mark.parametrize("s", [2, 4, 9])
def test_error_estimate_is_third_order(s):
    """For y' = lam y the estimate is O(tau^3) like the local error it stands
    for: halving tau divides it by 8; for s = 2 (P_2(z) = 1 + z + z^2/2
    exactly) est = z^3 y / 5 in closed form."""
    lam = -2.0
    co = rkc.coefficients(s)
    F = lambda t, y: lam * y  # noqa: E731

    def est(tau):
        y0 = np.array([1.0])
        y1 = rkc.step(F, 0.0, y0, tau, co)
        return rkc.error_estimate(y0, y1, F(0, y0), F(tau, y1), tau)[0]

    assert est(1e-2) / est(5e-3) == pytest.approx(8.0, rel=0.02)
    if s == 2:
        z = lam * 1e-2
        assert est(1e-2) == pytest.approx(z ** 3 / 5.0, rel=1e-6)


def test_stage_choice_covers_the_step():
    """The stage count is the smallest s >= 2 whose stability interval covers
    tau rho; beyond s_max the step is shortened to fit beta(s_max)."""
    for tau_rho in [0.0, 1.0, 7.9, 8.0, 40.0, 166.0, 1000.0]:
        s, tau = rkc.stages_for(1.0, tau_rho, 250)
        assert tau == 1.0
        assert s == 2 or rkc.beta(s - 1) < tau_rho
        assert rkc.beta(s) >= tau_rho
        # beta(s) grows like 0.65 s^2 (ref. [9]); the choice sits near sqrt(tau rho / 0.65)
        assert s <= max(2, int(np.ceil(np.sqrt(tau_rho / 0.64))) + 1)
    s, tau = rkc.stages_for(1.0, 1e6, 16)
    assert s == 16 and tau == pytest.approx(rkc.beta(16) / 1e6, rel=1e-15)


@pytest.mark.parametrize("tol", [1e-3, 1e-5, 1e-7])
def test_adaptive_scalar_decay_controls_the_error(tol):
    """y' = -lam y from a deliberately large first step: the first attempt is
    rejected, every accepted step has err <= 1, the run ends exactly at t_end
    and every step is stable. With the local error held at tol per step, a
    second-order method takes steps ~ tol^(1/3) and reaches a global error
    ~ tol^(2/3): one decade of tolerance multiplies the steps by 10^(1/3) and
    divides the error by 10^(2/3)."""
    lam = 40.0

    def run(tl):
        out, rec = rkc.adaptive(lambda t, y: -lam * y, lambda t, y: lam, 0.0, np.array([1.0]), 0.5, 0.05, tl, tl)
        return out, rec, max(abs(y[0] - np.exp(-lam * t)) for t, y in out)

    out, rec, gerr = run(tol)
    assert not rec[0].accepted and rec[0].err > 1.0
    assert all(r.err <= 1.0 for r in rec if r.accepted)
    assert all(r.err > 1.0 for r in rec if not r.accepted)
    assert out[-1][0] == 0.5
    assert all(rkc.beta(r.s) >= r.tau * lam for r in rec)
    out2, _, gerr2 = run(tol / 10)
    assert 10 ** (2 / 3) / 1.3 <= gerr / gerr2 <= 10 ** (2 / 3) * 1.3
    assert 10 ** (1 / 3) / 1.3 <= len(out2) / len(out) <= 10 ** (1 / 3) * 1.3


def test_adaptive_stiff_linear_system_exact_solution():
    """y' = A y with A = -diag(1, 1e4): the stiff component forces many stages,
    the smooth one sets the step; the solution matches exp(A t) y0."""
    d = np.array([1.0, 1e4])
    y0 = np.array([1.0, 1.0])
    out, rec = rkc.adaptive(lambda t, y: -d * y, lambda t, y: d.max(), 0.0, y0, 2.0, 1e-4, 1e-6, 1e-4)
    assert max(r.s for r in rec if r.accepted) >= 10
    for t, y in out[1:]:
        assert abs(y[0] - np.exp(-t)) <= 1e-3
        assert abs(y[1] - np.exp(-1e4 * t)) <= 1e-3
