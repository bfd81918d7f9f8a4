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
