"""Pins of the oracle's semi-discrete EQS system and RKC trajectories — CPU only.

Closed forms used:
  P1  two-layer Maxwell-Wagner relaxation under a step drive: the P1 solution
      stays piecewise linear in z and the interface potential obeys one scalar
      linear ODE, so RKC gives phi_inf + (phi_0 - phi_inf) P_s(-tau/T)^n.
  P1b kappa/eps uniform: K = cM, F = -cY, every stage is P_j(-c tau) x0.
  P2  one material + sinusoidal drive from rest: Y = z_I u with u the scalar
      RKC solution of u' = -c(u - g) + g'.
  P3  the c0 slab problem on states that depend on z only is a 1D P1 FEM in
      z with n-1 unknowns and layer-wise kappa(|G|); the 3D stages equal it.
  P9  eq. (3) on P1b: (1 - c tau)^n x0.
"""

import numpy as np
import pytest

import eqsgen
from oracle import rkc
from oracle.eqs import EqsOracle

EPS0 = 8.8541878128e-12


def cheb_closed(j, x):
    if abs(x) <= 1:
        return np.cos(j * np.arccos(x))
    if x > 1:
        return np.cosh(j * np.arccosh(x))
    return (-1) ** j * np.cosh(j * np.arccosh(-x))


def P_closed(co, j, z):
    return co.a[j] + co.b[j] * cheb_closed(j, co.w0 + co.w1 * z)


def lin(eps_r, kappa):
    return dict(eps_r=eps_r, kappa0=kappa, e_s=1.0, alpha=0.0, nonlinear=0)


def _maxwell_wagner(n, s, steps, tau_over_T, V0=1.0):
    e1, e2 = 4.0, 12.0
    k1, k2 = 3e-9, 1e-9
    case = eqsgen.layered_case(n, [(0.0, 0.5, lin(e1, k1)), (0.5, 1.0, lin(e2, k2))],
                               amp=V0, freq=0.0, phase=np.pi / 2)
    d1 = d2 = 0.5
    E1, E2 = EPS0 * e1, EPS0 * e2
    T = (E1 * d2 + E2 * d1) / (k1 * d2 + k2 * d1)
    phi0 = V0 * E2 * d1 / (E1 * d2 + E2 * d1)
    phiinf = V0 * k2 * d1 / (k1 * d2 + k2 * d1)
    o = EqsOracle(case)
    z = case.xyz[:, 2]

    def profile(phi_i):
        return np.where(z <= 0.5, phi_i * z / d1, phi_i + (V0 - phi_i) * (z - 0.5) / d2)

    tau = tau_over_T * T
    traj = o.rkc_trajectory(profile(phi0)[o.free], 0.0, tau, s, steps)
    return case, o, T, tau, phi0, phiinf, profile, traj


@pytest.mark.parametrize("s,tau_over_T", [(8, 2.5), (4, 0.7), (16, 30.0)])
def test_P1_maxwell_wagner_discrete_closed_form(s, tau_over_T):
    case, o, T, tau, phi0, phiinf, profile, traj = _maxwell_wagner(8, s, 12, tau_over_T)
    co = rkc.coefficients(s)
    R = P_closed(co, s, -tau / T)
    for nstep, Y in enumerate(traj):
        phi_i = phiinf + (phi0 - phiinf) * R ** nstep
        np.testing.assert_allclose(Y, profile(phi_i)[o.free], rtol=0, atol=1e-12)


def test_P1_maxwell_wagner_order_two_in_time():
    errs = []
    for k in (1, 2, 4):
        case, o, T, tau, phi0, phiinf, profile, traj = _maxwell_wagner(4, 8, 10 * k, 0.1 / k)
        t_end = len(traj[1:]) * tau
        exact = profile(phiinf + (phi0 - phiinf) * np.exp(-t_end / T))[o.free]
        errs.append(np.abs(traj[-1] - exact).max())
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.15)
    assert errs[1] / errs[2] == pytest.approx(4.0, rel=0.15)


def test_P1b_uniform_ratio_every_stage():
    case = eqsgen.case_c1(n=5, seed=2)
    c = 4.0e3
    eps = case.eps_r * EPS0
    case.kappa0 = c * eps
    case.nonlinear[:] = 0
    case.amp[:] = 0.0
    o = EqsOracle(case)
    x0 = eqsgen.random_state(case.n_nodes, seed=8)[o.free]
    s, tau = 12, 7.0 / c
    co = rkc.coefficients(s)
    stages = []
    o.rkc_trajectory(x0, 0.0, tau, s, 2, stages=stages)
    for n, rec in enumerate(stages):
        base = P_closed(co, s, -c * tau) ** n
        for j, (tj, Yj, Fj) in enumerate(rec):
            expect = (1.0 if j == 0 else P_closed(co, j, -c * tau)) * base
            np.testing.assert_allclose(Yj, expect * x0, rtol=0, atol=1e-11 * abs(x0).max())


def test_P9_explicit_euler_eq3():
    case = eqsgen.case_c1(n=4, seed=2)
    c = 2.0e3
    case.kappa0 = c * case.eps_r * EPS0
    case.nonlinear[:] = 0
    case.amp[:] = 0.0
    o = EqsOracle(case)
    x = eqsgen.random_state(case.n_nodes, seed=1)[o.free]
    x0 = x.copy()
    tau = 0.3 / c
    for n in range(5):
        x = o.euler_step(n * tau, x, tau)
    np.testing.assert_allclose(x, (1 - c * tau) ** 5 * x0, rtol=0, atol=1e-12)


def test_P2_single_material_sinusoidal_drive():
    n, s, steps = 4, 8, 10
    c = 700.0
    case = eqsgen.layered_case(n, [(0.0, 1.0, lin(6.0, c * 6.0 * EPS0))], amp=1.3, freq=50.0)
    o = EqsOracle(case)
    zI = case.xyz[o.free, 2]
    tau = 4e-4
    stages = []
    traj = o.rkc_trajectory(np.zeros(o.n_free), 0.0, tau, s, steps, stages=stages)

    A, f = 1.3, 50.0
    g = lambda t: A * np.sin(2 * np.pi * f * t)
    gd = lambda t: 2 * np.pi * f * A * np.cos(2 * np.pi * f * t)
    co = rkc.coefficients(s)
    u = np.zeros(1)
    us = [u.copy()]
    for k in range(steps):
        u = rkc.step(lambda t, uu: -c * (uu - g(t)) + gd(t), k * tau, u, tau, co)
        us.append(u.copy())
    for k, Y in enumerate(traj):
        np.testing.assert_allclose(Y, zI * us[k][0], rtol=0, atol=1e-12)
    for rec in stages:  # every stage stays proportional to z_I
        for (_, Yj, _) in rec:
            u_j = Yj[np.argmax(zI)] / zI.max()
            np.testing.assert_allclose(Yj, zI * u_j, rtol=0, atol=1e-12)


def _z_only_fem(case, amp, n):
    """1D P1 FEM in z for states whose node values depend on z only.

    On the Kuhn mesh with layer-wise materials such states form an invariant
    subspace of F (each layer carries a uniform field, and a uniform total
    current J = kappa G + eps G' makes the weak form vanish for every test
    function that is zero at z = 0 and z = 1), so the 3D RKC stages must
    equal RKC on this (n-1)-unknown system. Written independently of the 3D
    element loop: layer k carries eps_k, kappa_k(|G_k|) with G_k the layer's
    potential gradient."""
    h = 1.0 / n
    zc = (np.arange(n) + 0.5) * h
    layer_mat = ((zc > 0.4) & (zc < 0.6)).astype(int)  # the c0 slab by centroid
    eps = EPS0 * case.eps_r[layer_mat]
    f = case.freq[1]
    Mz = np.zeros((n + 1, n + 1))
    for k in range(n):
        Mz[k:k + 2, k:k + 2] += eps[k] / h * np.array([[1, -1], [-1, 1]])
    Mii = Mz[1:n, 1:n]

    def full(y, t):
        return np.concatenate([[0.0], y, [amp * np.sin(2 * np.pi * f * t)]])

    def F(t, y):
        phi = full(y, t)
        gd = 2 * np.pi * f * amp * np.cos(2 * np.pi * f * t)
        G = np.diff(phi) / h
        m = layer_mat
        kap = np.where(case.nonlinear[m] == 1,
                       case.kappa0[m] * (1 + (np.abs(G) / case.e_s[m]) ** case.alpha[m]), case.kappa0[m])
        J = kap * G  # conductive current density per layer (times -1)
        r = J[1:] - J[:-1]  # -[K phi]_i = J_i - J_{i-1}
        r = r - Mz[1:n, n] * gd  # b = -M_ID g'
        return np.linalg.solve(Mii, r)

    return F, full


@pytest.mark.parametrize("amp,steps", [(1.0, 30), (3.2, 30)])
def test_P3_c0_equals_z_only_1d_fem(amp, steps):
    n = 8
    case = eqsgen.case_c0(n)
    case.amp[1] = amp
    o = EqsOracle(case)
    F1, full = _z_only_fem(case, amp, n)
    co = rkc.coefficients(case.s)
    stages3 = []
    traj3 = o.rkc_trajectory(np.zeros(o.n_free), 0.0, case.tau, case.s, steps, stages=stages3)
    level = np.rint(case.xyz[o.free, 2] * n).astype(int)  # z-level of each free node
    y = np.zeros(n - 1)
    scale = max(np.abs(Y).max() for Y in traj3)
    for k in range(steps):
        rec = []
        y = rkc.step(F1, k * case.tau, y, case.tau, co, rec)
        for (tj, Yj, Fj), (tj2, yj, fj) in zip(stages3[k], rec):
            assert tj == tj2
            np.testing.assert_allclose(Yj, yj[level - 1], rtol=0, atol=1e-12 * scale)
            if Fj is not None:
                np.testing.assert_allclose(Fj, fj[level - 1], rtol=0, atol=1e-11 * np.abs(fj).max())
        np.testing.assert_allclose(traj3[k + 1], y[level - 1], rtol=0, atol=1e-12 * scale)
    if amp > 3:  # the strong drive really switches the varistor slab on
        assert o.max_rate * case.tau > 0.1  # sigma/eps rose ~3000-fold


def test_stability_bound_is_enforced():
    case = eqsgen.case_c1(n=3, seed=2)
    c = 1e6
    case.kappa0 = c * case.eps_r * EPS0
    case.nonlinear[:] = 0
    o = EqsOracle(case)
    with pytest.raises(RuntimeError, match="stability"):
        o.rkc_trajectory(np.zeros(o.n_free), 0.0, 1e-4, 4, 1)


def test_P1b_adaptive_steps_equal_scalar_run():
    """Adaptive RKC (ref. [9]'s estimate and controller) on P1b: with
    kappa/eps = c everywhere and g = 0, every stage is a polynomial in -c tau
    times x0, and with atol = 0 every component's weighted error equals the
    scalar problem's, so the FE run attempts, accepts and rejects exactly the
    steps (tau, s) of adaptive RKC on y' = -c y, and x_n = y_n x0."""
    case = eqsgen.case_c1(n=5, seed=2)
    c = 4.0e3
    case.kappa0 = c * case.eps_r * EPS0
    case.nonlinear[:] = 0
    case.amp[:] = 0.0
    o = EqsOracle(case)
    x0 = eqsgen.random_state(case.n_nodes, seed=9)[o.free]
    t_end, tau0, rtol = 3e-3, 2e-3, 1e-4
    out, rec = o.rkc_adaptive(x0, 0.0, t_end, tau0, 0.0, rtol)
    sout, srec = rkc.adaptive(lambda t, y: -c * y, lambda t, y: c, 0.0, np.array([1.0]), t_end, tau0, 0.0, rtol)
    assert [(r.accepted, r.s) for r in rec] == [(r.accepted, r.s) for r in srec]
    # err comes from differences of nearby states, so tau agrees to ~1e-10 (rounding)
    np.testing.assert_allclose([r.tau for r in rec], [r.tau for r in srec], rtol=1e-9)
    assert any(not r.accepted for r in rec) and max(r.s for r in rec) > 2
    for (t, x), (ts, y) in zip(out, sout):
        assert t == pytest.approx(ts, rel=1e-12)
        np.testing.assert_allclose(x, y[0] * x0, rtol=0, atol=1e-11 * abs(x0).max())
    # and the scalar run tracks the exact decay
    assert abs(sout[-1][1][0] - np.exp(-c * t_end)) <= 50 * rtol
