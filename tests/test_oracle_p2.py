"""Pins of the oracle's second-order (10-node) tetrahedra (Sec. III's P2 elements,
Sec. V's P2 model) - CPU only.

The oracle integrates with a 4-point rule; the pins integrate the same basis
exactly by another route: grad N_i . grad N_j is a quadratic polynomial in the
barycentric coordinates, and
    int_T lambda_0^k0 lambda_1^k1 lambda_2^k2 lambda_3^k3 = 6|T| k0! k1! k2! k3! / (k0+k1+k2+k3+3)!.
Further pins: the constant nullspace, quadratic patch tests (P2 holds every
quadratic exactly), brute-force dense assembly, and the time-integration
closed forms P1b and P2 on a second-order mesh.
"""

import itertools
from math import factorial

import numpy as np
import pytest

import eqsgen
from oracle import fem, rkc
from oracle.eqs import EqsOracle

EPS0 = 8.8541878128e-12
EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def bary_grads(p):
    """Gradients of the barycentric coordinates from the inverse of [1 p]."""
    T = np.hstack([np.ones((4, 1)), np.asarray(p, float)])
    Ti = np.linalg.inv(T)  # lambda = Ti^T [1, x]
    return Ti[1:, :].T, abs(np.linalg.det(T)) / 6.0


def basis_grad_polys(g):
    """grad N_i as dicts {exponent tuple: 3-vector coefficient} in lambda."""
    e = [tuple(int(k == a) for k in range(4)) for a in range(4)]
    zero = (0, 0, 0, 0)
    polys = []
    for a in range(4):  # (4 lambda_a - 1) grad lambda_a
        polys.append({e[a]: 4.0 * g[a], zero: -g[a]})
    for a, b in EDGES:  # 4 (lambda_b grad lambda_a + lambda_a grad lambda_b)
        polys.append({e[b]: 4.0 * g[a], e[a]: 4.0 * g[b]})
    return polys


def integrate(poly, vol):
    return sum(c * 6.0 * vol * np.prod([factorial(k) for k in ex]) / factorial(sum(ex) + 3)
               for ex, c in poly.items())


def exact_matrix(p):
    g, vol = bary_grads(p)
    P = basis_grad_polys(g)
    A = np.zeros((10, 10))
    for i in range(10):
        for j in range(10):
            prod = {}
            for (ea, ca), (eb, cb) in itertools.product(P[i].items(), P[j].items()):
                ex = tuple(x + y for x, y in zip(ea, eb))
                prod[ex] = prod.get(ex, 0.0) + float(ca @ cb)
            A[i, j] = integrate(prod, vol)
    return A, vol


def test_reference_tet_equals_exact_integration():
    p = [[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]]
    A, vol = fem.element_matrix_p2(p)
    E, v2 = exact_matrix(p)
    assert vol == pytest.approx(1 / 6) and v2 == pytest.approx(1 / 6)
    np.testing.assert_allclose(A, E, rtol=0, atol=1e-14)
    # integer entries times 30 (the reference tet's P2 stiffness in closed form)
    np.testing.assert_allclose(30 * A, np.round(30 * A), atol=1e-12)
    np.testing.assert_allclose(A.sum(axis=1), 0.0, atol=1e-14)  # constants are in the space


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_general_tets_equal_exact_integration(seed):
    rng = np.random.default_rng(seed)
    p = rng.normal(size=(4, 3))
    A, vol = fem.element_matrix_p2(p)
    E, _ = exact_matrix(p)
    np.testing.assert_allclose(A, E, rtol=0, atol=1e-12 * np.abs(E).max())
    # orientation and vertex order do not matter (permute vertices with their edges)
    perm = (2, 0, 3, 1)
    q = p[list(perm)]
    B, _ = fem.element_matrix_p2(q)
    # local index of every node of the permuted tet in the original numbering
    idx = list(perm) + [4 + EDGES.index(tuple(sorted((perm[a], perm[b])))) for a, b in EDGES]
    np.testing.assert_allclose(B, A[np.ix_(idx, idx)], rtol=0, atol=1e-12 * np.abs(A).max())


def _jittered_p2(n, seed, amount=0.12):
    case = eqsgen.case_c0_p2(n)
    rng = np.random.default_rng(seed)
    h = 1.0 / (2 * n)
    xyz = case.xyz.copy()
    inner = np.all((xyz > 1e-12) & (xyz < 1 - 1e-12), axis=1)
    # move the vertices of the underlying P1 mesh, then put every midpoint back
    # at the middle of its edge (straight-sided second-order tets)
    xyz[inner] += amount * h * rng.uniform(-1, 1, size=(inner.sum(), 3))
    for k, (a, b) in enumerate(EDGES):
        xyz[case.tets[:, 4 + k]] = 0.5 * (xyz[case.tets[:, a]] + xyz[case.tets[:, b]])
    case.xyz = xyz
    return case


@pytest.mark.parametrize("n", [2, 3])
def test_assembly_matches_dense_brute_force(n):
    case = _jittered_p2(n, seed=n)
    w = np.random.default_rng(7).uniform(1.0, 3.0, size=case.n_tets)
    A = fem.assemble(case.xyz, case.tets, w).toarray()
    D = np.zeros_like(A)
    for e, t in enumerate(case.tets):
        E, _ = exact_matrix(case.xyz[t[:4]])
        D[np.ix_(t, t)] += w[e] * E
    np.testing.assert_allclose(A, D, rtol=0, atol=1e-12 * np.abs(D).max())
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    np.testing.assert_allclose(A @ np.ones(case.n_nodes), 0.0, atol=1e-13 * np.abs(A).max())


def test_quadratic_patch_tests():
    """Second-order elements hold every quadratic exactly, so on interior rows
    the stiffness product of an interpolated quadratic phi equals
    -Laplace(phi) int N_i: zero for a harmonic quadratic, and for phi = x^2
    -2 int N_i with int N_a = -|T|/20 (vertex) and int N_ab = |T|/5 (edge)."""
    case = _jittered_p2(3, seed=5)
    x, y, z = case.xyz.T
    A = fem.assemble(case.xyz, case.tets, np.ones(case.n_tets))
    inner = np.all((case.xyz > 1e-12) & (case.xyz < 1 - 1e-12), axis=1)
    harm = x * x - y * y + 3 * x * y - 2 * y * z + z
    assert np.abs((A @ harm)[inner]).max() <= 1e-12
    mass = np.zeros(case.n_nodes)
    for t in case.tets:
        _, vol = bary_grads(case.xyz[t[:4]])
        mass[t[:4]] += -vol / 20.0
        mass[t[4:]] += vol / 5.0
    np.testing.assert_allclose((A @ (x * x))[inner], (-2.0 * mass)[inner], rtol=0, atol=1e-12)


def test_K_of_x_p2_invariants():
    case = eqsgen.case_p2(n=3, seed=2)
    rng = np.random.default_rng(3)
    xv = rng.uniform(-2, 2, size=case.n_nodes)
    y = fem.apply_K(case, xv)
    # constants: K(x)1 row sums and shift invariance
    np.testing.assert_allclose(fem.apply_K(case, xv + 0.7), y, rtol=0, atol=1e-12 * np.abs(y).max())
    Kf = fem.assemble_K_frozen(case, xv)
    np.testing.assert_allclose(Kf @ xv, y, rtol=0, atol=1e-12 * np.abs(y).max())
    np.testing.assert_allclose(Kf @ np.ones(case.n_nodes), 0.0, atol=1e-13 * abs(Kf).max())
    assert abs(Kf - Kf.T).max() <= 1e-14 * abs(Kf).max()
    # linear kappa law: K(x) = kappa/eps M
    case.nonlinear[:] = 0
    M = fem.assemble_M(case)
    case.kappa0 = 3.0e3 * EPS0 * case.eps_r  # uniform ratio 3e3
    np.testing.assert_allclose(fem.apply_K(case, xv), 3.0e3 * (M @ xv), rtol=0,
                               atol=1e-12 * np.abs(M @ xv).max() * 3e3)


def test_P1b_uniform_ratio_on_second_order_mesh():
    case = eqsgen.case_p2(n=2, seed=2)
    c = 2.5e3
    case.kappa0 = c * case.eps_r * EPS0
    case.nonlinear[:] = 0
    case.amp[:] = 0.0
    o = EqsOracle(case)
    x0 = eqsgen.random_state(case.n_nodes, seed=4)[o.free]
    s, tau = 8, 5.0 / c
    co = rkc.coefficients(s)
    traj = o.rkc_trajectory(x0, 0.0, tau, s, 3)
    from test_oracle_eqs import P_closed

    for n, Y in enumerate(traj):
        np.testing.assert_allclose(Y, P_closed(co, s, -c * tau) ** n * x0, rtol=0, atol=1e-11 * abs(x0).max())


def test_P2_single_material_drive_is_linear_in_z():
    """One material, sinusoidal drive from rest: z is in the second-order
    space and discretely harmonic, so every state is z_I u with u the scalar
    RKC solution of u' = -c (u - g) + g'."""
    case = eqsgen.case_c0_p2(2)
    case.tet_mat[:] = 0
    c = 700.0
    case.kappa0[:] = c * EPS0 * case.eps_r
    case.nonlinear[:] = 0
    o = EqsOracle(case)
    s, tau, steps = 8, 1e-4, 6
    traj = o.rkc_trajectory(np.zeros(o.n_free), 0.0, tau, s, steps)
    w = 2 * np.pi * case.freq[1]
    u = np.array([0.0])
    rkc_scalar = [u]
    co = rkc.coefficients(s)
    for n in range(steps):
        u = rkc.step(lambda t, v: -c * (v - np.sin(w * t)) + w * np.cos(w * t), n * tau, u, tau, co)
        rkc_scalar.append(u)
    zI = case.xyz[o.free, 2]
    for Y, uu in zip(traj, rkc_scalar):
        np.testing.assert_allclose(Y, zI * uu[0], rtol=0, atol=1e-12)
