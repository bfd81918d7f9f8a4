"""Pins of the oracle's finite-element operators (CPU only).

Each test checks the oracle against something other than itself: a worked
closed form, an invariant of the P1 discretisation of eq. (1)-(2), or an
independent dense construction with library routines on tiny meshes.
"""

import os

import numpy as np
import pytest
import scipy.linalg as sla

import eqsgen
from oracle import fem
from oracle.eqs import EqsOracle

EPS0 = 8.8541878128e-12


def _perturbed(case, seed, amount=0.15):
    """Jitter interior node positions by up to amount*h so meshes are unstructured."""
    rng = np.random.default_rng(seed)
    h = 1.0 / case.n
    xyz = case.xyz.copy()
    interior = np.all((xyz > 1e-12) & (xyz < 1 - 1e-12), axis=1)
    xyz[interior] += rng.uniform(-amount * h, amount * h, size=(interior.sum(), 3))
    case.xyz = xyz
    return case


def _dense_reference(xyz, tets, w):
    """Independent dense assembly: barycentric coefficients from inv([1 p_a])."""
    n = xyz.shape[0]
    A = np.zeros((n, n))
    for e, v in enumerate(tets):
        B = np.hstack([np.ones((4, 1)), xyz[v]])
        coef = np.linalg.inv(B)  # column a: lambda_a = coef[0,a] + coef[1:,a].x
        grads = coef[1:, :].T
        vol = abs(np.linalg.det(B)) / 6.0
        A[np.ix_(v, v)] += w[e] * vol * grads @ grads.T
    return A


def test_reference_tet_matches_golden(golden_dir):
    rows = [l for l in open(os.path.join(golden_dir, "reference_tet.txt")) if not l.startswith("#")]
    expected = np.array([[float(v) for v in r.split()] for r in rows if r.strip()]) / 6.0
    p = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)
    A, vol = fem.element_matrix(p)
    assert vol == pytest.approx(1.0 / 6.0, rel=1e-15)
    np.testing.assert_allclose(A, expected, atol=1e-15)


def test_element_matrix_affine_invariance():
    """A_e scales as h for a scaled tet and is invariant under rotation + vertex relabelling."""
    rng = np.random.default_rng(0)
    p = rng.normal(size=(4, 3))
    A, vol = fem.element_matrix(p)
    Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    A2, vol2 = fem.element_matrix(2.5 * p @ Q.T + 7.0)
    np.testing.assert_allclose(A2, 2.5 * A, rtol=1e-12, atol=1e-12 * abs(A).max())
    assert vol2 == pytest.approx(vol * 2.5 ** 3, rel=1e-12)
    perm = [2, 0, 3, 1]
    A3, _ = fem.element_matrix(p[perm])
    np.testing.assert_allclose(A3, A[np.ix_(perm, perm)], rtol=1e-12, atol=1e-13 * abs(A).max())


def test_flat_tet_rejected():
    p = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], dtype=float)
    with pytest.raises(ValueError):
        fem.element_matrix(p)
    xyz, tets = eqsgen.kuhn_cube_mesh(2)
    tets = tets.copy()
    assert fem.first_flat_tet(xyz, tets) == -1
    tets[5] = [0, 1, 2, 0]
    assert fem.first_flat_tet(xyz, tets) == 5


@pytest.mark.parametrize("n", [2, 3, 4])
def test_assembly_matches_dense_brute_force(n):
    case = _perturbed(eqsgen.case_c0(n), seed=n)
    w = np.random.default_rng(n).uniform(0.5, 3.0, size=case.n_tets)
    A = fem.assemble(case.xyz, case.tets, w).toarray()
    ref = _dense_reference(case.xyz, case.tets, w)
    np.testing.assert_allclose(A, ref, rtol=0, atol=1e-13 * abs(ref).max())


def test_mesh_counts_and_valence():
    """Kuhn mesh: (n+1)^3 nodes, 6 n^3 tets, 14 neighbours per interior node."""
    n = 5
    case = eqsgen.case_c0(n)
    assert case.n_nodes == (n + 1) ** 3 and case.n_tets == 6 * n ** 3
    M = fem.assemble_M(case)
    nnz_row = np.diff(M.indptr)
    ijk = np.rint(case.xyz * n).astype(int)
    interior = np.all((ijk > 0) & (ijk < n), axis=1)
    assert np.all(nnz_row[interior] == 15)
    # every sub-cube's 6 tets fill it exactly
    vols = [fem.element_matrix(case.xyz[t])[1] for t in case.tets[:60]]
    np.testing.assert_allclose(vols, 1.0 / (6 * n ** 3), rtol=1e-13)


def test_constant_nullspace_and_shift_invariance():
    """Full M 1 = 0, K(x) 1 = 0 (row sums), K(x + c)(x + c) = K(x) x."""
    case = _perturbed(eqsgen.case_c1(n=6, seed=5), seed=1)
    M = fem.assemble_M(case)
    assert abs(M @ np.ones(case.n_nodes)).max() <= 1e-13 * abs(M.data).max()
    x = eqsgen.random_state(case.n_nodes, seed=3, scale=2.0)
    K = fem.assemble_K_frozen(case, x)
    assert abs(K @ np.ones(case.n_nodes)).max() <= 1e-13 * abs(K.data).max()
    y = fem.apply_K(case, x)
    y2 = fem.apply_K(case, x + 0.731)
    np.testing.assert_allclose(y2, y, rtol=0, atol=1e-12 * abs(y).max())
    # the element loop equals the frozen matrix times x
    np.testing.assert_allclose(K @ x, y, rtol=0, atol=1e-13 * abs(y).max())


def test_symmetry_definiteness_and_rayleigh_bounds():
    case = _perturbed(eqsgen.case_c1(n=5, seed=7), seed=2)
    o = EqsOracle(case)
    Mii = o.M_II.toarray()
    np.testing.assert_allclose(Mii, Mii.T, rtol=0, atol=1e-14 * abs(Mii).max())
    np.linalg.cholesky(Mii)  # SPD after Dirichlet elimination
    x = eqsgen.random_state(case.n_nodes, seed=11, scale=0.1)
    K = fem.assemble_K_frozen(case, x)
    Kii = K[o.free][:, o.free].toarray()
    np.testing.assert_allclose(Kii, Kii.T, rtol=0, atol=1e-14 * abs(Kii).max())
    assert np.linalg.eigvalsh(K.toarray()).min() >= -1e-12 * abs(K.data).max()
    lam = sla.eigh(Kii, Mii, eigvals_only=True)
    kap = fem.element_kappa(case, x)
    ratio = kap / (EPS0 * case.eps_r[case.tet_mat])
    assert lam.min() >= ratio.min() * (1 - 1e-9)
    assert lam.max() <= ratio.max() * (1 + 1e-9)


def test_patch_linear_field():
    """A linear potential has the exact constant field; with uniform kappa the
    rows of nodes off the boundary vanish, and the nonlinear law is applied to
    the exact |E|."""
    case = _perturbed(eqsgen.case_c0(4), seed=9)
    G = np.array([0.3, -0.7, 1.1])  # grad(phi)
    x = case.xyz @ G + 0.25
    # nonlinear material everywhere
    case.tet_mat[:] = 1
    y = fem.apply_K(case, x)
    emag = np.linalg.norm(G)
    kappa = case.kappa0[1] * (1 + (emag / case.e_s[1]) ** case.alpha[1])
    # expected y = kappa * (sum_e A_e) x = kappa * L x with L the unit Laplacian
    L = fem.assemble(case.xyz, case.tets, np.ones(case.n_tets))
    np.testing.assert_allclose(y, kappa * (L @ x), rtol=0, atol=1e-12 * kappa * abs(L @ x).max() + 1e-30)
    ijk_inside = np.all((case.xyz > 1e-12) & (case.xyz < 1 - 1e-12), axis=1)
    assert abs(y[ijk_inside]).max() <= 1e-12 * kappa * np.abs(L.data).max()
    # element conductivities equal the law at |G| for every tet
    np.testing.assert_allclose(fem.element_kappa(case, x), kappa, rtol=1e-12)


def test_pcg_sgs_matches_dense_solve():
    case = _perturbed(eqsgen.case_c1(n=6, seed=3), seed=4)
    o = EqsOracle(case, dense_limit=0)
    rng = np.random.default_rng(0)
    r = rng.normal(size=o.n_free)
    ref = np.linalg.solve(o.M_II.toarray(), r)
    res = fem.pcg_sgs(o.M_II, r, rtol=1e-13)
    assert res.status == 0 and res.relres <= 1e-13
    assert np.linalg.norm(res.x - ref) <= 1e-10 * np.linalg.norm(ref)
    # the dense (Cholesky) path agrees too
    o2 = EqsOracle(case)
    assert o2.dense
    np.testing.assert_allclose(o2.solve(r), ref, rtol=0, atol=1e-11 * abs(ref).max())
    # zero right-hand side gives zero with no iterations
    z = fem.pcg_sgs(o.M_II, np.zeros(o.n_free), x0=np.ones(o.n_free))
    assert z.iters == 0 and not z.x.any()
    # maxit reached is reported
    bad = fem.pcg_sgs(o.M_II, r, rtol=1e-15, maxit=1)
    assert bad.status == 1 and bad.iters == 1


@pytest.mark.parametrize("threads", [1, 4])
def test_pcg_jacobi_matches_dense_solve(threads):
    """The Jacobi-preconditioned CG (the reference solver for the large meshes,
    row loops on OpenMP threads) against numpy's dense solve, on one thread
    and on several."""
    case = _perturbed(eqsgen.case_c1(n=6, seed=3), seed=4)
    o = EqsOracle(case, dense_limit=0, solver="jacobi", threads=threads)
    rng = np.random.default_rng(1)
    r = rng.normal(size=o.n_free)
    ref = np.linalg.solve(o.M_II.toarray(), r)
    res = fem.pcg_jacobi(o.M_II, r, rtol=1e-13, threads=threads)
    assert res.status == 0 and res.relres <= 1e-13
    assert np.linalg.norm(res.x - ref) <= 1e-10 * np.linalg.norm(ref)
    np.testing.assert_allclose(o.solve(r), ref, rtol=0, atol=1e-10 * abs(ref).max())
    # a start vector is honoured: the exact solution needs no iteration
    ex = fem.pcg_jacobi(o.M_II, r, x0=res.x, rtol=1e-12, threads=threads)
    assert ex.iters == 0 and np.array_equal(ex.x, res.x)
    z = fem.pcg_jacobi(o.M_II, np.zeros(o.n_free), x0=np.ones(o.n_free), threads=threads)
    assert z.iters == 0 and not z.x.any()
    bad = fem.pcg_jacobi(o.M_II, r, rtol=1e-15, maxit=1, threads=threads)
    assert bad.status == 1 and bad.iters == 1


def test_warm_started_trajectory_equals_cold_sgs():
    """Warm starts (each stage solve from the previous solution) and the Jacobi
    solver change only iteration counts: the RKC trajectory equals the one with
    cold-started SGS solves to well below the parity bars."""
    case = eqsgen.case_c1(n=12, seed=1)
    a = EqsOracle(case, dense_limit=0)
    b = EqsOracle(case, dense_limit=0, solver="jacobi", warm=True, threads=2)
    ya = a.rkc_trajectory(np.zeros(a.n_free), 0.0, case.tau, case.s, 3)
    yb = b.rkc_trajectory(np.zeros(b.n_free), 0.0, case.tau, case.s, 3)
    scale = max(np.linalg.norm(y) for y in ya)
    assert max(np.linalg.norm(p - q) for p, q in zip(ya, yb)) <= 1e-12 * scale


def test_dirichlet_rhs_is_capacitive_coupling():
    """b(t) = -M_ID g'(t): with uniform eps the discrete harmonic extension of
    the top drive is exactly z on the free nodes (linear functions are in the
    P1 space), so M_II^{-1} b(t) = z_I g'(t)."""
    case = eqsgen.case_c0(6)
    case.tet_mat[:] = 0
    o = EqsOracle(case)
    t = 0.0013
    w = o.solve(o.b(t))
    gd = 2 * np.pi * 50.0 * np.cos(2 * np.pi * 50.0 * t)
    np.testing.assert_allclose(w, case.xyz[o.free, 2] * gd, rtol=0, atol=1e-12 * abs(gd))
