"""Second-order (10-node) tetrahedra on the GPU (eqs_set_mesh_p2) against the
FP64 oracle: the fused element pass K(x)x and the stage right-hand side entry
by entry (1e-12 relative), the M product (1e-13), the AMG-preconditioned
solve, RKC trajectories (1e-9 with CG at rel-res 1e-12; the slab mesh has
4,335 free DOF, so the oracle's solves are dense Cholesky), and the element
pass and M product on every node of the 2.1M-DOF second-order workload.
"""

import numpy as np
import pytest

import eqsgen
from oracle import fem
from oracle.eqs import EqsOracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1612_09447_amd import EQS_PREC_FP32, EQS_PREC_FP64, Context  # noqa: E402

DEV = torch.device("cuda:0")


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def relinf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def ctx_for(case, precision=EQS_PREC_FP64):
    c = Context(0, torch.cuda.current_stream(DEV))
    c.setup_case(case, precision=precision)
    return c


def smooth_state(case, seed):
    rng = np.random.default_rng(seed)
    x, y, z = case.xyz.T
    k = rng.uniform(1, 3, size=3)
    return 1.6 * z + 0.1 * np.sin(np.pi * k[0] * x) * np.sin(np.pi * k[1] * y) * np.sin(np.pi * k[2] * z)


@pytest.mark.parametrize("maker", [lambda: eqsgen.case_c0_p2(8), lambda: eqsgen.case_p2(n=10, seed=3)])
@pytest.mark.parametrize("generic", [False, True])
def test_p2_element_pass_and_rhs_match_oracle(maker, generic, monkeypatch):
    case = maker()
    if generic:
        monkeypatch.setenv("EQS_KX_GENERIC", "1")
    o = EqsOracle(case, dense_limit=0)
    with ctx_for(case) as c:
        print(f"[p2] {case.name}: {c.describe().splitlines()[1]}", flush=True)
        for seed, (x, t) in enumerate([(eqsgen.random_state(case.n_nodes, 3, 1.5), 0.0017),
                                       (smooth_state(case, 4), 0.0043)]):
            y = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
            c.apply_K(t, T(x), y)
            ref = fem.apply_K(case, o.embed(x[o.free], t))
            e1 = relinf(y.cpu().numpy(), ref)
            r = torch.zeros(o.n_free, dtype=torch.float64, device=DEV)
            c.stage_rhs(t, T(x[o.free]), r)
            e2 = relinf(r.cpu().numpy(), o.stage_rhs(t, x[o.free]))
            print(f"[p2] generic={generic} state {seed}: K(x)x {e1:.2e}, stage rhs {e2:.2e}", flush=True)
            assert e1 <= 1e-12 and e2 <= 1e-12


def test_p2_M_product_and_solve():
    """The M product and an AMG-PCG solve; second-order M (vertex and edge rows of
    different lengths alternating) is stored with its rows sorted by length
    within 256-row windows, a path this test therefore covers."""
    case = eqsgen.case_p2(n=10, seed=3)
    o = EqsOracle(case, dense_limit=0)
    with ctx_for(case, EQS_PREC_FP32) as c:
        d = c.describe()
        assert "M: sell64s" in d and "A0: sell64s" in d, d
        info = c.info()
        assert info["n_free"] == o.n_free
        x = np.random.default_rng(5).normal(size=o.n_free)
        y = torch.zeros(o.n_free, dtype=torch.float64, device=DEV)
        c.apply_M(T(x), y)
        ref = fem.csr_matvec(o.M_II, x)
        assert relinf(y.cpu().numpy(), ref) <= 1e-13
        rhs = o.stage_rhs(0.0021, smooth_state(case, 6)[o.free])
        z = torch.zeros_like(y)
        st = c.solve_M(T(rhs), z, rtol=1e-10, maxit=500)
        true = np.linalg.norm(rhs - fem.csr_matvec(o.M_II, z.cpu().numpy())) / np.linalg.norm(rhs)
        print(f"[p2] n=10 second-order M: {o.M_II.nnz} nonzeros, {info['n_levels']} AMG levels, CG {st['iters']} "
              f"iterations, oracle residual {true:.2e}", flush=True)
        assert st["relres"] <= 1e-10 and true <= 1.01e-10


@pytest.mark.parametrize("precision", [EQS_PREC_FP64, EQS_PREC_FP32])
def test_p2_slab_trajectory_matches_oracle(precision):
    case = eqsgen.case_c0_p2(8)
    case.amp[1] = 3.0  # into the varistor's nonlinear range
    steps = 25
    o = EqsOracle(case)
    assert o.dense
    ref = o.rkc_trajectory(np.zeros(o.n_free), 0.0, case.tau, case.s, steps)
    with ctx_for(case, precision) as c:
        x = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        worst, its = 0.0, 0
        for n in range(steps):
            st = c.rkc_step(n * case.tau, case.tau, case.s, x, rtol=1e-12, maxit=500)
            its += st["total_iters"]
            worst = max(worst, np.linalg.norm(x.cpu().numpy()[o.free] - ref[n + 1]))
    err = worst / max(np.linalg.norm(r) for r in ref)
    print(f"[p2] slab, {steps} RKC({case.s}) steps, precision {precision}: err {err:.2e}, {its} CG iterations",
          flush=True)
    assert err <= 1e-9


def test_p2_inclusions_first_steps_match_oracle():
    case = eqsgen.case_p2(n=12, seed=1)
    case.s = 12
    o = EqsOracle(case, solver="jacobi", warm=True)
    ref = o.rkc_trajectory(np.zeros(o.n_free), 0.0, case.tau, case.s, 3)
    with ctx_for(case, EQS_PREC_FP32) as c:
        x = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        got = [np.zeros(o.n_free)]
        for n in range(3):
            c.rkc_step(n * case.tau, case.tau, case.s, x, rtol=1e-12, maxit=500)
            got.append(x.cpu().numpy()[o.free])
    err = max(np.linalg.norm(a - b) for a, b in zip(got, ref)) / max(np.linalg.norm(r) for r in ref)
    print(f"[p2] inclusions n=12 ({o.n_free} free DOF), 3 RKC(12) steps: err {err:.2e}", flush=True)
    assert err <= 1e-9


def test_p2_full_size_element_pass_and_M_product():
    """The second-order workload at 2.1M free DOF (64^3 cubes, 1.57M 10-node
    tets): the element pass on every node and the M product on every row."""
    case = eqsgen.case_p2(n=64, seed=1)
    print(f"[p2] full size: {case.n_nodes} nodes, {case.n_tets} tets", flush=True)
    is_dir = np.zeros(case.n_nodes, bool)
    is_dir[case.dir_nodes] = True
    free = np.flatnonzero(~is_dir)
    with ctx_for(case, EQS_PREC_FP32) as c:
        print("[p2] " + c.describe().splitlines()[1], flush=True)
        x = smooth_state(case, 7)
        t = 0.0031
        y = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        c.apply_K(t, T(x), y)
        xbar = x.copy()
        xbar[case.dir_nodes] = (case.amp * np.sin(2 * np.pi * case.freq * t + case.phase))[case.dir_drive]
        ref, rate = fem.apply_K(case, xbar, with_rate=True)
        e1 = relinf(y.cpu().numpy(), ref)
        M = fem.assemble_M(case)[free][:, free].tocsr()
        v = np.random.default_rng(8).normal(size=free.size)
        z = torch.zeros(free.size, dtype=torch.float64, device=DEV)
        c.apply_M(T(v), z)
        e2 = relinf(z.cpu().numpy(), fem.csr_matvec(M, v))
        print(f"[p2] full size: element pass {e1:.2e} (max sigma/eps {rate:.3g}), M product {e2:.2e}, "
              f"nnz(M) {M.nnz}", flush=True)
        assert e1 <= 1e-12 and e2 <= 1e-13
