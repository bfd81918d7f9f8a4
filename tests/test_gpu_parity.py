"""GPU parity: every entry point of the C ABI against the FP64 CPU oracle.

Sizes are small enough for the oracle's dense solves (several SELL slices and
256-thread blocks, ragged tails), plus the workload shapes of the slab (c0)
and inclusion (c1/c2) recipes. Tolerances (floating point, FP64 path):
  * element pass and SpMV: |gpu - oracle|_inf <= 1e-12 |oracle|_inf (rounding
    order of the atomics and of the two element formulas);
  * trajectories: max_n |x_n - x_n^ref| / max_n |x_n^ref| <= 1e-9 with CG at
    rel-res 1e-12 (plain FP64) and <= 1e-8 with the FP32 preconditioner.
"""

import numpy as np
import pytest

import eqsgen
from oracle import fem
from oracle.eqs import EqsOracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1612_09447_amd import (  # noqa: E402
    EQS_ERR_BREAKDOWN,
    EQS_ERR_INVALID_ARG,
    EQS_ERR_NOT_CONVERGED,
    EQS_ERR_STATE,
    EQS_PREC_FP32,
    EQS_PREC_FP64,
    Context,
    EqsError,
)

DEV = torch.device("cuda:0")


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def N(t):
    return t.detach().cpu().numpy()


def ctx_for(case, precision=None, **amg):
    c = Context(0, torch.cuda.current_stream(DEV))
    c.setup_case(case, precision=precision, **amg)
    return c


def inclusion_case(n, seed=1):
    c = eqsgen.case_c1(n=n, seed=seed)
    return c


def relinf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# ------------------------------------------------------------ element pass
@pytest.mark.parametrize("maker", [lambda: eqsgen.case_c0(8), lambda: inclusion_case(12), lambda: inclusion_case(7, 3)])
def test_apply_K_matches_oracle(maker):
    case = maker()
    print(f"[apply_K] case {case.name} n={case.n} tets={case.n_tets}", flush=True)
    with ctx_for(case) as c:
        for seed, scale in [(1, 0.05), (2, 1.0), (3, 4.0)]:
            x = eqsgen.random_state(case.n_nodes, seed, scale)
            t = 0.0031 * seed
            y = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
            c.apply_K(t, T(x), y)
            o = EqsOracle(case)
            xbar = o.embed(x[o.free], t)
            ref = fem.apply_K(case, xbar)
            assert relinf(N(y), ref) <= 1e-12, (seed, relinf(N(y), ref))


def test_element_pass_on_many_blocks_matches_oracle():
    """The element pass on a mesh of 2.6 M tets (2,573 blocks of 1,024), whose
    blocks include nodes shared between many blocks, against the oracle."""
    case = inclusion_case(76, 2)
    o = EqsOracle(case)
    with ctx_for(case) as c:
        print("[element] " + c.describe().splitlines()[1], flush=True)
        x = eqsgen.random_state(case.n_nodes, 5, 1.5)
        t = 0.0023
        y = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        c.apply_K(t, T(x), y)
        ref = fem.apply_K(case, o.embed(x[o.free], t))
        assert relinf(N(y), ref) <= 1e-12
        r = torch.zeros(o.n_free, dtype=torch.float64, device=DEV)
        c.stage_rhs(t, T(x[o.free]), r)
        assert relinf(N(r), o.stage_rhs(t, x[o.free])) <= 1e-12


def test_apply_K_relies_on_connectivity_only():
    case = inclusion_case(9, 5)
    x = eqsgen.random_state(case.n_nodes, 7, 2.0)
    xyz2, tets2, dn2, perm = eqsgen.permute_nodes(case.xyz, case.tets, case.dir_nodes, seed=11)
    case2 = eqsgen.make_case("c1", n=9, seed=5)
    case2.xyz, case2.tets, case2.dir_nodes = xyz2, tets2, dn2
    case2.tets, case2.tet_mat, _ = eqsgen.shuffle_tets(case2.tets, case2.tet_mat, seed=12)
    x2 = np.empty_like(x)
    x2[perm] = x
    with ctx_for(case) as c1, ctx_for(case2) as c2:
        y1 = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        y2 = torch.zeros_like(y1)
        c1.apply_K(0.002, T(x), y1)
        c2.apply_K(0.002, T(x2), y2)
        assert relinf(N(y2)[perm], N(y1)) <= 1e-12


def test_stage_rhs_matches_oracle():
    case = inclusion_case(12)
    o = EqsOracle(case)
    with ctx_for(case) as c:
        for t in [0.0, 0.0013, 0.0047]:
            Y = eqsgen.random_state(case.n_nodes, 4, 0.7)[o.free]
            r = torch.zeros(o.n_free, dtype=torch.float64, device=DEV)
            c.stage_rhs(t, T(Y), r)
            ref = o.stage_rhs(t, Y)
            assert relinf(N(r), ref) <= 1e-12, t


def test_apply_M_matches_oracle():
    case = inclusion_case(13, 2)
    o = EqsOracle(case)
    with ctx_for(case) as c:
        info = c.info()
        # the library stores only entries above roundoff (Kuhn tets give exact
        # zeros on face and body diagonals); the oracle keeps the structural pattern
        A = o.M_II.tocoo()
        d = o.M_II.diagonal()
        keep = (A.row == A.col) | (np.abs(A.data) > 1e-14 * np.sqrt(np.abs(d[A.row] * d[A.col])))
        assert info["n_free"] == o.n_free and info["nnz_M"] == int(keep.sum())
        # nearly uniform first-order rows keep the natural row order (second-order M sorts; tests/test_gpu_p2.py)
        assert "M: sell64," in c.describe()
        x = np.random.default_rng(0).normal(size=o.n_free)
        y = torch.zeros(o.n_free, dtype=torch.float64, device=DEV)
        c.apply_M(T(x), y)
        assert relinf(N(y), o.M_II @ x) <= 1e-13


# ---------------------------------------------------------- preconditioner
@pytest.mark.parametrize("prec,tol", [(EQS_PREC_FP64, 1e-12), (EQS_PREC_FP32, 2e-5)])
def test_preconditioner_symmetric_positive(prec, tol):
    case = inclusion_case(14, 4)
    with ctx_for(case, precision=prec) as c:
        info = c.info()
        assert info["n_levels"] >= 2, info
        n = info["n_free"]
        rng = np.random.default_rng(1)
        X, Y = rng.normal(size=n), rng.normal(size=n)
        bx = torch.zeros(n, dtype=torch.float64, device=DEV)
        by = torch.zeros_like(bx)
        c.apply_preconditioner(T(X), bx)
        c.apply_preconditioner(T(Y), by)
        bx, by = N(bx), N(by)
        assert abs(bx @ Y - X @ by) <= tol * np.linalg.norm(bx) * np.linalg.norm(Y)
        assert bx @ X > 0 and by @ Y > 0
        # V-cycle is a contraction in the energy norm: I - B M has spectral radius < 1
        o = EqsOracle(case)
        e = rng.normal(size=n)
        for _ in range(3):
            be = torch.zeros(n, dtype=torch.float64, device=DEV)
            c.apply_preconditioner(T(o.M_II @ e), be)
            e_new = e - N(be)
            ratio = np.sqrt(e_new @ (o.M_II @ e_new)) / np.sqrt(e @ (o.M_II @ e))
            assert ratio < 0.9, ratio
            e = e_new


@pytest.mark.parametrize("prec,tol", [(EQS_PREC_FP64, 1e-12), (EQS_PREC_FP32, 2e-5)])
def test_preconditioner_same_in_every_layout(prec, tol, monkeypatch):
    """Each storage layout of the coarse operators (SELL with 1, 2, 4, 8 lanes
    per row, with and without rows sorted by length within windows, with 4, 8
    or 16 entries per lane in flight, CSR with lanes)
    gives the same V-cycle up to summation order."""
    case = inclusion_case(14, 4)
    n = None
    outs = {}
    X = None
    layouts = [(lay, "8") for lay in ("sell1", "sell2", "sell4", "sell8", "csr", "sell1s", "sell2s", "sell4s", "sell8s")]
    layouts += [("sell1", "4"), ("sell1s", "16"), ("sell2s", "4"), ("sell4", "16"), ("sell8s", "16")]
    for lay, unroll in layouts:
        monkeypatch.setenv("EQS_LAYOUT", lay)
        monkeypatch.setenv("EQS_UNROLL", unroll)
        with ctx_for(case, precision=prec, coarse_max=24) as c:
            info = c.info()
            assert info["n_levels"] >= 3, info  # coarse levels smooth in the forced layout
            assert "layout set by EQS_LAYOUT" in c.describe()
            if X is None:
                n = info["n_free"]
                X = np.random.default_rng(7).normal(size=n)
            z = torch.zeros(n, dtype=torch.float64, device=DEV)
            c.apply_preconditioner(T(X), z)
            outs[lay, unroll] = N(z)
            print(f"[layout] prec={prec} {lay} u{unroll} levels={info['n_levels']}", flush=True)
    for key, z in outs.items():
        assert relinf(z, outs["sell1", "8"]) <= tol, key
    monkeypatch.setenv("EQS_UNROLL", "6")
    with pytest.raises(EqsError):
        Context(0, torch.cuda.current_stream(DEV))
    monkeypatch.setenv("EQS_UNROLL", "8")
    monkeypatch.setenv("EQS_LAYOUT", "sell3")
    with pytest.raises(EqsError):
        Context(0, torch.cuda.current_stream(DEV))


@pytest.mark.parametrize("coarse_max,min_levels", [(8, 4), (512, 2)])
@pytest.mark.parametrize("prec,tol", [(EQS_PREC_FP64, 1e-12), (EQS_PREC_FP32, 2e-5)])
def test_folded_vcycle_matches_plain(prec, tol, coarse_max, min_levels, monkeypatch):
    """The folded operators (pre-smoothers inside the restrictions, the two
    lowest levels as two products) give the plain V(1,1) cycle up to rounding,
    on a deep hierarchy and on a two-level one."""
    case = inclusion_case(14, 4)
    outs = {}
    X = None
    for fold in ("0", "1"):
        monkeypatch.setenv("EQS_FOLD", fold)
        with ctx_for(case, precision=prec, coarse_max=coarse_max) as c:
            info = c.info()
            assert info["n_levels"] >= min_levels, info
            d = c.describe()
            # folded: every level strictly between the finest and the tail
            # restricts through R (I - A w D^-1); the tail needs three levels
            assert ("(I-AwD^-1)" in d) == (fold == "1" and info["n_levels"] >= 4), d
            assert ("[G Q]" in d) == (fold == "1" and info["n_levels"] >= 3), d
            if X is None:
                X = np.random.default_rng(11).normal(size=info["n_free"])
            z = torch.zeros(info["n_free"], dtype=torch.float64, device=DEV)
            c.apply_preconditioner(T(X), z)
            outs[fold] = N(z)
            print(f"[fold] prec={prec} fold={fold} levels={info['level_rows']}", flush=True)
    assert relinf(outs["1"], outs["0"]) <= tol


# ------------------------------------------------------------------ solve
@pytest.mark.parametrize("prec", [EQS_PREC_FP64, EQS_PREC_FP32])
def test_solve_M_matches_dense(prec):
    case = inclusion_case(12, 6)
    o = EqsOracle(case)
    rng = np.random.default_rng(3)
    rhs = rng.normal(size=o.n_free)
    ref = o.solve(rhs)
    with ctx_for(case, precision=prec) as c:
        y = torch.zeros(o.n_free, dtype=torch.float64, device=DEV)
        st = c.solve_M(T(rhs), y, rtol=1e-11, maxit=300)
        print(f"[solve_M] prec={prec} iters={st['iters']} relres={st['relres']:.2e}", flush=True)
        got = N(y)
        true_rr = np.linalg.norm(rhs - o.M_II @ got) / np.linalg.norm(rhs)
        assert st["relres"] <= 1e-11 and true_rr <= 1.5e-11
        assert abs(st["relres"] - true_rr) <= 1e-12
        assert np.linalg.norm(got - ref) <= 1e-8 * np.linalg.norm(ref)
        assert st["iters"] < 60


def test_solve_M_edge_cases():
    case = inclusion_case(10, 2)
    o = EqsOracle(case)
    rng = np.random.default_rng(4)
    with ctx_for(case) as c:
        n = o.n_free
        # exact start vector: no iterations (Sec. IV: an accurate start vector needs none)
        rhs = rng.normal(size=n)
        y = T(o.solve(rhs))
        st = c.solve_M(T(rhs), y, rtol=1e-10)
        assert st["iters"] == 0
        # zero right-hand side: zero solution whatever the start
        y = T(rng.normal(size=n))
        st = c.solve_M(T(np.zeros(n)), y, rtol=1e-10)
        assert st["iters"] == 0 and not N(y).any()
        # iteration limit is reported, results still written
        y = torch.zeros(n, dtype=torch.float64, device=DEV)
        st = c.solve_M(T(rhs), y, rtol=1e-14, maxit=2, allow_not_converged=True)
        assert st["rc"] == EQS_ERR_NOT_CONVERGED and st["iters"] == 2 and st["relres"] < 1
        # a garbage start (scaled by 1e30) still converges
        y = T(1e30 * rng.normal(size=n))
        st = c.solve_M(T(rhs), y, rtol=1e-10, maxit=400)
        assert np.linalg.norm(rhs - o.M_II @ N(y)) <= 2e-10 * np.linalg.norm(rhs)


def test_nonfinite_values_end_in_breakdown_and_the_context_recovers():
    """A NaN that reaches the CG scalars ends the solve with EQS_ERR_BREAKDOWN
    (forced from the host: every kernel runs to its end on NaN data): in the
    right-hand side of eqs_solve_M and, through the element pass, in a free
    potential of eqs_rkc_step. The context then solves and steps as before: a
    step from a finite state matches a fresh context's step."""
    case = eqsgen.case_c0(8)
    case.amp[1] = 3.0
    rng = np.random.default_rng(5)
    with ctx_for(case) as c, ctx_for(case) as fresh:
        n = c.info()["n_free"]
        rhs = rng.normal(size=n)
        rhs[n // 2] = np.nan
        y = torch.zeros(n, dtype=torch.float64, device=DEV)
        with pytest.raises(EqsError) as e:
            c.solve_M(T(rhs), y, rtol=1e-10, maxit=100)
        assert e.value.code == EQS_ERR_BREAKDOWN
        rhs[n // 2] = 1.0
        y.zero_()
        assert c.solve_M(T(rhs), y, rtol=1e-10, maxit=400)["relres"] <= 1.01e-10
        free = np.setdiff1d(np.arange(case.n_nodes), case.dir_nodes)
        x = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        x[int(free[len(free) // 3])] = float("nan")
        with pytest.raises(EqsError) as e:
            c.rkc_step(0.0, case.tau, case.s, x, rtol=1e-10, maxit=100)
        assert e.value.code == EQS_ERR_BREAKDOWN
        x.zero_()
        xf = torch.zeros_like(x)
        for k in range(2):
            st = c.rkc_step(k * case.tau, case.tau, case.s, x, rtol=1e-10)
            stf = fresh.rkc_step(k * case.tau, case.tau, case.s, xf, rtol=1e-10)
        d = float((x - xf).norm() / xf.norm())
        print(f"[breakdown] after the failed step: {st['total_iters']} vs {stf['total_iters']} CG iterations, "
              f"rel. difference to a fresh context {d:.1e}", flush=True)
        # equal iteration counts: equal up to the order of the element pass's atomic adds; else (a
        # convergence test on the other side of its threshold) equal to the solve tolerance
        assert d <= (1e-12 if st["total_iters"] == stf["total_iters"] else 1e-9)


def test_call_order_and_argument_errors():
    case = inclusion_case(5, 2)
    c = Context(0, torch.cuda.current_stream(DEV))
    x = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
    with pytest.raises(EqsError) as e:
        c.apply_K(0.0, x, torch.zeros_like(x))
    assert e.value.code == EQS_ERR_STATE
    with pytest.raises(EqsError) as e:
        c.set_materials(case.eps_r, case.kappa0, case.e_s, case.alpha, case.nonlinear, case.tet_mat)
    assert e.value.code == EQS_ERR_STATE
    c.set_mesh(case.xyz, case.tets)
    bad = case.tets.copy()
    bad[3] = [0, 1, 2, 0]
    with pytest.raises(EqsError) as e:
        c.set_mesh(case.xyz, np.where(bad < 0, 0, bad) * 0 + 10 ** 7)
    assert e.value.code == EQS_ERR_INVALID_ARG
    c.set_mesh(case.xyz, bad)
    c.set_materials(case.eps_r, case.kappa0, case.e_s, case.alpha, case.nonlinear, case.tet_mat)
    c.set_dirichlet(case.dir_nodes, case.dir_drive, case.amp, case.freq, case.phase)
    with pytest.raises(EqsError) as e:  # flat tet found at build time
        c.build_preconditioner()
    assert e.value.code == EQS_ERR_INVALID_ARG and "zero volume" in str(e.value)
    c.close()


# ------------------------------------------------------------ RKC steps
def trajectory_error(case, steps, rtol, precision=None, **amg):
    o = EqsOracle(case)
    ref = o.rkc_trajectory(np.zeros(o.n_free), 0.0, case.tau, case.s, steps)
    with ctx_for(case, precision=precision, **amg) as c:
        x = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        worst, iters = 0.0, []
        for n in range(steps):
            st = c.rkc_step(n * case.tau, case.tau, case.s, x, rtol=rtol, maxit=500)
            iters.append(st["total_iters"] / st["stages"])
            got = N(x)
            worst = max(worst, np.linalg.norm(got[o.free] - ref[n + 1]))
            # Dirichlet entries hold g(t_{n+1})
            g = o.g((n + 1) * case.tau)
            dg = float(np.abs(got[o.dir_nodes] - g).max())
            assert dg <= 1e-13 * max(1.0, float(np.abs(g).max())), dg  # same sine, rounded in another order
    scale = max(np.linalg.norm(r) for r in ref)
    return worst / scale, float(np.mean(iters))


def test_rkc_c0_full_trajectory_plain_fp64():
    """c0: n = 8, slab, 200 RKC(8) steps at the recipe tolerance 1e-10."""
    case = eqsgen.case_c0(8)
    err, it = trajectory_error(case, case.steps, case.rtol)
    print(f"[rkc c0] err={err:.3e} mean CG iters/stage={it:.2f}", flush=True)
    assert err <= 1e-9


def test_rkc_strongly_nonlinear_slab():
    case = eqsgen.case_c0(8)
    case.amp[1] = 3.2
    err, it = trajectory_error(case, 60, 1e-12)
    print(f"[rkc c0 strong] err={err:.3e} iters={it:.2f}", flush=True)
    assert err <= 1e-9


def test_rkc_inclusions_plain_and_mixed():
    case = inclusion_case(12, 1)
    case.s = 12
    err64, it64 = trajectory_error(case, 6, 1e-12, EQS_PREC_FP64)
    err32, it32 = trajectory_error(case, 6, 1e-10, EQS_PREC_FP32)
    print(f"[rkc incl] fp64 err={err64:.3e} it={it64:.2f}; fp32-AMG err={err32:.3e} it={it32:.2f}", flush=True)
    assert err64 <= 1e-9
    assert err32 <= 1e-8


def test_rkc_single_level_hierarchy():
    case = eqsgen.case_c0(4)  # 75 free nodes: the dense coarse solve is the preconditioner
    err, it = trajectory_error(case, 5, 1e-12)
    assert err <= 1e-9 and it <= 2


def test_stage_iterations_of_the_last_step():
    """eqs_stage_iters: one count per stage of the last RKC step, in stage
    order, adding up to the step's total with the step's extremes; a call
    that its argument checks reject changes nothing, a new set-up clears it."""
    case = eqsgen.case_c0(8)
    case.amp[1] = 3.0
    with ctx_for(case) as c:
        assert c.stage_iters() == []
        x = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        for n in range(3):
            st = c.rkc_step(n * case.tau, case.tau, case.s, x, rtol=1e-10)
            its = st["stage_iters"]
            print(f"[stage_iters] step {n + 1}: {its}", flush=True)
            assert len(its) == case.s == st["stages"] and sum(its) == st["total_iters"]
            assert max(its) == st["max_iters"] and min(its) == st["min_iters"]
        with pytest.raises(EqsError) as e:
            c.rkc_step(0.0, case.tau, 1, x, rtol=1e-10)
        assert e.value.code == EQS_ERR_INVALID_ARG
        assert c.stage_iters() == its
        c.setup_case(case)
        assert c.stage_iters() == []


def test_profile_counts_launches_that_worked():
    """Kernel-class timing: one element pass and one combination per stage,
    one launch of each CG-iteration class per iteration that did work (the
    launches enqueued after convergence return at entry and are not counted)."""
    # four levels or more: the finest restriction is a product of its own and
    # level 1 smooths on its own (not folded into the coarse tail)
    case = inclusion_case(24, 4)
    classes = ("element", "spmv_M", "presmooth0", "postsmooth0", "vcycle", "cg_update", "rkc_combine",
               "restrict0", "prolong0", "vcoarse", "finalise", "postsmooth1")
    with ctx_for(case, precision=EQS_PREC_FP32, coarse_max=32) as c:
        x = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        c.rkc_step(0.0, case.tau, case.s, x, rtol=1e-10)
        c.profile_enable(classes)
        st = c.rkc_step(case.tau, case.tau, case.s, x, rtol=1e-10)
        prof = {k: c.profile_read(k) for k in classes}
        c.profile_enable(())
        n_levels = c.info()["n_levels"]
    print(f"[profile] {st['total_iters']} iterations: " +
          ", ".join(f"{k} {v['launches']}x{1e3 * v['avg_ms']:.1f}us" for k, v in prof.items()), flush=True)
    assert prof["element"]["launches"] == case.s and prof["rkc_combine"]["launches"] == case.s
    assert n_levels >= 4
    for k in ("spmv_M", "presmooth0", "postsmooth0", "vcycle", "cg_update", "restrict0", "prolong0", "vcoarse",
              "postsmooth1"):
        assert prof[k]["launches"] == st["total_iters"], (k, prof[k], st)
    assert prof["finalise"]["launches"] == 3 * st["total_iters"]
    for k in classes:
        assert prof[k]["total_ms"] > 0.0, k
