"""Code paths that the workloads do not reach by themselves, forced by the
library's test switches (read when a context is created) and checked against
the FP64 oracle:

* EQS_KX_GENERIC=1: the element pass with each block's own LDS stride, the
  path taken by element blocks with more distinct nodes than the fixed stride
  (Sec. III's fused K(x)x); element by element to 1e-12.
* EQS_TUNE_FILE: the layout and block-size choices of one build are recorded
  and a second build replays them without timing, giving the same
  preconditioner; a malformed record is refused.
* EQS_TEST_REJECT_CHECK=1: the true-residual check that ends every CG solve
  reports "not converged" once per solve, so each solve restarts from its true
  residual; with the plain start vector the rest of the stage and the next
  stage's element pass are already queued behind that check and are queued
  again for the final solution. RKC trajectories (Sec. II) to 1e-9.
"""

import numpy as np
import pytest

import eqsgen
from oracle import fem
from oracle.eqs import EqsOracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1612_09447_amd import EQS_PREC_FP32, EQS_PREC_FP64, Context, EqsError  # noqa: E402

DEV = torch.device("cuda:0")


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def relinf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def make_ctx(case, precision=EQS_PREC_FP64):
    c = Context(0, torch.cuda.current_stream(DEV))
    c.setup_case(case, precision=precision)
    return c


@pytest.mark.parametrize("maker", [lambda: eqsgen.case_c0(8), lambda: eqsgen.case_c1(n=40, seed=2)])
def test_element_pass_per_block_stride_matches_oracle(maker, monkeypatch):
    case = maker()
    monkeypatch.setenv("EQS_KX_GENERIC", "1")
    o = EqsOracle(case, dense_limit=0)
    with make_ctx(case) as c:
        desc = c.describe()
        print("[paths] " + desc.splitlines()[1], flush=True)
        assert "per-block LDS stride" in desc
        for seed, scale, t in [(1, 0.3, 0.0017), (2, 2.5, 0.0041)]:
            x = eqsgen.random_state(case.n_nodes, seed, scale)
            y = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
            c.apply_K(t, T(x), y)
            ref = fem.apply_K(case, o.embed(x[o.free], t))
            assert relinf(y.cpu().numpy(), ref) <= 1e-12
            r = torch.zeros(o.n_free, dtype=torch.float64, device=DEV)
            c.stage_rhs(t, T(x[o.free]), r)
            assert relinf(r.cpu().numpy(), o.stage_rhs(t, x[o.free])) <= 1e-12


def test_tuning_record_replays_the_same_layouts(tmp_path, monkeypatch):
    case = eqsgen.case_c1(n=20, seed=3)
    rec = tmp_path / "tune.txt"
    monkeypatch.setenv("EQS_TUNE_FILE", str(rec))
    x = eqsgen.random_state(case.n_nodes, 9, 1.0)
    outs = []
    for k in range(2):
        with make_ctx(case, EQS_PREC_FP32) as c:
            desc = c.describe()
            n = c.info()["n_free"]
            r = T(np.random.default_rng(4).normal(size=n))
            z = torch.zeros(n, dtype=torch.float64, device=DEV)
            c.apply_preconditioner(r, z)
            outs.append((desc, z.cpu().numpy()))
        if k == 0:
            lines = rec.read_text().splitlines()
            print(f"[paths] tuning record: {len(lines)} entries, e.g. {lines[:2]}", flush=True)
            assert any(l.startswith("element ") for l in lines) and any("\tsell " in l or "\tcsr " in l for l in lines)
    assert "(tuning record)" not in outs[0][0] and outs[1][0].count("(tuning record)") == len(lines)
    assert np.array_equal(outs[0][1], outs[1][1])  # same layouts, same summation order
    rec.write_text(lines[0].split("\t")[0] + "\tsell 3 0 8\n")
    with pytest.raises(EqsError):
        make_ctx(case, EQS_PREC_FP32)


def run(case, steps, rtol, precision):
    with make_ctx(case, precision) as c:
        x = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        out, its = [], 0
        for n in range(steps):
            st = c.rkc_step(n * case.tau, case.tau, case.s, x, rtol=rtol, maxit=500)
            assert st["max_relres"] <= rtol
            its += st["total_iters"]
            out.append(x.cpu().numpy().copy())
    return out, its


@pytest.mark.parametrize("precision", [EQS_PREC_FP64, EQS_PREC_FP32])
def test_restart_after_rejected_check_keeps_trajectory(precision, monkeypatch):
    case = eqsgen.case_c0(8)
    case.amp[1] = 3.0  # into the varistor's nonlinear range
    steps, rtol = 12, 1e-12
    o = EqsOracle(case)
    ref = o.rkc_trajectory(np.zeros(o.n_free), 0.0, case.tau, case.s, steps)
    plain, its_plain = run(case, steps, rtol, precision)
    monkeypatch.setenv("EQS_TEST_REJECT_CHECK", "1")
    forced, its_forced = run(case, steps, rtol, precision)
    scale = max(np.linalg.norm(r) for r in ref)
    err = max(np.linalg.norm(f[o.free] - r) for f, r in zip(forced, ref[1:])) / scale
    dif = max(np.linalg.norm(f - p) for f, p in zip(forced, plain)) / scale
    print(f"[paths] restart path precision={precision}: err vs oracle {err:.2e}, vs unforced run {dif:.2e}, "
          f"CG iterations {its_forced} (unforced {its_plain})", flush=True)
    assert its_forced > its_plain  # every solve iterated again after its rejected check
    assert err <= 1e-9
    assert dif <= 1e-9
