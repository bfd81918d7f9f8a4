"""Deterministic element pass (eqs_set_deterministic): K(x)x summed in an
order fixed at set-up instead of by FP64 atomics (Sec. III's fused K(x)x).

Against the oracle element by element (1e-12 relative, as the atomic pass);
two passes, and two RKC trajectories on separate contexts with the same
operator layouts, equal bit for bit;
the same with each block's own LDS stride; the switch is refused after the
build and for second-order meshes.
"""

import numpy as np
import pytest

import eqsgen
from oracle import fem
from oracle.eqs import EqsOracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1612_09447_amd import EQS_ERR_INVALID_ARG, EQS_ERR_STATE, EQS_PREC_FP32, Context, EqsError  # noqa: E402

DEV = torch.device("cuda:0")


def T(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64), device=DEV)


def relinf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def ctx(case, deterministic=True, precision=None):
    c = Context(0, torch.cuda.current_stream(DEV))
    c.setup_case(case, precision=precision, deterministic=deterministic)
    return c


@pytest.mark.parametrize("generic", [False, True])
@pytest.mark.parametrize("maker", [lambda: eqsgen.case_c0(8), lambda: eqsgen.case_c1(n=14, seed=4),
                                   lambda: eqsgen.case_c1(n=40, seed=2)])
def test_deterministic_pass_matches_oracle_and_repeats_bitwise(maker, generic, monkeypatch):
    case = maker()
    if generic:
        monkeypatch.setenv("EQS_KX_GENERIC", "1")
    o = EqsOracle(case, dense_limit=0)
    with ctx(case) as c:
        line = c.describe().splitlines()[1]
        print(f"[det] {case.name} n={case.n}: {line}", flush=True)
        assert ("deterministic sums" in line) != generic and ("per-block LDS stride" in line) == generic
        for seed, scale, t in [(1, 0.3, 0.0017), (2, 2.5, 0.0041)]:
            x = eqsgen.random_state(case.n_nodes, seed, scale)
            ys = []
            for _ in range(2):
                y = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
                c.apply_K(t, T(x), y)
                ys.append(y.cpu().numpy())
            assert np.array_equal(ys[0], ys[1])
            assert relinf(ys[0], fem.apply_K(case, o.embed(x[o.free], t))) <= 1e-12
            rs = []
            for _ in range(2):
                r = torch.zeros(o.n_free, dtype=torch.float64, device=DEV)
                c.stage_rhs(t, T(x[o.free]), r)
                rs.append(r.cpu().numpy())
            assert np.array_equal(rs[0], rs[1])
            assert relinf(rs[0], o.stage_rhs(t, x[o.free])) <= 1e-12


def test_deterministic_trajectories_repeat_bitwise_and_match_oracle(monkeypatch):
    # two contexts sum in the same order only with the same operator layouts:
    # the rule-based ones (the autotuner's timings may choose differently per build)
    monkeypatch.setenv("EQS_AUTOTUNE", "0")
    case = eqsgen.case_c1(n=12, seed=5)
    case.s = 12
    steps = 3
    o = EqsOracle(case)
    ref = o.rkc_trajectory(np.zeros(o.n_free), 0.0, case.tau, case.s, steps)
    finals = []
    for _ in range(2):
        with ctx(case, precision=EQS_PREC_FP32) as c:
            x = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
            worst = 0.0
            for n in range(steps):
                c.rkc_step(n * case.tau, case.tau, case.s, x, rtol=1e-12, maxit=500)
                worst = max(worst, np.linalg.norm(x.cpu().numpy()[o.free] - ref[n + 1]))
            finals.append(x.cpu().numpy())
        err = worst / max(np.linalg.norm(r) for r in ref)
        print(f"[det] c1 n=12, {steps} RKC({case.s}) steps on the FP32 hierarchy: err {err:.2e}", flush=True)
        assert err <= 1e-9
    assert np.array_equal(finals[0], finals[1])


def test_deterministic_switch_limits():
    case = eqsgen.case_c0(8)
    with ctx(case, deterministic=False) as c:
        c.set_deterministic(False)  # unchanged: accepted
        with pytest.raises(EqsError) as e:
            c.set_deterministic(True)
        assert e.value.code == EQS_ERR_STATE
    p2 = eqsgen.case_c0_p2(4)
    c = Context(0, torch.cuda.current_stream(DEV))
    with pytest.raises(EqsError) as e:
        c.setup_case(p2, deterministic=True)
    assert e.value.code == EQS_ERR_INVALID_ARG
    c.close()
