"""Parity on the benchmark workloads beyond the small cases.

* C1 (64^3 cubes, 266,175 free DOF, RKC(12)): the first step against the FP64
  oracle (SGS-PCG to rel-res 1e-13), for the plain FP64 path and the FP32
  precision form, with CG at rel-res 1e-12 (the kernels' own error), and the
  precision form at the workload's tolerance 1e-8 for the record.
* C3 (64 instances, n in {16, ..., 48}): every instance of the packed batch
  against the same instance run alone, one RKC(8) step.
"""

import numpy as np
import pytest

import eqsgen
from oracle.eqs import EqsOracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1612_09447_amd import EQS_PREC_FP32, EQS_PREC_FP64, Batch, Context  # noqa: E402

DEV = torch.device("cuda:0")


def run(case, precision, steps, rtol):
    with Context(0, torch.cuda.current_stream(DEV)) as c:
        c.setup_case(case, precision=precision)
        x = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        its = 0
        for n in range(steps):
            st = c.rkc_step(n * case.tau, case.tau, case.s, x, rtol=rtol, maxit=500)
            its += st["total_iters"]
        return x.cpu().numpy(), its


def test_c1_first_step_matches_oracle():
    case = eqsgen.case_c1()
    print(f"[c1] {case.n_nodes} nodes, {case.n_tets} tets, s={case.s}", flush=True)
    o = EqsOracle(case)
    ref = o.rkc_trajectory(np.zeros(o.n_free), 0.0, case.tau, case.s, 1)
    scale = max(np.linalg.norm(r) for r in ref)
    for prec, rtol, bar in [(EQS_PREC_FP64, 1e-12, 1e-9), (EQS_PREC_FP32, 1e-12, 1e-9), (EQS_PREC_FP32, 1e-8, 1e-6)]:
        x, its = run(case, prec, 1, rtol)
        err = np.linalg.norm(x[o.free] - ref[-1]) / scale
        print(f"[c1] precision {prec} rtol {rtol:g}: err {err:.2e}, {its} CG iterations", flush=True)
        assert err <= bar, (prec, rtol, err)
        assert np.abs(x[o.dir_nodes] - o.g(case.tau)).max() <= 1e-13


def test_c3_batch_instances_match_standalone_runs():
    cases = eqsgen.case_batch()
    rtol = 1e-10
    stream = torch.cuda.current_stream(DEV)
    inputs = []
    for c in cases:
        ctx = Context(0, stream)
        ctx.set_inputs(c)
        inputs.append(ctx)
    b = Batch(inputs, precision=EQS_PREC_FP32, stream=stream)
    for ctx in inputs:
        ctx.close()
    xs = [torch.zeros(c.n_nodes, dtype=torch.float64, device=DEV) for c in cases]
    res = b.rkc_steps(1, 0.0, cases[0].tau, cases[0].s, xs, rtol)
    b.close()
    print(f"[c3] {len(cases)} instances, per-instance CG iterations {res['iters'].min()}..{res['iters'].max()}",
          flush=True)
    assert (res["relres"] <= rtol * 1.01).all()
    worst = 0.0
    for c, xb in zip(cases, xs):
        alone, _ = run(c, EQS_PREC_FP32, 1, rtol)
        d = np.linalg.norm(xb.cpu().numpy() - alone) / np.linalg.norm(alone)
        worst = max(worst, d)
    print(f"[c3] worst relative difference batch vs alone: {worst:.2e}", flush=True)
    assert worst <= 1e-8
