"""Parity of the batched workload (64 instances, n in {16, ..., 48}): every
instance of the packed batch against the same instance run alone, one RKC(8)
step. (The c1 and c2 trajectories against the oracle are in
test_gpu_trajectory.py.)
"""

import numpy as np
import pytest

import eqsgen

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
