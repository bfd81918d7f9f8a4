"""Batched form: independent instances packed into one context.

Every instance of a batch must follow its own trajectory: checked against the
FP64 oracle (rel. L2 <= 1e-9 over the trajectory, CG at rel-res 1e-12) and
against the same instance run alone. Instances of different sizes, materials
and drives converge in different numbers of CG iterations.
"""

import numpy as np
import pytest

import eqsgen
from eqsgen.cases import _inclusion_case
from oracle.eqs import EqsOracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1612_09447_amd import EQS_ERR_INVALID_ARG, EQS_PREC_FP64, Batch, Context, EqsError  # noqa: E402

DEV = torch.device("cuda:0")
SPECS = [(7, 11, 1.0, 50.0), (9, 12, 1.6, 80.0), (11, 13, 0.7, 30.0), (8, 14, 1.9, 65.0)]


def instances():
    out = []
    for n, seed, amp, freq in SPECS:
        c = _inclusion_case("c3", n, seed, (2.0, 15.0), (6.0, 14.0), amp=amp, freq=freq)
        c.s, c.tau = 8, 1e-4
        out.append(c)
    return out


def test_batch_instances_follow_their_own_trajectories():
    cases = instances()
    steps, rtol = 4, 1e-12
    stream = torch.cuda.current_stream(DEV)
    inputs = []
    for c in cases:
        ctx = Context(0, stream)
        ctx.set_inputs(c)
        inputs.append(ctx)
    b = Batch(inputs, precision=EQS_PREC_FP64, stream=stream)
    xs = [torch.zeros(c.n_nodes, dtype=torch.float64, device=DEV) for c in cases]
    res = b.rkc_steps(steps, 0.0, cases[0].tau, cases[0].s, xs, rtol)
    print(f"[batch] per-instance CG iterations {res['iters'].tolist()} relres {res['relres'].max():.2e}", flush=True)
    assert (res["relres"] <= rtol * 1.01).all()
    assert len(set(res["iters"].tolist())) > 1  # instances converge independently
    for c, x in zip(cases, xs):
        o = EqsOracle(c)
        ref = o.rkc_trajectory(np.zeros(o.n_free), 0.0, c.tau, c.s, steps)
        got = x.cpu().numpy()
        err = np.linalg.norm(got[o.free] - ref[-1]) / max(np.linalg.norm(r) for r in ref)
        assert err <= 1e-9, err
        assert np.abs(got[o.dir_nodes] - o.g(steps * c.tau)).max() <= 1e-13
        # the same instance alone
        with Context(0, stream) as one:
            one.setup_case(c, precision=EQS_PREC_FP64)
            y = torch.zeros(c.n_nodes, dtype=torch.float64, device=DEV)
            for k in range(steps):
                one.rkc_step(k * c.tau, c.tau, c.s, y, rtol=rtol)
            alone = y.cpu().numpy()
        assert np.linalg.norm(got - alone) <= 1e-9 * np.linalg.norm(alone)
    b.close()
    for ctx in inputs:
        ctx.close()


def test_instance_validation():
    cases = instances()[:2]
    xyz = np.concatenate([c.xyz for c in cases])
    off = cases[0].n_nodes
    tets = np.concatenate([cases[0].tets, cases[1].tets + off])
    node_off = np.array([0, off, xyz.shape[0]])
    tet_off = np.array([0, cases[0].n_tets, tets.shape[0]])
    bad = tets.copy()
    bad[0, 0] = off + 3  # a tet of instance 0 reaching into instance 1
    with Context(0, torch.cuda.current_stream(DEV)) as ctx:
        ctx.set_mesh(xyz, bad)
        ctx.set_instances(node_off, tet_off)
        mats = np.concatenate([cases[0].tet_mat, cases[1].tet_mat + cases[0].n_mat])
        ctx.set_materials(np.concatenate([c.eps_r for c in cases]), np.concatenate([c.kappa0 for c in cases]),
                          np.concatenate([c.e_s for c in cases]), np.concatenate([c.alpha for c in cases]),
                          np.concatenate([c.nonlinear for c in cases]), mats)
        dn = np.concatenate([cases[0].dir_nodes, cases[1].dir_nodes + off])
        dd = np.concatenate([cases[0].dir_drive, cases[1].dir_drive + 2])
        ctx.set_dirichlet(dn, dd, np.concatenate([c.amp for c in cases]), np.concatenate([c.freq for c in cases]),
                          np.concatenate([c.phase for c in cases]))
        with pytest.raises(EqsError) as e:
            ctx.build_preconditioner()
        assert e.value.code == EQS_ERR_INVALID_ARG and "another instance" in str(e.value)


@pytest.mark.parametrize("reject", ["0", "1"])
def test_batch_of_more_instances_than_one_finaliser_workgroup(reject, monkeypatch):
    """20 instances: the CG finalisers run two workgroups (16 instances each)
    and a separate summary kernel. Every instance follows its own trajectory as
    in a batch of four; with EQS_TEST_REJECT_CHECK=1 every solve restarts once
    from its true residual (the summary kernel clears the one-shot flag after
    both workgroups have read it), with the same result."""
    monkeypatch.setenv("EQS_TEST_REJECT_CHECK", reject)
    cases = []
    for k in range(20):
        n, seed, amp, freq = SPECS[k % len(SPECS)]
        c = _inclusion_case("c3", 7 + k % 2, seed + k, (2.0, 15.0), (6.0, 14.0), amp=amp * (1 + 0.05 * k),
                            freq=freq)
        c.s, c.tau = 8, 1e-4
        cases.append(c)
    steps, rtol = 2, 1e-12
    stream = torch.cuda.current_stream(DEV)
    inputs = []
    for c in cases:
        ctx = Context(0, stream)
        ctx.set_inputs(c)
        inputs.append(ctx)
    b = Batch(inputs, precision=EQS_PREC_FP64, stream=stream)
    for ctx in inputs:
        ctx.close()
    xs = [torch.zeros(c.n_nodes, dtype=torch.float64, device=DEV) for c in cases]
    res = b.rkc_steps(steps, 0.0, cases[0].tau, cases[0].s, xs, rtol)
    b.close()
    print(f"[batch20] reject={reject} CG iterations {res['iters'].tolist()}", flush=True)
    assert (res["relres"] <= rtol * 1.01).all()
    for c, x in zip(cases, xs):
        o = EqsOracle(c)
        ref = o.rkc_trajectory(np.zeros(o.n_free), 0.0, c.tau, c.s, steps)
        err = np.linalg.norm(x.cpu().numpy()[o.free] - ref[-1]) / max(np.linalg.norm(r) for r in ref)
        assert err <= 1e-9, (c.n, err)
