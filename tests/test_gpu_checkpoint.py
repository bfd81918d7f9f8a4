"""Checkpoint and resume (eqs_state_size / eqs_state_save / eqs_state_load).

A run of four RKC steps (Sec. II) is compared with a run stopped after two
steps, saved, loaded into a fresh context built the same way, and continued
for two: with the deterministic element pass and rule-based layouts (so that
separate contexts sum in the same order) the final potentials are equal bit
for bit, for the plain, the Galerkin (eq. (5)) and the network start vectors
(Sec. IV: the window, its reduced matrices, the replay buffer, the network's
weights and Adam moments all travel). Mismatched contexts and truncated
buffers are refused.
"""

import numpy as np
import pytest

import eqsgen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1612_09447_amd import EQS_ERR_INVALID_ARG, EQS_PREC_FP32, Context, EqsError  # noqa: E402

DEV = torch.device("cuda:0")


def make(case, guess):
    c = Context(0, torch.cuda.current_stream(DEV))
    c.setup_case(case, precision=EQS_PREC_FP32, deterministic=True)
    if guess == "mlp":
        c.set_guess("mlp", init=eqsgen.mlp_init(4), batch=64, warmup=8)
    elif guess != "previous":
        c.set_guess(guess)
    return c


def steps(c, case, x, n0, n):
    its = 0
    for k in range(n0, n0 + n):
        its += c.rkc_step(k * case.tau, case.tau, case.s, x, rtol=1e-10, maxit=500)["total_iters"]
    return its


@pytest.mark.parametrize("guess", ["previous", "galerkin", "mlp"])
def test_resumed_run_equals_uninterrupted_run(guess, monkeypatch):
    monkeypatch.setenv("EQS_AUTOTUNE", "0")
    case = eqsgen.case_c1(n=12, seed=5)
    case.s = 12
    with make(case, guess) as a:
        xa = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        its_a = steps(a, case, xa, 0, 4)
    with make(case, guess) as b:
        xb = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        its_b = steps(b, case, xb, 0, 2)
        blob = b.state_save()
    with make(case, guess) as c:
        c.state_load(blob)
        its_b += steps(c, case, xb, 2, 2)
    d = torch.linalg.vector_norm(xa - xb) / torch.linalg.vector_norm(xa)
    print(f"[ckpt] {guess}: checkpoint {len(blob)} bytes, CG iterations {its_a} / {its_b}, "
          f"rel. difference {float(d):.2e}", flush=True)
    assert its_a == its_b
    assert torch.equal(xa, xb)


def test_checkpoint_refused_by_other_contexts(monkeypatch):
    monkeypatch.setenv("EQS_AUTOTUNE", "0")
    case = eqsgen.case_c1(n=12, seed=5)
    with make(case, "galerkin") as b:
        x = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        steps(b, case, x, 0, 1)
        blob = b.state_save()
    for other, guess in [(case, "previous"), (eqsgen.case_c1(n=11, seed=5), "galerkin")]:
        with make(other, guess) as c:
            with pytest.raises(EqsError) as e:
                c.state_load(blob)
            assert e.value.code == EQS_ERR_INVALID_ARG
    with make(case, "galerkin") as c:
        for bad in (blob[:-8], blob + bytes(8), bytes(len(blob))):
            with pytest.raises(EqsError) as e:
                c.state_load(bad)
            assert e.value.code == EQS_ERR_INVALID_ARG
        c.state_load(blob)  # the intact checkpoint still loads
