"""The per-step JSON-lines records (paper_1612_09447_amd.steplog) - CPU only:
a stand-in context returns the stats dict that Context.rkc_step returns."""

import json

from paper_1612_09447_amd.steplog import StepLog


class FakeCtx:
    def __init__(self):
        self.calls = []

    def rkc_step(self, t, dt, s, x, rtol, maxit=1000):
        self.calls.append((t, dt, s, rtol, maxit))
        return dict(stages=s, total_iters=7 * s + len(self.calls), max_iters=9, min_iters=6, not_converged=0,
                    guess_used=0, guess_fallbacks=0, max_relres=9.5e-9, train_loss=0.0, rc=0)


def test_one_record_per_step(tmp_path):
    path = tmp_path / "steps.jsonl"
    ctx = FakeCtx()
    with StepLog(path, run="c2 main", precision="fp32") as log:
        for n in range(3):
            st = log.step(ctx, n, n * 1e-4, 1e-4, 16, None, 1e-8, maxit=500)
            assert st["stages"] == 16
    recs = [json.loads(l) for l in path.read_text().splitlines()]
    assert [r["step"] for r in recs] == [0, 1, 2]
    assert ctx.calls[1] == (1e-4, 1e-4, 16, 1e-8, 500)
    r = recs[2]
    assert r["run"] == "c2 main" and r["precision"] == "fp32" and r["stages"] == 16
    assert r["cg_iters"] == 7 * 16 + 3 and r["cg_iters_per_stage"] == round((7 * 16 + 3) / 16, 3)
    assert r["max_relres"] == 9.5e-9 and r["wall_ms"] >= 0.0 and r["t"] == 2e-4
    # appends to an existing file
    with StepLog(path) as log:
        log.step(ctx, 3, 3e-4, 1e-4, 8, None, 1e-8)
    assert len(path.read_text().splitlines()) == 4


def test_each_stage_count_is_recorded(tmp_path):
    class StageCtx(FakeCtx):
        def rkc_step(self, t, dt, s, x, rtol, maxit=1000):
            st = super().rkc_step(t, dt, s, x, rtol, maxit)
            st["stage_iters"] = [6 + (k % 4) for k in range(s)]
            st["total_iters"] = sum(st["stage_iters"])
            return st

    path = tmp_path / "steps.jsonl"
    with StepLog(path, run="c0") as log:
        log.step(StageCtx(), 0, 0.0, 1e-4, 8, None, 1e-10)
        log.step(FakeCtx(), 1, 1e-4, 1e-4, 8, None, 1e-10)  # stats without per-stage counts
    with_counts, without = [json.loads(l) for l in path.read_text().splitlines()]
    assert with_counts["stage_iters"] == [6, 7, 8, 9, 6, 7, 8, 9]
    assert with_counts["cg_iters"] == sum(with_counts["stage_iters"])
    assert "stage_iters" not in without
