"""Per-step records of a run as JSON lines.

``StepLog`` appends one JSON object per RKC step: the step index and time,
the stage count, the CG iterations of the step (total, mean per stage, extremes, and each
stage's count),
the largest final relative residual, the start-vector counters and the host
wall time of the call (``eqs_rkc_step`` returns after the step's work has
finished, so the wall time is the step's). It only formats what the library
returns; it does no arithmetic of the method.
"""

from __future__ import annotations

import json
import time


class StepLog:
    def __init__(self, path, run: str = "", **fields):
        self._f = open(path, "a", buffering=1)
        self._run = run
        self._fields = fields

    def step(self, ctx, n, t, dt, s, x, rtol, maxit=1000, **kw):
        """ctx.rkc_step(t, dt, s, x, rtol, maxit) with one record written; returns its stats."""
        t0 = time.perf_counter()
        st = ctx.rkc_step(t, dt, s, x, rtol, maxit=maxit, **kw)
        wall = time.perf_counter() - t0
        self.write(n, t, dt, st, wall)
        return st

    def write(self, n, t, dt, st, wall_s):
        rec = {"run": self._run, "step": int(n), "t": float(t), "dt": float(dt), "stages": st["stages"],
               "cg_iters": st["total_iters"], "cg_iters_per_stage": round(st["total_iters"] / max(1, st["stages"]), 3),
               "max_iters": st["max_iters"], "min_iters": st["min_iters"], "max_relres": st["max_relres"],
               "not_converged": st["not_converged"], "guess_used": st["guess_used"],
               "guess_fallbacks": st["guess_fallbacks"], "wall_ms": round(wall_s * 1e3, 3), **self._fields}
        if st.get("stage_iters") is not None:
            rec["stage_iters"] = list(st["stage_iters"])
        self._f.write(json.dumps(rec) + "\n")

    def close(self):
        if self._f:
            self._f.close()
            self._f = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
