"""Reference RKC trajectories from the FP64 CPU oracle, computed in a child
process while the other tests run.

The oracle integrates eq. (2) with RKC (Sec. II, its ref. [9]) from
phi(0) = 0 at t = 0 and every M-solve to rel-res 1e-13 (Jacobi-preconditioned
CG on OpenMP threads, each stage solve started from the previous stage's
solution). Only ``oracle/`` and the input generator ``eqsgen`` are used.

Run as a script: ``python tests/oracle_refs.py <case> <steps> <rtol> <out.npz>``;
writes the step-end states over the free nodes (``states[n]`` = x_n, n = 0..
steps) and prints one progress line per step. ``start(...)`` launches such a
run in the background and ``load(...)`` waits for it.
"""

from __future__ import annotations

import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
# progress logs of the reference runs (EQS_TEST_LOG_DIR, else a folder under the ignored build directory)
LOG_DIR = os.environ.get("EQS_TEST_LOG_DIR") or os.path.join(ROOT, "_build", "test_logs", "oracle_refs")

# reference runs a test may ask for: name -> (case, steps, stage-solve rel-res).
# The 1e-13 runs are the method's result; the 1e-8 runs are the oracle at the
# workloads' own tolerance, the floor of what any solver at that tolerance
# reaches.
REFS = {"c1_10": ("c1", 10, 1e-13), "c1_10_rtol8": ("c1", 10, 1e-8), "c2_1": ("c2", 1, 1e-13),
        "c2_1_rtol8": ("c2", 1, 1e-8)}


def compute(case_name: str, steps: int, out: str, rtol: float = 1e-13, threads=None) -> None:
    import numpy as np

    sys.path.insert(0, ROOT)
    import eqsgen
    from oracle.eqs import EqsOracle

    t0 = time.time()
    case = eqsgen.make_case(case_name)
    o = EqsOracle(case, solve_rtol=rtol, solver="jacobi", warm=True, threads=threads)
    print(f"[oracle_refs] {case_name} rel-res {rtol:g}: {o.n_free} free DOF, set-up {time.time() - t0:.1f}s",
          flush=True)
    iters = []

    def cb(n, t, Y):
        iters.append(o.last_iters)
        print(f"[oracle_refs] {case_name}: step {n + 1}/{steps} done at {time.time() - t0:.1f}s "
              f"(last solve {o.last_iters} CG iterations)", flush=True)

    states = o.rkc_trajectory(np.zeros(o.n_free), 0.0, case.tau, case.s, steps, callback=cb)
    tmp = out + ".tmp.npz"
    np.savez(tmp, states=np.stack(states), free=o.free, tau=case.tau, s=case.s, steps=steps,
             max_rate=o.max_rate)
    os.replace(tmp, out)
    print(f"[oracle_refs] {case_name}: wrote {out} after {time.time() - t0:.1f}s", flush=True)


class Pending:
    """A reference run in a child process."""

    def __init__(self, name: str, out_dir: str, threads: int):
        case, steps, rtol = REFS[name]
        self.name = name
        self.out = os.path.join(out_dir, f"{name}.npz")
        os.makedirs(LOG_DIR, exist_ok=True)
        self.log_path = os.path.join(LOG_DIR, f"{name}.log")
        self._log = open(self.log_path, "w")
        env = dict(os.environ, OMP_NUM_THREADS=str(threads))
        self.proc = subprocess.Popen([sys.executable, os.path.abspath(__file__), case, str(steps), repr(rtol), self.out],
                                     stdout=self._log, stderr=subprocess.STDOUT, env=env, cwd=ROOT)

    def wait(self, timeout: float, echo=print):
        """Block until the run ends, passing its progress lines to ``echo`` as
        they come; returns the loaded arrays."""
        import numpy as np

        t_end = time.time() + timeout
        seen = 0
        while True:
            rc = self.proc.poll()
            with open(self.log_path) as f:
                lines = f.read().splitlines()
            for ln in lines[seen:]:
                echo(ln)
            seen = len(lines)
            if rc is not None:
                break
            if time.time() > t_end:
                self.stop()
                raise TimeoutError(f"oracle reference {self.name} did not finish within {timeout:.0f}s")
            time.sleep(2.0)
        if rc != 0:
            raise RuntimeError(f"oracle reference {self.name} failed (exit {rc}); log {self.log_path}")
        with np.load(self.out) as z:
            return {k: z[k] for k in z.files}

    def stop(self):
        if self.proc.poll() is None:
            self.proc.kill()
            self.proc.wait()
        self._log.close()


if __name__ == "__main__":
    compute(sys.argv[1], int(sys.argv[2]), sys.argv[4], float(sys.argv[3]))
