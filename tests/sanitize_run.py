"""Runs the sanitizer driver (tests/native/abi_sanitize.cpp, built by
paper_1612_09447_amd.build.build_sanitized with host-side AddressSanitizer and
UndefinedBehaviorSanitizer) and checks that it finished with no sanitizer
finding."""

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
SUPP = os.path.join(NATIVE, "lsan_runtime.supp")


def sources():
    from paper_1612_09447_amd import build as b

    return [os.path.join(b.CSRC, f) for f in os.listdir(b.CSRC)] + [
        b.SAN_DRIVER, os.path.join(b.INCLUDE, "eqs.h"), os.path.abspath(b.__file__)]


def stale():
    """The driver is missing or older than a source it is built from."""
    from paper_1612_09447_amd import build as b

    if not os.path.exists(b.SAN_EXE):
        return True
    t = os.path.getmtime(b.SAN_EXE)
    return any(os.path.getmtime(p) > t for p in sources())


def run(mode, timeout, extra_env=None):
    from paper_1612_09447_amd import build as b

    env = dict(os.environ)
    # a finding (or a failed libstdc++ assertion: handle_abort) ends the run
    # with a report and a stack; leaks are checked at exit, except
    # the runtimes' own allocations (suppressions); the shadow gap stays
    # mappable for the GPU runtime's address-space reservations
    env["ASAN_OPTIONS"] = "halt_on_error=1:abort_on_error=0:handle_abort=1:detect_leaks=1:protect_shadow_gap=0:exitcode=99"
    env["LSAN_OPTIONS"] = f"suppressions={SUPP}:print_suppressions=0:exitcode=98"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    for k in list(env):
        if k.startswith("EQS_"):
            del env[k]
    env.update(extra_env or {})
    r = subprocess.run([b.SAN_EXE, mode], capture_output=True, text=True, timeout=timeout, env=env)
    out = r.stdout + r.stderr
    print(out[-6000:], flush=True)
    assert "ERROR: AddressSanitizer" not in out and "ERROR: LeakSanitizer" not in out, "AddressSanitizer finding"
    assert "runtime error:" not in out, "UndefinedBehaviorSanitizer finding"
    assert r.returncode == 0, f"driver exit status {r.returncode}"
    assert f"SANITIZE OK {mode}" in r.stdout
    return out
