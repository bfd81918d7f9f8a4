import os
import shutil
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
TESTS = os.path.dirname(os.path.abspath(__file__))
if TESTS not in sys.path:
    sys.path.insert(0, TESTS)

# oracle reference trajectories running in child processes (see oracle_refs.py)
_PENDING = {}
_TMP = []


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")
    config.addinivalue_line("markers", "oracle_refs(*names): uses oracle reference trajectories (oracle_refs.REFS), "
                                       "started in the background when the test is selected")


def pytest_collection_finish(session):
    """Start the oracle reference runs that the selected tests need, so that
    they compute while the tests before them run."""
    import oracle_refs

    if session.config.option.collectonly:
        return
    names = []
    for item in session.items:
        for m in item.iter_markers("oracle_refs"):
            names += [n for n in m.args if n not in names]
    if not names:
        return
    d = tempfile.mkdtemp(prefix="eqs_oracle_refs_")
    _TMP.append(d)
    cpus = len(os.sched_getaffinity(0))
    box = os.environ.get("OMP_NUM_THREADS", "")
    total = int(box) if box.isdigit() and int(box) > 0 else cpus
    threads = max(1, min(cpus, total) // len(names))
    for n in names:
        _PENDING[n] = oracle_refs.Pending(n, d, threads)


def pytest_sessionfinish(session, exitstatus):
    for p in _PENDING.values():
        p.stop()
    for d in _TMP:
        shutil.rmtree(d, ignore_errors=True)


@pytest.fixture(scope="session")
def oracle_ref(pytestconfig):
    """oracle_ref(name) -> {"states", "free", ...} of a reference run, waiting
    for it (its progress lines are shown as they come)."""
    capman = pytestconfig.pluginmanager.getplugin("capturemanager")
    cache = {}

    def echo(line):
        with capman.global_and_fixture_disabled():
            print(line, flush=True)

    def get(name):
        if name not in cache:
            if name not in _PENDING:
                raise RuntimeError(f"oracle reference {name} was not started: mark the test oracle_refs({name!r})")
            cache[name] = _PENDING[name].wait(timeout=780, echo=echo)
        return cache[name]

    return get


@pytest.fixture(scope="session")
def golden_dir():
    return os.path.join(ROOT, "tests", "golden")
