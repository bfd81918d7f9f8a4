"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
with the GPU: the sanitizer driver's abi mode calls every C ABI entry point on
device 0 (first- and second-order meshes, both hierarchy precisions, steps
with every start-vector kind of Sec. IV, adaptive steps, checkpoints, the
caller's workspace, instances, batches, the network, kernel timing and the
error paths) and must end with no finding and no leak of the library's own
memory. It runs once with the defaults and once per group of the library's
switches, so that their set-up paths run sanitized too: plain launches with
rule-based layouts, 32-bit column ids and the unfolded V-cycle; forced SELL
layouts with sorted rows, the per-block LDS stride and the restart path; CSR
for every coarse operator; and a tuning record written, then replayed. The
driver is built beforehand on the CPU with the library."""

import pytest

import sanitize_run

pytestmark = pytest.mark.gpu

VARIANTS = {
    "defaults": {},
    "plain-launches-rule-layouts-unfolded": {"EQS_USE_GRAPHS": "0", "EQS_AUTOTUNE": "0", "EQS_INDEX16": "0",
                                             "EQS_FOLD": "0"},
    "sell4-sorted-generic-stride-restarts": {"EQS_LAYOUT": "sell4s", "EQS_UNROLL": "16", "EQS_KX_GENERIC": "1",
                                             "EQS_TEST_REJECT_CHECK": "1", "EQS_TUNE_LOG": "all"},
    "csr-coarse-operators": {"EQS_LAYOUT": "csr"},
}


@pytest.mark.parametrize("name", list(VARIANTS))
def test_c_abi_end_to_end_under_asan_and_ubsan(name):
    assert not sanitize_run.stale(), "build the sanitizer driver first (paper_1612_09447_amd.build.build_sanitized)"
    print(f"[sanitize] switches: {VARIANTS[name] or 'none'}", flush=True)
    sanitize_run.run("abi", timeout=110, extra_env=VARIANTS[name])


def test_tuning_record_written_then_replayed_under_asan_and_ubsan(tmp_path):
    assert not sanitize_run.stale(), "build the sanitizer driver first (paper_1612_09447_amd.build.build_sanitized)"
    rec = tmp_path / "tune.txt"
    sanitize_run.run("abi", timeout=110, extra_env={"EQS_TUNE_FILE": str(rec)})
    assert rec.stat().st_size > 0
    sanitize_run.run("abi", timeout=110, extra_env={"EQS_TUNE_FILE": str(rec)})
