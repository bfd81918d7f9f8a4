"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
with the GPU: the sanitizer driver's abi mode calls every C ABI entry point on
device 0 (first- and second-order meshes, both hierarchy precisions, steps
with every start-vector kind of Sec. IV, adaptive steps, checkpoints, the
caller's workspace, instances, batches, the network, kernel timing and the
error paths) and must end with no finding and no leak of the library's own
memory. The driver is built beforehand on the CPU with the library."""

import pytest

import sanitize_run

pytestmark = pytest.mark.gpu


def test_c_abi_end_to_end_under_asan_and_ubsan():
    assert not sanitize_run.stale(), "build the sanitizer driver first (paper_1612_09447_amd.build.build_sanitized)"
    sanitize_run.run("abi", timeout=110)
