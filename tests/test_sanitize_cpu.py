"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer,
on the CPU: the sanitizer driver's host mode runs the set-up algorithms that
need no GPU (mesh validation and ordering, assembly of M on the free nodes of
eq. (2), the smoothed-aggregation hierarchy, Sec. II's RKC coefficients) and
the C ABI's argument checks, and must end with no finding and no leak. The
driver is rebuilt first when a source is newer than it."""

import sanitize_run


def test_host_code_under_asan_and_ubsan():
    if sanitize_run.stale():
        from paper_1612_09447_amd import build as b

        b.build_sanitized(8)
    out = sanitize_run.run("host", timeout=120)
    assert "AMG levels" in out
