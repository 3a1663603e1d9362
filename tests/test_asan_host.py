"""The library's host code under AddressSanitizer.

The sources that carry the host-side logic (argument checks, workspace layouts, the batched
planner and tuner, the stream scheduler) are rebuilt with the sanitizer on the host side only and
linked with the regular fused-kernel objects.  The host-only ABI tests (tests/test_abi.py: every
argument check, the workspace arithmetic, plan validation and its error paths) then run in a
child Python with the sanitizer's runtime preloaded; any report fails the test."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_library_under_asan(tmp_path):
    from paper_2303_14102_amd import build as b
    if not os.path.exists(os.path.join(b.HERE, "libsilhouette.so")):
        pytest.skip("library not built")
    try:
        rt = b.asan_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    lib = b.build_asan()
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, SIL_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0:exitcode=23")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_abi.py")]
    res = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = res.stdout + res.stderr
    print(out[-3000:])
    assert "AddressSanitizer" not in out
    assert res.returncode == 0
    assert " passed" in out
