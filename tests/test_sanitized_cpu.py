"""The C ABI's error paths under the host address and undefined-behaviour
sanitizers, without a GPU: tests/c/abi_errors.c linked against the
sanitized build of the host translation units (made by __graft_entry__.build()).
Without a device only the host-side checks run (NULL handles, bad arguments,
the bin rule, the virial object's validation)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c", "build", "abi_errors_asan")


def test_error_paths_under_sanitizers_host_only():
    if not os.path.exists(EXE):
        pytest.skip("sanitized drivers not built (paper_2102_03691_amd._build.build_sanitized)")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", HIP_VISIBLE_DEVICES="",
               ROCR_VISIBLE_DEVICES="")
    r = subprocess.run([EXE], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "abi_errors: ok" in r.stdout
