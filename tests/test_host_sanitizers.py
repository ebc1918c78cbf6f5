"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer:
a host-only sanitized build (paper_2603_19600_amd/sanitize.py, no device code)
and a C++ driver that drives the C ABI through its argument validation, which
returns before any device work, so it runs without a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="no hipcc")
def test_abi_validation_is_clean_under_asan_and_ubsan():
    from paper_2603_19600_amd import sanitize

    exe = sanitize.build()
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["HIP_VISIBLE_DEVICES"] = ""
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out
    assert r.returncode == 0, out
    assert "0 failures" in r.stdout, out
