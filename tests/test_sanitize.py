"""The host code of the library under AddressSanitizer and
UndefinedBehaviorSanitizer: build the host-instrumented library
(build.build(sanitize=True); device code unchanged) and run the CPU ABI
tests against it in a child process with the sanitizer runtime preloaded.
Any sanitizer report aborts the child (no recovery), failing this test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.timeout(900)
def test_abi_tests_pass_under_address_and_ub_sanitizers():
    sys.path.insert(0, ROOT)
    from paper_1501_04840_amd import build
    lib = build.build(sanitize=True)
    env = dict(os.environ)
    env["OT_DYN_LIB"] = lib
    env["LD_PRELOAD"] = build.asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "passed" in r.stdout
