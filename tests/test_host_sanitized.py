"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU): code
creation over well-formed codes of extreme shape (rows of degree 32 and 64, a VN of degree 63 and
64, 4-cycles everywhere, n = 4194304) and over malformed matrices, QC bases and layer partitions,
and the entry points' argument checks.  The cases run in a child process with the sanitizer
runtime preloaded; a sanitizer report fails it."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_host_code_under_sanitizers():
    sys.path.insert(0, ROOT)
    from paper_2102_11089_amd import build as B
    lib = B.build_sanitized()
    env = dict(os.environ)
    env["LD_PRELOAD"] = B.asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "sanitized_host_cases.py"), lib], env=env,
                       capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "ERROR: AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert "sanitized host cases done" in r.stdout
