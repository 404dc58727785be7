"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer:
tests/test_abi.py (validation, plans, batches, groups, schedules, the tune
cache parser) run against a library whose host objects are instrumented.  Any
out-of-bounds access, use after free or undefined behaviour aborts the run."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_abi_suite_is_clean_under_asan_and_ubsan():
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import sanitize_host
    sanitize_host.build()
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=sanitize_host.env(), capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, tail
