"""The oracle's pins run again on an AddressSanitizer + UndefinedBehavior
Sanitizer build of oracle.c (host code only; any report aborts the run), so
that an out-of-bounds access or undefined arithmetic in the checker cannot
hide behind values that happen to pass."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_pins_clean_under_sanitizers():
    import oracle
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("libasan not available")
    oracle.build(force=True, sanitize=True)
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", ORACLE_SANITIZE="1")
    files = [os.path.join(ROOT, "tests", f) for f in ("test_oracle_pins.py", "test_oracle_mts.py",
                                                        "test_oracle_chrono.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *files], env=env,
                       capture_output=True, text=True, timeout=900, cwd=ROOT)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
