"""The float64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only: plain gcc, no GPU code involved) and run on a C driver that
calls every oracle function at small sizes and at its edge cases (n = 1,
a failing pivot, NaN input, empty and tied argmax / top-k).  Any
out-of-bounds access, leak or undefined operation fails the test."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_address_and_undefined_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_driver")
        cmd = ["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
               "-ffp-contract=off", "-fopenmp",
               os.path.join(ROOT, "oracle", "gp_oracle.c"),
               os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"), "-o", exe, "-lm"]
        subprocess.check_call(cmd)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
        r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
