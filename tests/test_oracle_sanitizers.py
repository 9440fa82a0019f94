"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code, g++), driven through every entry point on small lattices that
cover its node classes and options (oracle/sanitize_driver.cpp): no sanitizer
report and finite results.  Marked slow: compiling takes about half a minute."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_runs_clean_under_address_and_undefined_behaviour_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_sanitized")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-fopenmp", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-o", exe,
               os.path.join(ROOT, "oracle", "lbm_oracle.cpp"), os.path.join(ROOT, "oracle", "sanitize_driver.cpp")]
        subprocess.run(cmd, check=True, capture_output=True, text=True, timeout=600)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
                   OMP_NUM_THREADS="2")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "0 failures" in r.stdout
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
