"""The FP64 oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

Host code only: ``tests/oracle_sanitize_main.cpp`` includes
``oracle/trevr_oracle.cpp`` as one translation unit and drives its C ABI
(every option flag, 1-10 bands, N_side 1-4, active subsets, the forward-mode
derivative, the complex source tables, the unit functions).  It is built with
g++ and statically linked sanitizer runtimes, so no library is preloaded; any
report (out-of-bounds access, use after free, signed overflow, misaligned or
null access, ...) ends the run with a nonzero status.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-static-libasan", "-static-libubsan",
           os.path.join(HERE, "oracle_sanitize_main.cpp"), "-o", exe]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    assert "unit functions: ok" in r.stdout
