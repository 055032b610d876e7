"""The C ABI's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

The library is compiled again with the sanitizers on its host code only
(each ``-fsanitize=`` behind ``-Xarch_host``; device code unchanged) and
linked without them; ``tests/abi_sanitize_main.cpp``, built with clang and
the sanitizer runtimes, drives every path that runs without a GPU (sizing
for all options, band counts and N_side values, forest sizing, argument and
handle validation, status strings).  Any report ends the run with a nonzero
status.  Kernels and HIP calls are not covered (they need a GPU; the GPU
tests and the HIP runtime's own checks cover those).
"""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CLANG = "/opt/rocm/llvm/bin/clang++"


@pytest.mark.skipif(shutil.which("hipcc") is None or not os.path.exists(CLANG),
                    reason="hipcc / clang++ not available")
def test_c_abi_host_code_under_asan_and_ubsan(tmp_path):
    sys.path.insert(0, os.path.join(ROOT, "paper_2310_15235_amd"))
    import build
    san = []
    for f in ("-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all",
              "-fno-omit-frame-pointer"):
        san += ["-Xarch_host", f]
    objs, procs = [], []
    for src in build.SOURCES:
        o = str(tmp_path / (src + ".o"))
        objs.append(o)
        procs.append(subprocess.Popen(
            ["hipcc"] + build._flags("gfx950") + san +
            ["-c", os.path.join(ROOT, "paper_2310_15235_amd", "csrc", src), "-o", o],
            stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL))
    assert all(p.wait() == 0 for p in procs)
    lib = str(tmp_path / "libtrevr2_san.so")
    subprocess.check_call(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", lib] + objs)
    exe = str(tmp_path / "abi_sanitize")
    subprocess.check_call([CLANG, "-std=c++17", "-g", "-O1", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                           os.path.join(HERE, "abi_sanitize_main.cpp"), "-L", str(tmp_path),
                           "-ltrevr2_san", "-Wl,-rpath," + str(tmp_path), "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-4000:]
    assert "C ABI host paths: ok" in r.stdout
