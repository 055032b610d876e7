"""Compile the HIP library libtrevr2.so for gfx950 (in-tree).

Each source is compiled to an object in parallel (one hipcc per file), then
the objects are linked into one shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libtrevr2.so")
OBJ = os.path.join(ROOT, "_build")
SOURCES = ["api.hip", "tree_build.hip", "compute_j.hip", "compute_j_bwd.hip", "forest.hip"]


def _flags(arch: str):
    return [f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def hipcc_command(out: str = SO, arch: str = "gfx950"):
    """One-shot command (compile and link every source in one hipcc call)."""
    return ["hipcc"] + _flags(arch) + ["-shared", "-o", out] + \
           [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False, arch: str = "gfx950") -> str:
    os.makedirs(OBJ, exist_ok=True)
    objs = [os.path.join(OBJ, s.replace(".hip", ".o")) for s in SOURCES]

    def compile_one(i):
        cmd = ["hipcc"] + _flags(arch) + ["-c", os.path.join(CSRC, SOURCES[i]), "-o", objs[i]]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        return r.returncode, r.stdout, cmd

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        results = list(ex.map(compile_one, range(len(SOURCES))))
    for rc, out, cmd in results:
        lines = [ln for ln in out.splitlines() if "packed-fp32-ops" not in ln]
        if lines and (rc != 0 or verbose):
            print("\n".join(lines), file=sys.stderr)
        if rc != 0:
            raise subprocess.CalledProcessError(rc, cmd)
    tmp = SO + ".tmp"
    subprocess.check_call(["hipcc", f"--offload-arch={arch}", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(SO)
