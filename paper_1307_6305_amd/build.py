"""Build the HIP library ``libamg.so`` in-tree for gfx950.

Every HIP source is compiled with hipcc for ``--offload-arch=gfx950`` with
packed FP32 instructions disabled.  Floating-point contraction is off in the
setup unit, so that matching keys and coarse sums are correctly rounded
binary64 operations.  Host-only C++ goes through g++.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libamg.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC]
HIP_FLAGS = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
SOURCES = [
    ("validate.cpp", "g++", []),
    ("api.hip", "hipcc", []),
    ("setup.hip", "hipcc", ["-ffp-contract=off"]),
    ("solve.hip", "hipcc", []),
    ("batch.hip", "hipcc", []),
    ("serve.hip", "hipcc", []),
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link ``libamg.so``; returns its path."""
    os.makedirs(OBJ, exist_ok=True)
    objs, cmds = [], []
    for src, tool, extra in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(OBJ, src + ".o")
        if tool == "g++":
            cmd = ["g++"] + COMMON + extra + ["-c", path, "-o", obj]
        else:
            cmd = [HIPCC] + HIP_FLAGS + COMMON + extra + ["-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        cmds.append(cmd)
        objs.append(obj)
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", "6"))))
    with ThreadPoolExecutor(jobs) as ex:
        for f in [ex.submit(_run, c) for c in cmds]:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    _run(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
