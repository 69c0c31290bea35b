"""Build ``libltl.so`` (HIP for gfx950) in-tree with hipcc.

Usage: ``python -m paper_2406_17284_amd.build``. The shared library lands next to this
file and is what :mod:`paper_2406_17284_amd.ltl` loads.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libltl.so")
ARCH = "gfx950"

SOURCES = ["cat_kernel.hip", "flow_kernel.hip", "direct_kernel.hip", "batch_kernel.hip", "ltl_api.cpp", "batch_api.cpp", "tuning_cache.cpp"]

# hipcc flags: gfx950 only; packed FP32 instructions disabled in device code.
HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    objs, procs = [], []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for src in SOURCES:   # the translation units compile in parallel
        path = os.path.join(CSRC, src)
        obj = os.path.join(HERE, "_build", src + ".o")
        cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for cmd, pr in procs:
        if pr.wait() != 0:
            raise subprocess.CalledProcessError(pr.returncode, cmd)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
