"""Build libvanse.so for gfx950 with hipcc (in-tree).

Five translation units compiled in parallel and linked into one shared
library: ``csrc/vanse.hip`` (the C ABI, set-up and read-out kernels) and
``csrc/step_{f64,f32,f32s,f16s}.hip`` (the step-kernel instances of each
storage precision, from ``csrc/step_inst.hpp``).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libvanse.so")
OBJ_DIR = os.path.join(HERE, "_build")
SOURCES = [os.path.join(HERE, "csrc", f) for f in
           ("step_f32.hip", "step_f64.hip", "step_f32s.hip", "step_f16s.hip", "vanse.hip")]
INCLUDE = [os.path.join(ROOT, "include"), os.path.join(HERE, "csrc")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # fuse a multiply and an add into an FMA only within one expression:
    # the same source then rounds the same way in every unrolled copy of a
    # sweep loop, so a node's result does not depend on its tile
    "-ffp-contract=on",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def _jobs() -> int:
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    return max(1, min(len(SOURCES), n, int(os.environ.get("MAX_JOBS", "16"))))


def build(verbose: bool = False) -> str:
    """Compile every source and link paper_2409_02964_amd/libvanse.so (always)."""
    os.makedirs(OBJ_DIR, exist_ok=True)
    inc = [f"-I{d}" for d in INCLUDE]

    def compile_one(src):
        obj = os.path.join(OBJ_DIR, os.path.basename(src).replace(".hip", ".o"))
        cmd = [hipcc(), *HIPCC_FLAGS, *inc, "-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.check_call(cmd)
        return obj

    with ThreadPoolExecutor(_jobs()) as pool:
        objs = list(pool.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
