"""Build libcmcg.so (all HIP sources, gfx950) in-tree with hipcc.

Each source is compiled to an object file in parallel (they share no device code), then the
objects are linked into the shared library."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcmcg.so")
OBJ = os.path.join(HERE, "_build")
# (source, object, extra flags): f1_kernels.hip builds as two objects, one per precision of its
# stream-kernel instances
UNITS = [
    ("f1_kernels.hip", "f1_kernels_fp32.o", ["-DCMCG_F1_PART=1"]),
    ("f1_kernels.hip", "f1_kernels_fp64.o", ["-DCMCG_F1_PART=2"]),
    ("cmcg_api.hip", "cmcg_api.o", []),
    ("f1_solver.hip", "f1_solver.o", []),
    ("f2_kernels.hip", "f2_kernels.o", []),
    ("riesz_mg.hip", "riesz_mg.o", []),
    ("f2_solver.hip", "f2_solver.o", []),
    ("static_apply.hip", "static_apply.o", []),
    ("f1_serve.hip", "f1_serve.o", []),
]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # every multiply-add the kernels want is written as fma(); nothing else is contracted, so
    # a cell's arithmetic does not depend on how a kernel variant was unrolled
    "-ffp-contract=off",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def _jobs() -> int:
    try:
        return max(1, min(16, int(os.environ.get("MAX_JOBS", "0")) or os.cpu_count() or 1))
    except ValueError:
        return max(1, min(16, os.cpu_count() or 1))


def build(verbose: bool = True) -> str:
    os.makedirs(OBJ, exist_ok=True)

    def compile_one(unit) -> str:
        src, obj, extra = unit
        obj = os.path.join(OBJ, obj)
        cmd = [hipcc()] + FLAGS + extra + ["-c", "-o", obj, os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    with ThreadPoolExecutor(max_workers=_jobs()) as ex:
        objs = list(ex.map(compile_one, UNITS))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
