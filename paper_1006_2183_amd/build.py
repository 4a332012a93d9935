"""Compile the HIP library for gfx950 (in-tree shared objects, loaded via ctypes).

Two builds of the same source: ``libsgspgemm.so`` (the library) and
``libsgspgemm_check.so`` (SG_CHECK=1: the same kernels plus invariant
counters, read with sg_plan_check, for the test suite). They compile in
parallel.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "sg_spgemm.hip")
LIB = os.path.join(HERE, "libsgspgemm.so")
CHECK_LIB = os.path.join(HERE, "libsgspgemm_check.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # packed FP32 instructions stay off: hipcc would otherwise form them from scalar code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, check: bool = True) -> str:
    jobs = [(LIB, [])]
    if check:
        jobs.append((CHECK_LIB, ["-DSG_CHECK=1"]))
    procs = []
    for out, extra in jobs:
        tmp = out + ".tmp"
        cmd = [HIPCC] + FLAGS + extra + ["-o", tmp, SRC]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((out, tmp, subprocess.Popen(cmd)))
    for out, tmp, p in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, f"hipcc {out}")
        os.replace(tmp, out)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, check="--no-check" not in sys.argv)
    print(LIB)
