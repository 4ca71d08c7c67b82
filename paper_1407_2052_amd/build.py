"""Build the native library libamrvac.so (gfx950) in-tree.

    python -m paper_1407_2052_amd.build

Compiles the HIP kernels and the host runtime behind include/amrvac.h with
hipcc for gfx950.  All HIP code is compiled with packed-FP32 instructions
disabled and without automatic FMA contraction (the kernels write their
fused multiply-adds explicitly, which makes results independent of how the
compiler schedules each template instantiation).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libamrvac.so")
SOURCES = ["kernels.hip", "adjoint.hip", "runtime.cpp", "adjoint.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("AMRVAC_ARCH", "gfx950")


def build(verbose: bool = False) -> str:
    objs = []
    common = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-ffp-contract=off",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall", "-Wno-unused-function"]
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    # the four translation units compile side by side (kernels.hip dominates)
    procs = []
    for src in SOURCES:
        obj = os.path.join(bdir, src + ".o")
        cmd = [HIPCC, "-c", *common, "-x", "hip", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    failed = [cmd for cmd, p in procs if p.wait() != 0]
    if failed:
        raise subprocess.CalledProcessError(1, failed[0])
    cmd = [HIPCC, "-shared", f"--offload-arch={ARCH}", *objs, "-o", OUT + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
