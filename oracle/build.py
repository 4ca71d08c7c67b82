"""Build the CPU oracle shared library (test infrastructure only).

    python oracle/build.py

Compiles amrvac_oracle.cpp with g++ -O2 -ffp-contract=off (no FMA
contraction, no fast-math) and OpenMP over blocks into oracle/liborc.so.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "amrvac_oracle.cpp")
OUT = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unused-function", SRC, "-o", OUT + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    build(verbose="-q" not in sys.argv)
