"""Build the CPU oracle shared library (test infrastructure) with gcc.

The oracle is compiled without fast-math, FMA contraction or
architecture-specific tuning so that its floating-point conversion is the
plain IEEE round-to-nearest product it is written as.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nn_oracle.c")
LIB = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = [
        "gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp",
        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
        "-o", tmp, SRC,
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
