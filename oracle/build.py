"""Build the CPU oracle library (plain C, gcc) in place: oracle/liboracle.so.

The oracle is test infrastructure; building it is part of the project build
so that the tests and the benchmark's CPU baseline can load it.  Flags: no
fast-math, no FMA contraction, generic x86-64 (the library may run on a
different host than the one that built it), OpenMP over i.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nbody_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
          "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
          "-Wno-unused-parameter"]


def build(verbose: bool = False, src: str = SRC, out: str = OUT) -> str:
    """Compile src (default: the oracle) into the shared library out."""
    tmp = out + ".tmp"
    cmd = ["gcc", *CFLAGS, src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
