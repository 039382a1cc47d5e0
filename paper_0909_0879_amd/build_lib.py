"""Build libnbody.so (HIP, gfx950) in place with hipcc.

Device code is compiled without FMA contraction (every fused multiply-add
is written out explicitly) and with packed FP32 instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libnbody.so")
SOURCES = [os.path.join(CSRC, "nbody_kernels.hip"), os.path.join(CSRC, "nbody_api.cpp")]
ARCH = os.environ.get("NBODY_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
]


def build(verbose: bool = False, extra=()) -> str:
    tmp = OUT + ".tmp"
    cmd = ["hipcc", *FLAGS, *extra, "-x", "hip", SOURCES[0], "-x", "hip", SOURCES[1], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
