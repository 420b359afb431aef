"""Build the HIP library libgks.so for gfx950 (hipcc, in-tree)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgks.so")
ROOT = os.path.dirname(HERE)

FLAGS = [
    "-O3", "-std=c++20", "-fPIC", "-shared", "--offload-arch=gfx950",
    # packed FP32 instructions stay off (wrong results seen with some forms)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]


def build(verbose=False, extra=()):
    src = os.path.join(CSRC, "gks_api.hip")
    cmd = ["hipcc", *FLAGS, *extra, "-I", os.path.join(ROOT, "include"), "-o", LIB + ".tmp", src]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=tuple(sys.argv[1:]))
