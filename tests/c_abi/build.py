"""Build the plain C user of the library (tests/c_abi/sine_c) with gcc
against include/gks.h and the in-tree libgks.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
EXE = os.path.join(HERE, "sine_c")


def build(verbose=False):
    libdir = os.path.join(ROOT, "paper_1901_00261_amd")
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-I", os.path.join(ROOT, "include"), "-o", EXE,
           os.path.join(HERE, "sine_c.c"), "-L", libdir, "-l:libgks.so", "-Wl,-rpath,$ORIGIN/../../paper_1901_00261_amd", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return EXE


if __name__ == "__main__":
    build(verbose=True)
