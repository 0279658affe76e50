"""Build the oracle's C library (liborc.so) with gcc.

Test infrastructure: only the tests, the smoke check and the benchmark's
CPU-baseline leg load the result.  Plain IEEE FP64: no fast-math and no FMA
contraction, so the arithmetic is the one written in the C sources.  -O3 for
the x86-64-v3 instruction set (AVX2), which every host of the GPU nodes has;
the library is built on one machine and run on another, so not -march=native.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["bem_oracle.c", "nearfield.c"]
LIB = os.path.join(HERE, "liborc.so")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    cmd = ["gcc", "-O3", "-march=x86-64-v3", "-fPIC", "-shared", "-std=c11", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", LIB + ".tmp"] + srcs + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
