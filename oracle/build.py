"""Compile the CPU oracle (test infrastructure) into ``oracle/liboracle.so``.

Plain gcc, OpenMP for independent points/queries only.  ``-ffp-contract=off``
keeps every multiply and add separate unless the source calls ``fmaf``; FMA
hardware makes those calls single fused instructions (correctly rounded, as
``fmaf`` is defined).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "taco_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-std=c11", "-O2", "-ftree-vectorize", "-mfma", "-mavx2", "-ffp-contract=off",
          "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
          "-Wno-unused-parameter"]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
