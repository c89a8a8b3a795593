"""Builds the C oracle (SU(2) and 2-D Ising) into oracle/libsu2_oracle.so with the host compiler.

Test infrastructure only (see oracle/__init__.py).  The flags keep each FP32
and FP64 operation a separately rounded IEEE operation (no contraction into
fused multiply-adds, no fast-math), so the oracle's arithmetic is what its
source says.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRCS = [os.path.join(HERE, "su2_oracle.c"), os.path.join(HERE, "ising_oracle.c")]
LIB = os.path.join(HERE, "libsu2_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           *SRCS, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
