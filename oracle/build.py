"""Build the C oracle (test infrastructure) into oracle/libref_plbm.so.

Plain gcc, FP64 semantics kept strict: no fast-math, no FMA contraction.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ref_plbm.c")
LIB = os.path.join(HERE, "libref_plbm.so")

CFLAGS = ["-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
          "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC"]


def build(verbose=False):
    cmd = ["gcc", *CFLAGS, SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
