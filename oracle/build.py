"""Compile the FP64 oracle (test infrastructure) into oracle/liboracle.so.

Run as a script or call build(). Plain gcc; OpenMP over queries."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sbh_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    # -fno-tree-slp-vectorize: gcc 11's basic-block vectorizer at -O3 drops the float32 rounding of
    # (double)(float)x in straight-line code (observed on the root's decoded centre of mass); the
    # oracle relies on such roundings being done
    cmd = ["gcc", "-O3", "-fno-tree-slp-vectorize", "-std=c99", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-shared", "-fPIC", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
