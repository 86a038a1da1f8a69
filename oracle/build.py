"""Build the CPU oracle (test infrastructure) as a shared library with gcc.

Plain IEEE double arithmetic: no FMA contraction, no fast-math, so every
operation in the oracle rounds exactly as written. OpenMP is linked for the
optional multi-threaded dominance and association loops (serial by default).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "nsga3_oracle.c")
LIB = os.path.join(HERE, "liboracle_nsga3.so")


def build(verbose=False):
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-Wall", "-Wextra", "-o", LIB, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
