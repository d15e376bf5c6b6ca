"""Build the CPU oracle shared library (test infrastructure only)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "teno_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

# No FMA contraction and no fast-math: the oracle evaluates every expression
# as written, in IEEE double precision (so -O3 changes its speed, never its
# results).  No -march=native: the library built on one host is loaded on
# another, whose CPU may lack the build host's instruction set.
CMD = ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
       "-ffp-contract=off", "-fno-fast-math", "-Wall", "-o", LIB, SRC]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = CMD[:-3] + ["-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
