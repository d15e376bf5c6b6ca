"""Build the CPU oracle shared libraries (test infrastructure only):
liboracle.so (triangles, teno_oracle.cpp) and liboracle3.so (tetrahedra,
teno3_oracle.cpp)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "teno_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")
SRC3 = os.path.join(HERE, "teno3_oracle.cpp")
LIB3 = os.path.join(HERE, "liboracle3.so")

# No FMA contraction and no fast-math: the oracle evaluates every expression
# as written, in IEEE double precision (so -O3 changes its speed, never its
# results).  No -march=native: the library built on one host is loaded on
# another, whose CPU may lack the build host's instruction set.
CMD = ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
       "-ffp-contract=off", "-fno-fast-math", "-Wall", "-o", LIB, SRC]


def _build_one(src: str, lib: str, verbose: bool) -> str:
    tmp = lib + ".tmp"
    cmd = CMD[:-3] + ["-o", tmp, src]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    _build_one(SRC3, LIB3, verbose)
    return _build_one(SRC, LIB, verbose)


def build3(verbose: bool = False) -> str:
    return _build_one(SRC3, LIB3, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
