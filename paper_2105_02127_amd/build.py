"""Build libteno.so in-tree: host set-up (g++) + HIP kernels and C ABI for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(os.path.dirname(HERE), "_build")
LIB = os.path.join(HERE, "libteno.so")
ARCH = os.environ.get("TENO_OFFLOAD_ARCH", "gfx950")

HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-pthread", "-ffp-contract=off", "-fno-fast-math",
              "-Wall", "-Wextra", "-Wno-unused-parameter"]
# Packed FP32 instructions are disabled; FP64 kernels may contract to FMA.
# Code object v5 loads on both the system HIP runtime and the one bundled with
# the PyTorch wheel.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-parameter", "-Wno-unused-result"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False, resource_usage: bool = False, lib: str = LIB,
          extra_hip_flags=None) -> str:
    """Compile libteno.so.  extra_hip_flags (or TENO_HIPCC_EXTRA, space
    separated) are appended to the HIP compile line."""
    os.makedirs(BUILD, exist_ok=True)
    extra_hip = list(extra_hip_flags or []) + os.environ.get("TENO_HIPCC_EXTRA", "").split()
    # layout macros must reach both the host set-up and the kernels
    layout = [f for f in extra_hip if f.startswith(("-DTENO_TILE", "-DTENO_DENSE", "-DTENO_LARGE"))]
    setup_o = os.path.join(BUILD, "setup.o")
    setup3_o = os.path.join(BUILD, "setup3.o")
    api_o = os.path.join(BUILD, "teno_api.o")
    api3_o = os.path.join(BUILD, "teno3_api.o")
    _run(["g++", *HOST_FLAGS, *layout, "-c", os.path.join(CSRC, "setup.cpp"), "-o", setup_o],
         verbose)
    _run(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, "setup3.cpp"), "-o", setup3_o], verbose)
    extra = ["-Rpass-analysis=kernel-resource-usage"] if resource_usage else []
    _run(["hipcc", *HIP_FLAGS, *extra_hip, *extra, "-c", os.path.join(CSRC, "teno_api.hip"), "-o",
          api_o], verbose)
    # the tetrahedral path: a translation unit of its own
    _run(["hipcc", *HIP_FLAGS, *extra_hip, *extra, "-c", os.path.join(CSRC, "teno3_api.hip"), "-o",
          api3_o], verbose)
    tmp = lib + ".tmp"
    _run(["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-mcode-object-version=5",
          setup_o, setup3_o, api_o, api3_o, "-pthread",
          "-o", tmp], verbose)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose=True, resource_usage="--usage" in sys.argv))
