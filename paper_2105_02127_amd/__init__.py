"""MI355X-native unstructured-mesh finite-volume TENO residual (2D Euler, FP64).

The compute path is `libteno.so`: host C++ set-up plus hand-written HIP kernels
for gfx950 behind a C ABI (`include/teno.h`).  `teno` is the thin ctypes
binding; `inputs` builds seeded synthetic meshes and initial states.
Importing the package loads nothing native; `teno.load()` does, and fails
loudly when the library has not been built.
"""
__all__ = ["inputs", "teno"]
