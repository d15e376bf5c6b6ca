"""AddressSanitizer + UndefinedBehaviorSanitizer runs of the host code (CPU
only): the library's set-up of triangle and tetrahedral meshes (csrc/setup.cpp,
csrc/setup3.cpp) and both oracles, on seeded periodic and open meshes, through
the drivers in tests/sanitize/.  Any report fails the run."""
from __future__ import annotations

import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2105_02127_amd import inputs, inputs3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2105_02127_amd", "csrc")
SAN = os.path.join(ROOT, "tests", "sanitize")
FLAGS = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp", "-pthread",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="1")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _build(tmp, name, sources):
    exe = os.path.join(tmp, name)
    subprocess.run(FLAGS + sources + ["-o", exe], check=True, capture_output=True)
    return exe


def _run(exe, tmp, tags):
    r = subprocess.run([exe, tmp, *tags], env=ENV, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    return r.stdout


def test_triangle_setup_and_oracle_under_sanitizers(tmp_path):
    tmp = str(tmp_path)
    meshes = {"per": (inputs.jittered_periodic_mesh(9, 3), (1.0, 1.0)),
              "box": (inputs.jittered_box_mesh(10, 7, 4), (0.0, 0.0))}
    for tag, (m, per) in meshes.items():
        U = inputs.random_lines(m)
        with open(os.path.join(tmp, tag + ".txt"), "w") as fh:
            fh.write(f"{m.xy.shape[0]} {m.tri.shape[0]} {per[0]} {per[1]}\n")
        np.ascontiguousarray(m.xy, np.float64).tofile(os.path.join(tmp, tag + ".xy"))
        np.ascontiguousarray(m.tri, np.int32).tofile(os.path.join(tmp, tag + ".tri"))
        np.ascontiguousarray(U, np.float64).tofile(os.path.join(tmp, tag + ".u"))
    exe = _build(tmp, "san2d", [os.path.join(SAN, "san2d.cpp"), os.path.join(CSRC, "setup.cpp")])
    out = _run(exe, tmp, list(meshes))
    assert out.count(" ok") == len(meshes)


def test_tetrahedral_setup_and_oracle_under_sanitizers(tmp_path):
    tmp = str(tmp_path)
    meshes = {"per": inputs3.jittered_periodic_cube(5, 3), "box": inputs3.jittered_box3(4, 3, 3, 4)}
    for tag, m in meshes.items():
        U = inputs3.random_planes3(m)
        with open(os.path.join(tmp, tag + ".txt"), "w") as fh:
            fh.write(f"{m.n_vert} {m.n_cell} {m.period[0]} {m.period[1]} {m.period[2]}\n")
        np.ascontiguousarray(m.xyz, np.float64).tofile(os.path.join(tmp, tag + ".xyz"))
        np.ascontiguousarray(m.tet, np.int32).tofile(os.path.join(tmp, tag + ".tet"))
        np.ascontiguousarray(U, np.float64).tofile(os.path.join(tmp, tag + ".u"))
    exe = _build(tmp, "san3d", [os.path.join(SAN, "san3d.cpp"), os.path.join(CSRC, "setup3.cpp"),
                                os.path.join(CSRC, "setup.cpp")])
    out = _run(exe, tmp, list(meshes))
    assert out.count(" ok") == len(meshes)
