"""Host-side checks of libteno (no GPU): exported ABI, set-up parity with the
oracle (stencil lists exactly, least-squares operators to round-off), error
paths of mesh creation and set-up."""
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2105_02127_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def teno():
    from paper_2105_02127_amd import teno as t
    t.load()
    return t


def declared_functions():
    src = open(os.path.join(ROOT, "include", "teno.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(teno_\w+)\s*\(", src, flags=re.M)))


def test_every_declared_symbol_is_exported(teno):
    names = declared_functions()
    assert len(names) >= 20
    lib = teno.load()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(teno.SIGNATURES), set(names) ^ set(teno.SIGNATURES)


def _c_layout(struct, fields, tmp_path):
    """sizeof and field offsets of a struct of include/teno.h, from a C compiler."""
    src = tmp_path / f"{struct}.c"
    body = "".join(f'  printf("%zu\\n", offsetof({struct}, {f}));\n' for f in fields)
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "teno.h"\n'
                   f'int main(void) {{\n  printf("%zu\\n", sizeof({struct}));\n{body}  return 0;\n}}\n')
    exe = tmp_path / struct
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


@pytest.mark.parametrize("struct,cls", [("teno_params", "Params"), ("teno_info", "Info"),
                                        ("teno_diag", "Diag"), ("teno_batch_tuning", "BatchTuning")])
def test_struct_layouts_match_header(teno, tmp_path, struct, cls):
    import ctypes as C
    py = getattr(teno, cls)
    fields = [f for f, _ in py._fields_]
    size, offsets = _c_layout(struct, fields, tmp_path)
    assert C.sizeof(py) == size
    assert [getattr(py, f).offset for f in fields] == offsets


def test_default_params(teno):
    p = teno.default_params()
    assert (p.order, p.power, p.ct, p.eps, p.gamma, p.fallback, p.reorder, p.dk_prime) == \
        (5, 6, 1e-6, 1e-12, 1.4, 0, 1, 1e4)
    c = teno.default_params(variant=2)                  # the paper's CWENO values
    assert (c.power, c.eps, c.dk_prime) == (4, 1e-14, 1e4)


@pytest.mark.parametrize("n,order,seed", [(12, 3, 1), (12, 4, 2), (14, 5, 3), (16, 6, 4)])
def test_setup_parity_with_oracle(teno, oracle_mod, n, order, seed):
    m = inputs.jittered_periodic_mesh(n, seed)
    lm = teno.Mesh(m.xy, m.tri).setup(order=order)
    om = oracle_mod.OracleMesh(m.xy, m.tri)
    om.setup(oracle_mod.params(order=order), all_cells=False)
    info = lm.info()
    assert info.n_cell == om.n_cell and info.n_face == om.n_face
    assert info.rows_large == 2 * (order * (order + 1) // 2) - 1
    worst = 0.0
    for i in range(0, om.n_cell, 3):
        for k in range(4):
            np.testing.assert_array_equal(lm.stencil(i, k), om.stencil(i, k))
            Ml = lm.lsq_operator(i, k)
            Mo, _ = om.lsq_operator(i, k)
            worst = max(worst, np.abs(Ml - Mo).max() / np.abs(Mo).max())
    assert worst < 1e-11, worst
    perm = lm.perm
    assert sorted(perm.tolist()) == list(range(om.n_cell))


def test_user_order_option(teno):
    m = inputs.jittered_periodic_mesh(10, 5)
    lm = teno.Mesh(m.xy, m.tri).setup(order=3, reorder=0)
    np.testing.assert_array_equal(lm.perm, np.arange(m.n_cell))


def test_mesh_errors(teno):
    m = inputs.jittered_periodic_mesh(8, 1)
    with pytest.raises(teno.TenoError, match="order"):
        teno.Mesh(m.xy, m.tri).setup(order=7)
    with pytest.raises(teno.TenoError, match="C_T"):
        teno.Mesh(m.xy, m.tri).setup(order=3, ct=0.5)
    with pytest.raises(teno.TenoError, match="too small|candidates"):
        small = inputs.jittered_periodic_mesh(4, 1)
        teno.Mesh(small.xy, small.tri).setup(order=6)
    bad = m.tri.copy()
    bad[1] = bad[0]
    with pytest.raises(teno.TenoError, match="non-manifold|open"):
        teno.Mesh(m.xy, bad)
    with pytest.raises(teno.TenoError, match="open edge"):
        teno.Mesh(m.xy, m.tri[:-1])
    with pytest.raises(teno.TenoError, match="degenerate"):
        xy = m.xy.copy()
        xy[m.tri[0, 1]] = xy[m.tri[0, 0]]
        teno.Mesh(xy, m.tri)
    # without the periodic wrap a planar mesh has boundary (or folded) edges
    with pytest.raises(teno.TenoError, match="open edge|non-manifold"):
        teno.Mesh(m.xy, m.tri, period=None)
    with pytest.raises(teno.TenoError, match="characteristic"):
        teno.Mesh(m.xy, m.tri).setup(order=3, characteristic=2)


def test_tile_member_limit(teno):
    # 16 consecutive cells share one LDS list of distinct stencil members; a
    # shuffled cell order kept as given (reorder=0) scatters the tiles past
    # the limit, and the default reordering keeps them well inside it
    m = inputs.jittered_periodic_mesh(20, 8)
    rng = np.random.default_rng(0)
    tri = m.tri[rng.permutation(m.n_cell)]
    with pytest.raises(teno.TenoError, match="distinct stencil members"):
        teno.Mesh(m.xy, tri).setup(order=6, reorder=0)
    teno.Mesh(m.xy, tri).setup(order=6)


def test_orientation_fix_matches_oracle(teno, oracle_mod):
    m = inputs.jittered_periodic_mesh(10, 6)
    tri = m.tri.copy()
    tri[::3] = tri[::3][:, [0, 2, 1]]       # clockwise input for a third of the cells
    lm = teno.Mesh(m.xy, tri).setup(order=4)
    om = oracle_mod.OracleMesh(m.xy, tri)
    om.setup(oracle_mod.params(order=4), all_cells=False)
    for i in range(0, m.n_cell, 7):
        for k in range(4):
            np.testing.assert_array_equal(lm.stencil(i, k), om.stencil(i, k))


def test_solver_needs_a_device_or_fails_cleanly(teno):
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present: covered by the gpu tests")
    m = inputs.jittered_periodic_mesh(8, 1)
    lm = teno.Mesh(m.xy, m.tri).setup(order=3)
    with pytest.raises(teno.TenoError):
        teno.Solver(lm)


def test_boundary_faces_and_conditions(teno, oracle_mod):
    # boundary faces are numbered alike on both sides; bad kinds are refused
    m = inputs.jittered_box_mesh(9, 5, 2, 1.8, 1.0)
    lm = teno.Mesh(m.xy, m.tri, period=m.period)
    om = oracle_mod.OracleMesh(m.xy, m.tri, period=m.period)
    v, c = lm.boundary_faces()
    v2, c2 = om.boundary_faces()
    np.testing.assert_array_equal(v, v2)
    np.testing.assert_array_equal(c, c2)
    assert len(v) == 2 * (9 + 5) and lm.info().n_bface == len(v)
    with pytest.raises(teno.TenoError, match="kind"):
        lm.set_boundary(np.full(len(v), 4))
    with pytest.raises(teno.TenoError, match="states"):
        lm.set_boundary(np.full(len(v), teno.BC_PRESCRIBED))
    lm.set_boundary(np.full(len(v), teno.BC_REFLECTIVE))
    # an open edge on a doubly periodic mesh is still an error
    p = inputs.jittered_periodic_mesh(8, 1)
    with pytest.raises(teno.TenoError, match="open edge"):
        teno.Mesh(p.xy, p.tri[:-1])


@pytest.mark.parametrize("order", [3, 6])
def test_box_setup_parity_with_oracle(teno, oracle_mod, order):
    m = inputs.jittered_box_mesh(20, 12, 4, 20 / 12, 1.0)
    lm = teno.Mesh(m.xy, m.tri, period=m.period).setup(order=order)
    om = oracle_mod.OracleMesh(m.xy, m.tri, period=m.period)
    om.setup(oracle_mod.params(order=order), all_cells=False)
    for i in range(0, m.n_cell, 5):
        for k in range(4):
            np.testing.assert_array_equal(lm.stencil(i, k), om.stencil(i, k))
    for i in (0, 19, 231):
        for k in range(4):
            a = lm.lsq_operator(i, k)
            b, _ = om.lsq_operator(i, k)
            assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()


def test_disc_setup_parity_with_oracle(teno, oracle_mod):
    # the explosion problems' disc mesh: boundary faces, stencils and the
    # least-squares operators agree with the oracle's
    m = inputs.disc_mesh(1.0 / 14.0, 6)
    lm = teno.Mesh(m.xy, m.tri, period=m.period)
    om = oracle_mod.OracleMesh(m.xy, m.tri, period=m.period)
    v, c = lm.boundary_faces()
    v2, c2 = om.boundary_faces()
    np.testing.assert_array_equal(v, v2)
    np.testing.assert_array_equal(c, c2)
    lm.setup(order=5)
    om.setup(oracle_mod.params(order=5), all_cells=False)
    for i in range(0, m.n_cell, 7):
        for k in range(4):
            np.testing.assert_array_equal(lm.stencil(i, k), om.stencil(i, k))
    for i in (0, int(c[0]), m.n_cell - 1):
        for k in range(4):
            a = lm.lsq_operator(i, k)
            b, _ = om.lsq_operator(i, k)
            assert np.abs(a - b).max() <= 1e-10 * np.abs(b).max()


def test_degenerate_meshes_are_refused(teno, oracle_mod):
    # empty input, out-of-range vertex ids, and meshes with too few cells for
    # the stencils: both sides refuse with a message, neither crashes
    tri1 = np.array([[0, 1, 2]], np.int32)
    xy3 = np.array([[0.0, 0.0], [0.5, 0.0], [0.0, 0.5]])
    with pytest.raises(teno.TenoError, match="empty"):
        teno.Mesh(np.zeros((0, 2)), np.zeros((0, 3), np.int32))
    with pytest.raises(RuntimeError, match="empty"):
        oracle_mod.OracleMesh(np.zeros((0, 2)), np.zeros((0, 3), np.int32))
    with pytest.raises(teno.TenoError, match="out of range"):
        teno.Mesh(xy3, np.array([[0, 1, 5]], np.int32), period=(0.0, 0.0))
    with pytest.raises(teno.TenoError, match="too few"):
        teno.Mesh(xy3, tri1, period=(0.0, 0.0)).setup(order=3)
    box = inputs.jittered_box_mesh(3, 3, 1)
    with pytest.raises(teno.TenoError, match="too few"):
        teno.Mesh(box.xy, box.tri, period=box.period).setup(order=6)
    with pytest.raises(RuntimeError, match="too few"):
        oracle_mod.OracleMesh(box.xy, box.tri, period=box.period).setup(oracle_mod.params(order=6))


LDL_CHECK = r"""
#include <cmath>
#include <cstdio>
#include "tables.h"
using namespace teno;
// max |L D L^T - B| / max |B| of the compile-time factor, and the smallest
// pivot relative to the largest, for the smoothness form of degree R
template <int R>
void check() {
  using S = SmoothForm<R>;
  double worst = 0.0, scale = 0.0, dmin = 1e300, dmax = 0.0;
  for (int i = 0; i < S::N; ++i)
    for (int j = 0; j < S::N; ++j) {
      double s = 0.0;
      for (int k = 0; k <= (i < j ? i : j); ++k) s += S::LDL.Lt[k][i] * S::LDL.d[k] * S::LDL.Lt[k][j];
      worst = std::fmax(worst, std::fabs(s - S::B.v[i][j]));
      scale = std::fmax(scale, std::fabs(S::B.v[i][j]));
    }
  for (int k = 0; k < S::N; ++k) {
    dmin = std::fmin(dmin, S::LDL.d[k]);
    dmax = std::fmax(dmax, S::LDL.d[k]);
    if (S::LDL.Lt[k][k] != 1.0) worst = 1.0;
  }
  std::printf("%d %.3e %.3e\n", R, worst / scale, dmin / dmax);
}
int main() {
  check<2>();
  check<3>();
  check<4>();
  check<5>();
}
"""


def test_smoothness_form_factor(tmp_path):
    # the characteristic kernel forms its Gram matrices through B = L D L^T
    # (unit L, D > 0): the compile-time factor must reproduce B to round-off
    # and have positive pivots (B is positive definite on the zero-mean basis)
    src = tmp_path / "ldl.cpp"
    src.write_text(LDL_CHECK)
    exe = tmp_path / "ldl"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", os.path.join(ROOT, "paper_2105_02127_amd", "csrc"),
                    str(src), "-o", str(exe)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    rows = [line.split() for line in out if line.strip()]
    assert [int(r[0]) for r in rows] == [2, 3, 4, 5]
    for r, rel, piv in rows:
        assert float(rel) < 1e-14, (r, rel)
        assert float(piv) > 0.0, (r, piv)
