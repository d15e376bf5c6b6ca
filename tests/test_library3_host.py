"""Host-side checks of the tetrahedral path of libteno (no GPU): exported ABI,
set-up parity with the tetrahedral oracle (stencil lists exactly,
least-squares operators to round-off), error paths."""
import os
import re

import numpy as np
import pytest

from paper_2105_02127_amd import inputs3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def t3():
    from paper_2105_02127_amd import teno3 as t
    t.load()
    return t


@pytest.fixture(scope="module")
def tet():
    from oracle import tet as t
    t.lib()
    return t


def declared_functions():
    src = open(os.path.join(ROOT, "include", "teno3.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(teno3_\w+)\s*\(", src, flags=re.M)))


def test_every_declared_symbol_is_exported(t3):
    names = declared_functions()
    assert len(names) >= 15
    lib = t3.load()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(t3.SIGNATURES3), set(names) ^ set(t3.SIGNATURES3)


@pytest.mark.parametrize("n,order,seed", [(5, 3, 1), (5, 4, 2), (6, 5, 3), (7, 6, 4)])
def test_setup_parity_with_oracle(t3, tet, n, order, seed):
    m = inputs3.jittered_periodic_cube(n, seed)
    lm = t3.TetMesh(m.xyz, m.tet).setup(order=order)
    om = tet.OracleTetMesh(m.xyz, m.tet)
    om.setup(tet.params(order=order), all_cells=False)
    info = lm.info()
    assert info.n_cell == om.n_cell and info.n_face == om.n_face == 2 * om.n_cell
    nk = order * (order + 1) * (order + 2) // 6
    assert (info.rows_large, info.n_coef_large) == (2 * nk - 1, nk - 1)
    assert (info.rows_small, info.n_coef_small) == (19, 9)
    assert info.n_quad == (6 if order <= 4 else 7)
    worst = 0.0
    for i in range(0, om.n_cell, 7):
        for k in range(5):
            np.testing.assert_array_equal(lm.stencil(i, k), om.stencil(i, k))
            Ml = lm.lsq_operator(i, k)
            Mo, _ = om.lsq_operator(i, k)
            worst = max(worst, np.abs(Ml - Mo).max() / np.abs(Mo).max())
    # the two sides integrate the basis over the stencil cells with different
    # exact rules (Grundmann-Moller against collapsed Gauss), so A differs by
    # rounding, amplified in pinv(A) by the conditioning of the monomial
    # least squares: at degree 5 (min |R_jj| / max |R_jj| ~ 1e-4) entries
    # move by ~1e-10 of the largest, face values by ~2e-11 of the data range
    assert worst < (1e-11 if order <= 5 else 1e-9), worst
    assert sorted(lm.perm.tolist()) == list(range(om.n_cell))


def test_box_setup_and_boundary_faces_match_oracle(t3, tet):
    m = inputs3.jittered_box3(4, 3, 3, 7, (0, 0, 0), (1.0, 0.8, 0.7))
    lm = t3.TetMesh(m.xyz, m.tet, period=(0, 0, 0))
    om = tet.OracleTetMesh(m.xyz, m.tet, period=(0, 0, 0))
    lv, lc = lm.boundary_faces()
    ov, oc = om.boundary_faces()
    np.testing.assert_array_equal(lc, oc)
    np.testing.assert_array_equal(np.sort(lv, 1), np.sort(ov, 1))
    lm.setup(order=3)
    om.setup(tet.params(order=3), all_cells=False)
    for i in range(0, om.n_cell, 5):
        for k in range(5):
            np.testing.assert_array_equal(lm.stencil(i, k), om.stencil(i, k))


def test_user_order_option(t3):
    m = inputs3.jittered_periodic_cube(5, 5)
    lm = t3.TetMesh(m.xyz, m.tet).setup(order=3, reorder=0)
    np.testing.assert_array_equal(lm.perm, np.arange(m.n_cell))


def test_mesh_errors(t3):
    m = inputs3.jittered_periodic_cube(4, 1)
    with pytest.raises(t3.TenoError, match="order"):
        t3.TetMesh(m.xyz, m.tet).setup(order=7)
    with pytest.raises(t3.TenoError, match="C_T"):
        t3.TetMesh(m.xyz, m.tet).setup(order=3, ct=0.5)
    with pytest.raises(t3.TenoError, match="variant"):
        t3.TetMesh(m.xyz, m.tet).setup(order=3, variant=2)
    with pytest.raises(t3.TenoError, match="conservative"):
        t3.TetMesh(m.xyz, m.tet).setup(order=3, characteristic=2)
    with pytest.raises(t3.TenoError, match="too small|too few"):
        t3.TetMesh(m.xyz, m.tet).setup(order=6)
    bad = m.tet.copy()
    bad[1] = bad[0]
    with pytest.raises(t3.TenoError, match="non-manifold|open face"):
        t3.TetMesh(m.xyz, bad)
    with pytest.raises(t3.TenoError, match="open face"):
        t3.TetMesh(m.xyz, m.tet[:-1])
    with pytest.raises(t3.TenoError, match="degenerate"):
        xyz = m.xyz.copy()
        xyz[m.tet[0, 1]] = xyz[m.tet[0, 0]]
        t3.TetMesh(xyz, m.tet)
    with pytest.raises(t3.TenoError, match="out of range"):
        bad = m.tet.copy()
        bad[0, 0] = m.xyz.shape[0]
        t3.TetMesh(m.xyz, bad)
    mb = inputs3.jittered_box3(3, 3, 3, 2)
    lm = t3.TetMesh(mb.xyz, mb.tet, period=(0, 0, 0))
    with pytest.raises(t3.TenoError, match="transmissive or reflective"):
        lm.set_boundary(np.full(lm.boundary_faces()[0].shape[0], 3, np.int32))
