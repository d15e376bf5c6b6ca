"""CPU oracle of the TENO residual on tetrahedra -- TEST INFRASTRUCTURE ONLY.

Only `tests/` and `__graft_entry__.smoke()` may import this module.  It wraps
`liboracle3.so` (plain FP64 C++, see `teno3_oracle.cpp`) through ctypes; host
arrays, user cell order, U[cell][5] = (rho, rho u, rho v, rho w, E).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class Params(C.Structure):
    _fields_ = [("order", C.c_int32), ("variant", C.c_int32), ("power", C.c_int32),
                ("fallback", C.c_int32), ("ct", C.c_double), ("eps", C.c_double),
                ("gamma", C.c_double), ("tie_rel", C.c_double)]


class Diag(C.Structure):
    _fields_ = [("nonphysical", C.c_int64), ("first_bad_cell", C.c_int64),
                ("near_ties", C.c_int64), ("large_kept", C.c_int64), ("fallbacks", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def lib():
    global _lib
    if _lib is None:
        # ORACLE3_LIB names another build of the same source (mutation tests)
        path = os.environ.get("ORACLE3_LIB", _build.LIB3)
        if path == _build.LIB3 and not os.path.exists(path):
            _build.build3()
        L = C.CDLL(path)
        dp, ip, up, vp = C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_uint32), C.c_void_p
        L.oracle3_last_error.restype = C.c_char_p
        L.oracle3_mesh_create.restype = vp
        L.oracle3_mesh_create.argtypes = [C.c_int, dp, C.c_int, ip, dp]
        L.oracle3_mesh_destroy.argtypes = [vp]
        L.oracle3_mesh_counts.argtypes = [vp, ip, ip, ip]
        L.oracle3_mesh_geometry.argtypes = [vp, dp, dp, ip]
        L.oracle3_mesh_faces.argtypes = [vp, ip, ip, ip, ip, dp, dp, ip]
        L.oracle3_boundary_faces.argtypes = [vp, ip, ip]
        L.oracle3_set_boundary.argtypes = [vp, ip]
        L.oracle3_setup.argtypes = [vp, C.POINTER(Params), C.c_int]
        L.oracle3_face_pairing.argtypes = [vp, ip]
        L.oracle3_prepare_cells.argtypes = [vp, C.c_int, ip]
        L.oracle3_stencil.argtypes = [vp, C.c_int, C.c_int, ip, C.c_int]
        L.oracle3_lsq_operator.argtypes = [vp, C.c_int, C.c_int, dp, dp]
        L.oracle3_reconstruct_cells.argtypes = [vp, dp, C.c_int, ip, dp, up, dp, C.POINTER(Diag), up]
        L.oracle3_residual.argtypes = [vp, dp, dp, up, C.c_int, dp, C.POINTER(Diag), up]
        L.oracle3_residual_cells.argtypes = [vp, dp, C.c_int, ip, dp, up]
        L.oracle3_dt.restype = C.c_double
        L.oracle3_dt.argtypes = [vp, dp, C.c_double]
        L.oracle3_rk_step.argtypes = [vp, dp, dp, C.c_double, up, C.c_int, dp, C.POINTER(Diag), up]
        L.oracle3_face_rule.argtypes = [C.c_int, dp, dp]
        L.oracle3_tet_moment.restype = C.c_double
        L.oracle3_tet_moment.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
        L.oracle3_basis.argtypes = [C.c_int, ip, ip, ip, dp]
        L.oracle3_smoothness.restype = C.c_double
        L.oracle3_smoothness.argtypes = [C.c_int, dp]
        L.oracle3_select.restype = C.c_uint
        L.oracle3_select.argtypes = [C.POINTER(Params), dp, dp, ip]
        L.oracle3_hll.argtypes = [dp, dp, dp, C.c_double, dp]
        L.oracle3_set_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _u(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc):
    if rc < 0:
        raise RuntimeError("oracle3: " + lib().oracle3_last_error().decode())
    return rc


def params(order=4, ct=1e-6, eps=1e-12, power=6, gamma=1.4, variant=0, tie_rel=1e-10,
           fallback=0):
    """Scheme parameters: the paper's built-in TENO values (Sec. 3.2-3.3);
    variant 1 = the linear scheme on the large stencil."""
    p = Params()
    p.order, p.variant, p.power, p.fallback = order, variant, power, fallback
    p.ct, p.eps, p.gamma, p.tie_rel = ct, eps, gamma, tie_rel
    return p


def npt_of(order: int) -> int:
    return 6 if order <= 4 else 7


def stencil_rows(degree: int) -> int:
    return (degree + 1) * (degree + 2) * (degree + 3) // 3 - 1


def n_coef(degree: int) -> int:
    return (degree + 1) * (degree + 2) * (degree + 3) // 6 - 1


class OracleTetMesh:
    """Geometry, faces and (after `setup`) reconstruction data of one mesh."""

    def __init__(self, xyz, tet, period=(1.0, 1.0, 1.0)):
        L = lib()
        self._xyz = _f64(xyz)
        self._tet = np.ascontiguousarray(tet, dtype=np.int32)
        per = None if period is None else _f64(period)
        self.h = L.oracle3_mesh_create(self._xyz.shape[0], _d(self._xyz), self._tet.shape[0],
                                       _i(self._tet), None if per is None else _d(per))
        if not self.h:
            raise RuntimeError("oracle3: " + L.oracle3_last_error().decode())
        nc, nf, nb = C.c_int(), C.c_int(), C.c_int()
        L.oracle3_mesh_counts(self.h, C.byref(nc), C.byref(nf), C.byref(nb))
        self.n_cell, self.n_face, self.n_bface = nc.value, nf.value, nb.value
        self.prm = None
        self.npt = 0

    def __del__(self):
        if getattr(self, "h", None):
            lib().oracle3_mesh_destroy(self.h)
            self.h = None

    def geometry(self):
        vol = np.empty(self.n_cell)
        cen = np.empty((self.n_cell, 3))
        tet = np.empty((self.n_cell, 4), dtype=np.int32)
        lib().oracle3_mesh_geometry(self.h, _d(vol), _d(cen), _i(tet))
        return vol, cen, tet

    def faces(self):
        nf = self.n_face
        fL, fR, fLe, fRe = (np.empty(nf, dtype=np.int32) for _ in range(4))
        n = np.empty((nf, 3))
        ar = np.empty(nf)
        cf = np.empty((self.n_cell, 4), dtype=np.int32)
        lib().oracle3_mesh_faces(self.h, _i(fL), _i(fR), _i(fLe), _i(fRe), _d(n), _d(ar), _i(cf))
        return dict(L=fL, R=fR, Le=fLe, Re=fRe, normal=n, area=ar, cell_face=cf)

    def boundary_faces(self):
        v = np.empty((self.n_bface, 3), dtype=np.int32)
        c = np.empty(self.n_bface, dtype=np.int32)
        lib().oracle3_boundary_faces(self.h, _i(v), _i(c))
        return v, c

    def set_boundary(self, kind):
        k = np.ascontiguousarray(kind, dtype=np.int32)
        _check(lib().oracle3_set_boundary(self.h, _i(k)))
        return self

    def setup(self, prm: Params, all_cells: bool = True):
        _check(lib().oracle3_setup(self.h, C.byref(prm), 1 if all_cells else 0))
        self.prm = prm
        self.npt = npt_of(prm.order)
        return self

    def pairing(self):
        pr = np.empty((self.n_face, self.npt), dtype=np.int32)
        _check(lib().oracle3_face_pairing(self.h, _i(pr)))
        return pr

    def rows(self, k):
        return stencil_rows(self.prm.order - 1 if k == 4 else 2)

    def ncoef(self, k):
        return n_coef(self.prm.order - 1 if k == 4 else 2)

    def stencil(self, cell, k, brute=False):
        out = np.empty(self.rows(k), dtype=np.int32)
        _check(lib().oracle3_stencil(self.h, int(cell), int(k), _i(out), 1 if brute else 0))
        return out

    def lsq_operator(self, cell, k):
        m = np.empty((self.ncoef(k), self.rows(k)))
        rc = C.c_double()
        _check(lib().oracle3_lsq_operator(self.h, int(cell), int(k), _d(m), C.byref(rc)))
        return m, rc.value

    def reconstruct_cells(self, U, cells):
        """(fp [n][4][npt][5], flags [n] uint32, beta [n][5][5], diag);
        diag["tie_mask"] [n]: the 5-bit field of variable v is 0x1F where its
        selection met a near tie."""
        U = _f64(U)
        c = np.ascontiguousarray(cells, dtype=np.int32)
        fp = np.empty((c.size, 4, self.npt, 5))
        fl = np.empty(c.size, dtype=np.uint32)
        ties = np.zeros(c.size, dtype=np.uint32)
        beta = np.empty((c.size, 5, 5))
        dg = Diag(0, -1, 0, 0, 0)
        _check(lib().oracle3_reconstruct_cells(self.h, _d(U), c.size, _i(c), _d(fp), _u(fl),
                                               _d(beta), C.byref(dg), _u(ties)))
        d = dg.as_dict()
        d["tie_mask"] = ties
        return fp, fl, beta, d

    def residual(self, U, frozen_flags=None, want_fp=False):
        U = _f64(U)
        R = np.empty_like(U)
        if frozen_flags is not None:
            fl = np.ascontiguousarray(frozen_flags, dtype=np.uint32).copy()
        else:
            fl = np.empty(self.n_cell, dtype=np.uint32)
        fp = np.empty((self.n_cell, 4, self.npt, 5)) if want_fp else None
        ties = np.zeros(self.n_cell, dtype=np.uint32)
        dg = Diag(0, -1, 0, 0, 0)
        _check(lib().oracle3_residual(self.h, _d(U), _d(R), _u(fl),
                                      1 if frozen_flags is not None else 0,
                                      None if fp is None else _d(fp), C.byref(dg), _u(ties)))
        out = dict(R=R, flags=fl, diag=dg.as_dict())
        out["diag"]["tie_mask"] = ties
        if want_fp:
            out["fp"] = fp
        return out

    def residual_cells(self, U, cells):
        U = _f64(U)
        c = np.ascontiguousarray(cells, dtype=np.int32)
        R = np.empty((c.size, 5))
        fl = np.empty(c.size, dtype=np.uint32)
        _check(lib().oracle3_residual_cells(self.h, _d(U), c.size, _i(c), _d(R), _u(fl)))
        return R, fl

    def dt(self, U, cfl=0.4):
        return float(lib().oracle3_dt(self.h, _d(_f64(U)), float(cfl)))

    def rk_step(self, U, dt, frozen_flags3=None, want_stages=False):
        U = _f64(U)
        out = np.empty_like(U)
        if frozen_flags3 is not None:
            fl = np.ascontiguousarray(frozen_flags3, dtype=np.uint32).copy()
        else:
            fl = np.empty((3, self.n_cell), dtype=np.uint32)
        st = np.empty((3,) + U.shape) if want_stages else None
        ties = np.zeros((3, self.n_cell), dtype=np.uint32)
        dg = Diag(0, -1, 0, 0, 0)
        _check(lib().oracle3_rk_step(self.h, _d(U), _d(out), float(dt), _u(fl),
                                     1 if frozen_flags3 is not None else 0,
                                     None if st is None else _d(st), C.byref(dg), _u(ties)))
        res = dict(U=out, flags=fl, diag=dg.as_dict())
        res["diag"]["tie_mask"] = ties
        if want_stages:
            res["stages"] = st
        return res


def set_threads(n: int):
    lib().oracle3_set_threads(int(n))


def face_rule(order):
    b = np.empty((7, 3))
    w = np.empty(7)
    n = lib().oracle3_face_rule(int(order), _d(b), _d(w))
    return b[:n], w[:n]


def tet_moment(a, b, c, n=6):
    return float(lib().oracle3_tet_moment(a, b, c, n))


def basis(r):
    n = n_coef(r)
    ea, eb, ec = (np.empty(n, dtype=np.int32) for _ in range(3))
    mean = np.empty(n)
    lib().oracle3_basis(r, _i(ea), _i(eb), _i(ec), _d(mean))
    return ea, eb, ec, mean


def smoothness(r, coef):
    return float(lib().oracle3_smoothness(int(r), _d(_f64(coef))))


def select(beta, prm: Params):
    chi = np.empty(5)
    ties = C.c_int()
    fl = lib().oracle3_select(C.byref(prm), _d(_f64(beta)), _d(chi), C.byref(ties))
    return int(fl), chi, ties.value


def hll(uL, uR, n, gamma=1.4):
    out = np.empty(5)
    lib().oracle3_hll(_d(_f64(uL)), _d(_f64(uR)), _d(_f64(n)), float(gamma), _d(out))
    return out
