"""CPU oracle of the unstructured TENO residual -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the benchmark's CPU-baseline leg
may import this package.  It wraps `liboracle.so` (plain FP64 C++, see
`teno_oracle.cpp`) through ctypes; host arrays, user cell order.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


class Params(C.Structure):
    _fields_ = [("order", C.c_int32), ("nq", C.c_int32), ("variant", C.c_int32),
                ("power", C.c_int32), ("ct", C.c_double), ("eps", C.c_double),
                ("gamma", C.c_double), ("tie_rel", C.c_double),
                ("fallback", C.c_int32), ("characteristic", C.c_int32),
                ("dk_prime", C.c_double)]


class Diag(C.Structure):
    _fields_ = [("nonphysical", C.c_int64), ("first_bad_cell", C.c_int64),
                ("near_ties", C.c_int64), ("large_kept", C.c_int64),
                ("fallbacks", C.c_int64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def lib():
    global _lib
    if _lib is None:
        # ORACLE_LIB names another build of the same source (the mutation
        # tests load deliberately broken copies through it)
        path = os.environ.get("ORACLE_LIB", _build.LIB)
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int)
        up = C.POINTER(C.c_uint16)
        vp = C.c_void_p
        L.oracle_last_error.restype = C.c_char_p
        L.oracle_mesh_create.restype = vp
        L.oracle_mesh_create.argtypes = [C.c_int, dp, C.c_int, ip, dp]
        L.oracle_mesh_destroy.argtypes = [vp]
        L.oracle_mesh_counts.argtypes = [vp, ip, ip]
        L.oracle_mesh_geometry.argtypes = [vp, dp, dp, ip]
        L.oracle_mesh_faces.argtypes = [vp, ip, ip, ip, ip, dp, dp, ip]
        L.oracle_setup.argtypes = [vp, C.POINTER(Params), C.c_int]
        L.oracle_prepare_cells.argtypes = [vp, C.c_int, ip]
        L.oracle_stencil.argtypes = [vp, C.c_int, C.c_int, ip, C.c_int]
        L.oracle_lsq_operator.argtypes = [vp, C.c_int, C.c_int, dp, dp]
        L.oracle_lsq_solve.argtypes = [C.c_int, C.c_int, dp, dp, dp]
        L.oracle_gauss01.argtypes = [C.c_int, dp, dp]
        L.oracle_tref_moment.restype = C.c_double
        L.oracle_tref_moment.argtypes = [C.c_int, C.c_int, C.c_int]
        L.oracle_tri_moment.restype = C.c_double
        L.oracle_tri_moment.argtypes = [dp, C.c_int, C.c_int, C.c_int]
        L.oracle_smoothness.restype = C.c_double
        L.oracle_smoothness.argtypes = [C.c_int, dp]
        L.oracle_basis.argtypes = [C.c_int, ip, ip, dp]
        L.oracle_select.argtypes = [C.POINTER(Params), dp, dp, ip]
        L.oracle_hll.argtypes = [dp, dp, C.c_double, C.c_double, C.c_double, dp]
        L.oracle_boundary_count.argtypes = [vp]
        L.oracle_boundary_faces.argtypes = [vp, ip, ip]
        L.oracle_set_boundary.argtypes = [vp, ip, dp]
        L.oracle_char_basis.argtypes = [dp, C.c_double, C.c_double, C.c_double, dp, dp]
        L.oracle_cweno_weights.argtypes = [C.POINTER(Params), dp, dp, dp]
        L.oracle_reconstruct_cells.argtypes = [vp, dp, C.c_int, ip, dp, up, dp, C.POINTER(Diag),
                                               up]
        L.oracle_residual.argtypes = [vp, dp, dp, up, C.c_int, dp, C.POINTER(Diag), up]
        L.oracle_residual_cells.argtypes = [vp, dp, C.c_int, ip, dp, up]
        L.oracle_dt.restype = C.c_double
        L.oracle_dt.argtypes = [vp, dp, C.c_double]
        L.oracle_rk_step.argtypes = [vp, dp, dp, C.c_double, up, C.c_int, dp, C.POINTER(Diag),
                                     up]
        L.oracle_jvp.argtypes = [vp, dp, up, dp, dp]
        L.oracle_vjp.argtypes = [vp, dp, up, dp, dp]
        L.oracle_vjp_rk_step.argtypes = [vp, dp, up, C.c_double, dp, dp]
        L.oracle_vjp_scale.argtypes = [vp, dp, up, dp, dp]
        L.oracle_vjp_rk_step_scale.argtypes = [vp, dp, up, C.c_double, dp, dp]
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_get_threads.restype = C.c_int
        L.oracle_default_params.argtypes = [C.POINTER(Params)]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _i(a):
    return a.ctypes.data_as(C.POINTER(C.c_int))


def _u(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint16))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _check(rc):
    if rc < 0:
        raise RuntimeError("oracle: " + lib().oracle_last_error().decode())
    return rc


def params(order=5, ct=1e-6, eps=None, power=None, gamma=1.4, nq=0, variant=0, tie_rel=1e-10,
           fallback=0, dk_prime=1e4, characteristic=0):
    """Scheme parameters.  eps and power default to the paper's values of
    the variant: 1e-12 and 6 for TENO (Sec. 3.2), 1e-14 and 4 for CWENO
    (variant 2, Sec. 2.4).  characteristic=1 selects in characteristic
    variables, face by face (Sec. 2.3)."""
    if eps is None:
        eps = 1e-14 if variant == 2 else 1e-12
    if power is None:
        power = 4 if variant == 2 else 6
    p = Params()
    p.order, p.ct, p.eps, p.power, p.gamma, p.nq, p.variant, p.tie_rel = \
        order, ct, eps, power, gamma, nq, variant, tie_rel
    p.fallback = fallback
    p.dk_prime = dk_prime
    p.characteristic = characteristic
    return p


def set_threads(n: int):
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


class OracleMesh:
    """Geometry, faces and (after `setup`) reconstruction data of one mesh."""

    def __init__(self, xy, tri, period=(1.0, 1.0)):
        L = lib()
        self._xy = _f64(xy)
        self._tri = np.ascontiguousarray(tri, dtype=np.int32)
        per = None if period is None else _f64(period)
        self.h = L.oracle_mesh_create(self._xy.shape[0], _d(self._xy), self._tri.shape[0],
                                      _i(self._tri), None if per is None else _d(per))
        if not self.h:
            raise RuntimeError("oracle: " + L.oracle_last_error().decode())
        nc, nf = C.c_int(), C.c_int()
        L.oracle_mesh_counts(self.h, C.byref(nc), C.byref(nf))
        self.n_cell, self.n_face = nc.value, nf.value
        self.prm = None
        self.nq = 0

    def __del__(self):
        if getattr(self, "h", None):
            lib().oracle_mesh_destroy(self.h)
            self.h = None

    # geometry -------------------------------------------------------------
    def geometry(self):
        area = np.empty(self.n_cell)
        cen = np.empty((self.n_cell, 2))
        tri = np.empty((self.n_cell, 3), dtype=np.int32)
        lib().oracle_mesh_geometry(self.h, _d(area), _d(cen), _i(tri))
        return area, cen, tri

    def faces(self):
        nf = self.n_face
        fL, fR, fLe, fRe = (np.empty(nf, dtype=np.int32) for _ in range(4))
        n = np.empty((nf, 2))
        ln = np.empty(nf)
        cf = np.empty((self.n_cell, 3), dtype=np.int32)
        lib().oracle_mesh_faces(self.h, _i(fL), _i(fR), _i(fLe), _i(fRe), _d(n), _d(ln), _i(cf))
        return dict(L=fL, R=fR, Le=fLe, Re=fRe, normal=n, length=ln, cell_face=cf)

    # boundaries -----------------------------------------------------------
    def boundary_faces(self):
        """(verts [nb, 2], cell [nb]) of the boundary faces (open axes)."""
        nb = int(lib().oracle_boundary_count(self.h))
        v = np.empty((nb, 2), dtype=np.int32)
        c = np.empty(nb, dtype=np.int32)
        lib().oracle_boundary_faces(self.h, _i(v), _i(c))
        return v, c

    def set_boundary(self, kind, state=None):
        k = np.ascontiguousarray(kind, dtype=np.int32)
        st = None if state is None else _f64(state)
        _check(lib().oracle_set_boundary(self.h, _i(k), None if st is None else _d(st)))
        return self

    # setup ----------------------------------------------------------------
    def setup(self, prm: Params, all_cells: bool = True):
        _check(lib().oracle_setup(self.h, C.byref(prm), 1 if all_cells else 0))
        self.prm = prm
        self.nq = prm.nq if prm.nq > 0 else (prm.order + 1) // 2
        return self

    def prepare(self, cells):
        c = np.ascontiguousarray(cells, dtype=np.int32)
        _check(lib().oracle_prepare_cells(self.h, c.size, _i(c)))

    def rows(self, k):
        r = (self.prm.order - 1) if k == 3 else 2
        return (r + 1) * (r + 2) - 1

    def ncoef(self, k):
        r = (self.prm.order - 1) if k == 3 else 2
        return (r + 1) * (r + 2) // 2 - 1

    def stencil(self, cell, k, brute=False):
        out = np.empty(self.rows(k), dtype=np.int32)
        _check(lib().oracle_stencil(self.h, int(cell), int(k), _i(out), 1 if brute else 0))
        return out

    def lsq_operator(self, cell, k):
        m = np.empty((self.ncoef(k), self.rows(k)))
        rc = C.c_double()
        _check(lib().oracle_lsq_operator(self.h, int(cell), int(k), _d(m), C.byref(rc)))
        return m, rc.value

    # evaluation -------------------------------------------------------------
    @property
    def characteristic(self) -> bool:
        return bool(self.prm is not None and self.prm.characteristic)

    def reconstruct_cells(self, U, cells):
        """(fp [n][3][nq][4], flags, beta, diag).  flags: [n], or [n][3]
        (one per local edge) in characteristic variables, where beta is
        None.  diag["tie_mask"] is laid out like flags: nibble v is 0xF
        where the selection of variable v met a near tie."""
        U = _f64(U)
        c = np.ascontiguousarray(cells, dtype=np.int32)
        fp = np.empty((c.size, 3, self.nq, 4))
        fl = np.empty((c.size, 3) if self.characteristic else c.size, dtype=np.uint16)
        ties = np.zeros_like(fl)
        beta = np.empty((c.size, 4, 4))
        dg = Diag(0, -1, 0, 0, 0)
        _check(lib().oracle_reconstruct_cells(self.h, _d(U), c.size, _i(c), _d(fp), _u(fl),
                                              _d(beta), C.byref(dg), _u(ties)))
        d = dg.as_dict()
        d["tie_mask"] = ties
        return fp, fl, (None if self.characteristic else beta), d

    def residual(self, U, frozen_flags=None, want_fp=False):
        """flags: [n_cell], or [3][n_cell] (per local edge) in
        characteristic variables; diag["tie_mask"] is laid out like flags
        (nibble v = 0xF where variable v met a near tie)."""
        U = _f64(U)
        R = np.empty_like(U)
        if frozen_flags is not None:
            fl = np.ascontiguousarray(frozen_flags, dtype=np.uint16).copy()
        else:
            fl = np.empty((3, self.n_cell) if self.characteristic else self.n_cell,
                          dtype=np.uint16)
        fp = np.empty((self.n_cell, 3, self.nq, 4)) if want_fp else None
        ties = np.zeros(fl.shape, dtype=np.uint16)
        dg = Diag(0, -1, 0, 0, 0)
        _check(lib().oracle_residual(self.h, _d(U), _d(R), _u(fl),
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
        R = np.empty((c.size, 4))
        fl = np.empty((c.size, 3) if self.characteristic else c.size, dtype=np.uint16)
        _check(lib().oracle_residual_cells(self.h, _d(U), c.size, _i(c), _d(R), _u(fl)))
        return R, fl

    def dt(self, U, cfl=0.4):
        return float(lib().oracle_dt(self.h, _d(_f64(U)), float(cfl)))

    def rk_step(self, U, dt, frozen_flags3=None, want_stages=False):
        U = _f64(U)
        out = np.empty_like(U)
        if frozen_flags3 is not None:
            fl = np.ascontiguousarray(frozen_flags3, dtype=np.uint16).copy()
        else:
            fl = np.empty((3, 3, self.n_cell) if self.characteristic else (3, self.n_cell),
                          dtype=np.uint16)
        st = np.empty((3,) + U.shape) if want_stages else None
        ties = np.zeros(fl.shape, dtype=np.uint16)
        dg = Diag(0, -1, 0, 0, 0)
        _check(lib().oracle_rk_step(self.h, _d(U), _d(out), float(dt), _u(fl),
                                    1 if frozen_flags3 is not None else 0,
                                    None if st is None else _d(st), C.byref(dg), _u(ties)))
        res = dict(U=out, flags=fl, diag=dg.as_dict())
        res["diag"]["tie_mask"] = ties
        if want_stages:
            res["stages"] = st
        return res

    def jvp(self, U, flags, v):
        U, v = _f64(U), _f64(v)
        fl = np.ascontiguousarray(flags, dtype=np.uint16)
        Jv = np.empty_like(U)
        _check(lib().oracle_jvp(self.h, _d(U), _u(fl), _d(v), _d(Jv)))
        return Jv

    def vjp(self, U, flags, lam):
        U, lam = _f64(U), _f64(lam)
        fl = np.ascontiguousarray(flags, dtype=np.uint16)
        ub = np.empty_like(U)
        _check(lib().oracle_vjp(self.h, _d(U), _u(fl), _d(lam), _d(ub)))
        return ub

    def vjp_scale(self, U, flags, lam):
        """Comparison scale of vjp(U, flags, lam): per cell and variable, the
        summed magnitudes of the terms the adjoint adds there (see
        oracle_vjp_scale)."""
        U, lam = _f64(U), _f64(lam)
        fl = np.ascontiguousarray(flags, dtype=np.uint16)
        S = np.empty_like(U)
        _check(lib().oracle_vjp_scale(self.h, _d(U), _u(fl), _d(lam), _d(S)))
        return S

    def vjp_rk_step_scale(self, stages, flags3, dt, lam_out):
        """Comparison scale of vjp_rk_step (magnitudes through the stage
        chain); lam_out may itself be a scale of the previous step."""
        st, lam_out = _f64(stages), _f64(lam_out)
        fl = np.ascontiguousarray(flags3, dtype=np.uint16)
        S = np.empty_like(lam_out)
        _check(lib().oracle_vjp_rk_step_scale(self.h, _d(st), _u(fl), float(dt), _d(lam_out),
                                              _d(S)))
        return S

    def vjp_rk_step(self, stages, flags3, dt, lam_out):
        st, lam_out = _f64(stages), _f64(lam_out)
        fl = np.ascontiguousarray(flags3, dtype=np.uint16)
        lam_in = np.empty_like(lam_out)
        _check(lib().oracle_vjp_rk_step(self.h, _d(st), _u(fl), float(dt), _d(lam_out),
                                        _d(lam_in)))
        return lam_in


# ---------------------------------------------------------------------------
# Stand-alone helpers used by the pin tests
# ---------------------------------------------------------------------------
def gauss01(n):
    t, w = np.empty(n), np.empty(n)
    lib().oracle_gauss01(n, _d(t), _d(w))
    return t, w


def tref_moment(a, b, n=8):
    return float(lib().oracle_tref_moment(a, b, n))


def tri_moment(q, a, b, n=8):
    return float(lib().oracle_tri_moment(_d(_f64(q)), a, b, n))


def smoothness(r, coef):
    return float(lib().oracle_smoothness(int(r), _d(_f64(coef))))


def basis(r):
    n = (r + 1) * (r + 2) // 2 - 1
    ea, eb = np.empty(n, dtype=np.int32), np.empty(n, dtype=np.int32)
    mean = np.empty(n)
    lib().oracle_basis(r, _i(ea), _i(eb), _d(mean))
    return ea, eb, mean


def select(beta, prm: Params):
    b = _f64(beta)
    chi = np.empty(4)
    ties = C.c_int()
    fl = lib().oracle_select(C.byref(prm), _d(b), _d(chi), C.byref(ties))
    return fl, chi, ties.value


def cweno_weights(beta, prm: Params):
    """(omega, d): nonlinear and linear CWENO weights of the four stencils."""
    b = _f64(beta)
    w = np.empty(4)
    d = np.empty(4)
    lib().oracle_cweno_weights(C.byref(prm), _d(b), _d(w), _d(d))
    return w, d


def char_basis(u, n, gamma=1.4):
    """(R, L): right eigenvectors (columns) of the Euler flux Jacobian in
    direction n at state u, and L = R^-1; identity for a non-physical u."""
    R, L = np.empty((4, 4)), np.empty((4, 4))
    lib().oracle_char_basis(_d(_f64(u)), float(n[0]), float(n[1]), float(gamma), _d(R), _d(L))
    return R, L


def hll(uL, uR, n, gamma=1.4):
    out = np.empty(4)
    lib().oracle_hll(_d(_f64(uL)), _d(_f64(uR)), float(n[0]), float(n[1]), float(gamma), _d(out))
    return out


def lsq_solve(A, b):
    A = np.asfortranarray(A, dtype=np.float64)
    m, n = A.shape
    x = np.empty(n)
    Ac = np.ascontiguousarray(A.T)  # column-major of A == row-major of A^T
    _check(lib().oracle_lsq_solve(m, n, _d(Ac), _d(_f64(b)), _d(x)))
    return x
