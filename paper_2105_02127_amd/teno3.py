"""ctypes binding of the tetrahedral path of libteno (include/teno3.h).

Argument marshalling only: every step of the residual runs in the library's
HIP kernels (device) or host set-up code.  Device state tensors are float64
[n_cell, 5] = (rho, rho u, rho v, rho w, E) in the library's internal
(Morton) cell order; `TetMesh.to_internal` / `to_user` convert.  Flags are
uint32 bit patterns carried in int32 tensors.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import teno as _t
from .teno import Diag, Info, TenoError, _check, _ptr, _stream, default_params

_vp, _dp, _ip, _i32 = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_int32

# Every exported symbol of include/teno3.h with (restype, argtypes).
SIGNATURES3 = {
    "teno3_mesh_create": (C.c_int, [_i32, _dp, _i32, _ip, _dp, C.POINTER(_vp)]),
    "teno3_mesh_boundary_count": (C.c_int, [_vp, _ip]),
    "teno3_mesh_boundary_faces": (C.c_int, [_vp, _ip, _ip]),
    "teno3_mesh_set_boundary": (C.c_int, [_vp, _ip]),
    "teno3_mesh_setup": (C.c_int, [_vp, C.POINTER(_t.Params)]),
    "teno3_mesh_info": (C.c_int, [_vp, C.POINTER(Info)]),
    "teno3_mesh_permutation": (C.c_int, [_vp, _ip]),
    "teno3_mesh_stencil": (C.c_int, [_vp, _i32, _i32, _ip]),
    "teno3_mesh_lsq_operator": (C.c_int, [_vp, _i32, _i32, _dp]),
    "teno3_mesh_destroy": (None, [_vp]),
    "teno3_solver_create": (C.c_int, [_vp, _i32, C.POINTER(_vp)]),
    "teno3_solver_destroy": (None, [_vp]),
    "teno3_reconstruct": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "teno3_residual": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "teno3_max_dt": (C.c_int, [_vp, _vp, C.c_double, _vp, _vp]),
    "teno3_rk_stage": (C.c_int, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _vp]),
    "teno3_rk_step": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "teno3_diagnostics": (C.c_int, [_vp, C.POINTER(Diag), _i32, _vp]),
    "teno3_profile_enable": (C.c_int, [_vp, _i32]),
    "teno3_profile_read": (C.c_int, [_vp, _dp, C.POINTER(C.c_int64), _i32]),
}

KERNEL_KINDS3 = ("reconstruct", "flux_update", "dt")
_bound = None


def load():
    """libteno with the tetrahedral signatures set (raises if not built)."""
    global _bound
    L = _t.load()
    if _bound is not L:
        for name, (res, args) in SIGNATURES3.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = L
    return L


def _torch_index(idx, like):
    import torch
    return torch.as_tensor(idx.astype(np.int64), device=like.device)


class TetMesh:
    """Tetrahedral mesh plus (after `setup`) stencils and operators.
    period: the period of each axis, 0 for an open axis (None: all open)."""

    def __init__(self, xyz, tet, period=(1.0, 1.0, 1.0)):
        L = load()
        xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        tet = np.ascontiguousarray(tet, dtype=np.int32)
        per = None if period is None else np.ascontiguousarray(period, dtype=np.float64)
        h = C.c_void_p()
        _check(L.teno3_mesh_create(xyz.shape[0], xyz.ctypes.data_as(_dp), tet.shape[0],
                                   tet.ctypes.data_as(_ip),
                                   None if per is None else per.ctypes.data_as(_dp), C.byref(h)))
        self.h = h
        self.n_cell = int(tet.shape[0])
        self.params = None
        self._perm = None

    def __del__(self):
        if getattr(self, "h", None) and _t._lib is not None:
            _t._lib.teno3_mesh_destroy(self.h)
            self.h = None

    def setup(self, **kw):
        kw.setdefault("order", 4)
        p = default_params(**kw)
        _check(load().teno3_mesh_setup(self.h, C.byref(p)))
        self.params = p
        self._perm = None
        return self

    def info(self) -> Info:
        i = Info()
        _check(load().teno3_mesh_info(self.h, C.byref(i)))
        return i

    @property
    def perm(self) -> np.ndarray:
        """perm[internal] = user cell id."""
        if self._perm is None:
            p = np.empty(self.n_cell, dtype=np.int32)
            _check(load().teno3_mesh_permutation(self.h, p.ctypes.data_as(_ip)))
            self._perm = p
        return self._perm

    def to_internal(self, a):
        return a[self.perm] if isinstance(a, np.ndarray) else a[_torch_index(self.perm, a)]

    def to_user(self, a):
        inv = np.empty_like(self.perm)
        inv[self.perm] = np.arange(self.n_cell, dtype=np.int32)
        return a[inv] if isinstance(a, np.ndarray) else a[_torch_index(inv, a)]

    def boundary_faces(self):
        """(verts [n_bface, 3], cell [n_bface]) of the boundary faces."""
        n = C.c_int32()
        _check(load().teno3_mesh_boundary_count(self.h, C.byref(n)))
        v = np.empty((n.value, 3), dtype=np.int32)
        c = np.empty(n.value, dtype=np.int32)
        _check(load().teno3_mesh_boundary_faces(self.h, v.ctypes.data_as(_ip),
                                                c.ctypes.data_as(_ip)))
        return v, c

    def set_boundary(self, kind):
        """kind: int [n_bface] of BC_TRANSMISSIVE / BC_REFLECTIVE."""
        k = np.ascontiguousarray(kind, dtype=np.int32)
        _check(load().teno3_mesh_set_boundary(self.h, k.ctypes.data_as(_ip)))
        return self

    def stencil(self, cell: int, k: int) -> np.ndarray:
        i = self.info()
        out = np.empty(i.rows_large if k == 4 else i.rows_small, dtype=np.int32)
        _check(load().teno3_mesh_stencil(self.h, int(cell), int(k), out.ctypes.data_as(_ip)))
        return out

    def lsq_operator(self, cell: int, k: int) -> np.ndarray:
        i = self.info()
        rows = i.rows_large if k == 4 else i.rows_small
        nco = i.n_coef_large if k == 4 else i.n_coef_small
        out = np.empty((nco, rows))
        _check(load().teno3_mesh_lsq_operator(self.h, int(cell), int(k),
                                              out.ctypes.data_as(_dp)))
        return out


class TetSolver:
    """Device data of one tetrahedral mesh and the per-stage calls (all
    asynchronous on the given or current stream)."""

    def __init__(self, mesh: TetMesh, device: int = 0):
        if mesh.params is None:
            raise TenoError("call TetMesh.setup() first")
        h = C.c_void_p()
        _check(load().teno3_solver_create(mesh.h, int(device), C.byref(h)))
        self.h = h
        self.mesh = mesh
        self.device = device
        info = mesh.info()
        self.n_cell = info.n_cell
        self.n_pt = info.n_quad
        self.order = info.order

    def __del__(self):
        if getattr(self, "h", None) and _t._lib is not None:
            _t._lib.teno3_solver_destroy(self.h)
            self.h = None

    def _state(self, t, name):
        import torch
        return _ptr(t, (self.n_cell, 5), torch.float64, name)

    def _flags(self, t, n=1, name="flags"):
        import torch
        shape = (self.n_cell,) if n == 1 else (n, self.n_cell)
        return _ptr(t, shape, torch.int32, name, nullable=True)

    def _dt(self, t):
        import torch
        return _ptr(t, (1,), torch.float64, "dt")

    def empty_state(self):
        import torch
        return torch.empty((self.n_cell, 5), dtype=torch.float64, device=f"cuda:{self.device}")

    def empty_flags(self, n=1):
        import torch
        shape = (self.n_cell,) if n == 1 else (n, self.n_cell)
        return torch.zeros(shape, dtype=torch.int32, device=f"cuda:{self.device}")

    def reconstruct(self, U, face_states=None, flags=None, stream=None):
        import torch
        shape = (4 * self.n_pt, self.n_cell, 5)
        if face_states is None:
            face_states = torch.empty(shape, dtype=torch.float64, device=U.device)
        _check(load().teno3_reconstruct(self.h, self._state(U, "U"),
                                        _ptr(face_states, shape, torch.float64, "face_states"),
                                        self._flags(flags), _stream(stream)))
        return face_states

    def residual(self, U, R=None, flags=None, stream=None):
        R = self.empty_state() if R is None else R
        _check(load().teno3_residual(self.h, self._state(U, "U"), self._state(R, "R"),
                                     self._flags(flags), _stream(stream)))
        return R

    def max_dt(self, U, cfl=0.4, dt=None, stream=None):
        import torch
        dt = torch.empty(1, dtype=torch.float64, device=U.device) if dt is None else dt
        _check(load().teno3_max_dt(self.h, self._state(U, "U"), float(cfl), self._dt(dt),
                                   _stream(stream)))
        return dt

    def rk_stage(self, k, Un, Uk, Uk1, dt, flags=None, stream=None):
        _check(load().teno3_rk_stage(self.h, int(k), self._state(Un, "Un"), self._state(Uk, "Uk"),
                                     self._state(Uk1, "Uk1"), self._dt(dt), self._flags(flags),
                                     _stream(stream)))
        return Uk1

    def rk_step(self, U, dt, flags3=None, stream=None):
        _check(load().teno3_rk_step(self.h, self._state(U, "U"), self._dt(dt),
                                    self._flags(flags3, 3, "flags3"), _stream(stream)))
        return U

    def diagnostics(self, reset=False, stream=None) -> dict:
        d = Diag()
        _check(load().teno3_diagnostics(self.h, C.byref(d), 1 if reset else 0, _stream(stream)))
        return {f: getattr(d, f) for f, _ in Diag._fields_}

    def profile_enable(self, kinds=KERNEL_KINDS3):
        bits = sum(1 << KERNEL_KINDS3.index(k) for k in kinds)
        _check(load().teno3_profile_enable(self.h, bits))

    def profile_read(self, reset=True):
        ms = (C.c_double * 3)()
        n = (C.c_int64 * 3)()
        _check(load().teno3_profile_read(self.h, ms, n, 1 if reset else 0))
        return _t.ProfileReading(ms=dict(zip(KERNEL_KINDS3, list(ms))),
                                 launches=dict(zip(KERNEL_KINDS3, list(n))))
