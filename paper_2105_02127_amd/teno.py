"""ctypes binding of libteno (include/teno.h).

Argument marshalling only: every step of the residual runs in the library's
HIP kernels (device) or host set-up code.  PyTorch provides device memory and
the current stream.  Device state tensors are float64 [n_cell, 4] in the
library's internal (Morton) cell order; `Mesh.to_internal` / `to_user` convert.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("TENO_LIB", os.path.join(_HERE, "libteno.so"))
_lib = None


class Params(C.Structure):
    _fields_ = [("order", C.c_int32), ("n_quad", C.c_int32), ("variant", C.c_int32),
                ("power", C.c_int32), ("ct", C.c_double), ("eps", C.c_double),
                ("gamma", C.c_double), ("tie_rel", C.c_double), ("fallback", C.c_int32),
                ("reorder", C.c_int32), ("n_threads", C.c_int32), ("characteristic", C.c_int32),
                ("dk_prime", C.c_double)]


class Info(C.Structure):
    _fields_ = [("n_cell", C.c_int32), ("n_face", C.c_int32), ("order", C.c_int32),
                ("n_quad", C.c_int32), ("n_coef_large", C.c_int32), ("rows_large", C.c_int32),
                ("n_coef_small", C.c_int32), ("rows_small", C.c_int32),
                ("matrix_doubles_per_cell", C.c_int64), ("device_bytes", C.c_int64),
                ("min_rcond", C.c_double), ("face_state_doubles", C.c_int64),
                ("n_bface", C.c_int64)]


class BatchTuning(C.Structure):
    _fields_ = [("order_mode", C.c_int32), ("waves_per_cu", C.c_int32),
                ("item_order", C.c_int32), ("use_graph", C.c_int32)]


class BatchStats(C.Structure):
    _fields_ = [("captures", C.c_int64), ("replays", C.c_int64),
                ("descriptor_writes", C.c_int64)]


class Diag(C.Structure):
    _fields_ = [("nonphysical", C.c_int64), ("first_bad_cell", C.c_int64),
                ("near_ties", C.c_int64), ("fallbacks", C.c_int64)]


# Every exported symbol of include/teno.h with (restype, argtypes).
_vp, _dp, _ip, _i32 = C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_int32
SIGNATURES = {
    "teno_last_error": (C.c_char_p, []),
    "teno_default_params": (None, [C.POINTER(Params)]),
    "teno_mesh_create": (C.c_int, [_i32, _dp, _i32, _ip, _dp, C.POINTER(_vp)]),
    "teno_mesh_setup": (C.c_int, [_vp, C.POINTER(Params)]),
    "teno_mesh_info": (C.c_int, [_vp, C.POINTER(Info)]),
    "teno_mesh_permutation": (C.c_int, [_vp, _ip]),
    "teno_mesh_boundary_count": (C.c_int, [_vp, _ip]),
    "teno_mesh_boundary_faces": (C.c_int, [_vp, _ip, _ip]),
    "teno_mesh_set_boundary": (C.c_int, [_vp, _ip, _dp]),
    "teno_mesh_stencil": (C.c_int, [_vp, _i32, _i32, _ip]),
    "teno_mesh_lsq_operator": (C.c_int, [_vp, _i32, _i32, _dp]),
    "teno_mesh_destroy": (None, [_vp]),
    "teno_solver_create": (C.c_int, [_vp, _i32, C.POINTER(_vp)]),
    "teno_solver_destroy": (None, [_vp]),
    "teno_residual": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "teno_residual_frozen": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "teno_reconstruct": (C.c_int, [_vp, _vp, _vp, _vp, _vp]),
    "teno_max_dt": (C.c_int, [_vp, _vp, C.c_double, _vp, _vp]),
    "teno_max_dt_static": (C.c_int, [_vp, _vp, C.c_double, _vp, _vp]),
    "teno_rk_stage": (C.c_int, [_vp, _i32, _vp, _vp, _vp, _vp, _vp, _i32, _vp]),
    "teno_rk_step": (C.c_int, [_vp, _vp, _vp, _vp, _i32, _vp, _vp, _vp]),
    "teno_rk_step_dt": (C.c_int, [_vp, _vp, _vp, C.c_double, _vp, _vp]),
    "teno_vjp_residual": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "teno_vjp_rk_step": (C.c_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "teno_diagnostics": (C.c_int, [_vp, C.POINTER(Diag), _i32, _vp]),
    "teno_solver_set_boundary_states": (C.c_int, [_vp, _vp, _vp]),
    "teno_profile_enable": (C.c_int, [_vp, _i32]),
    "teno_profile_read": (C.c_int, [_vp, _dp, C.POINTER(C.c_int64), _i32]),
    "teno_batch_create": (C.c_int, [C.POINTER(_vp), _i32, C.POINTER(_vp)]),
    "teno_batch_set_tuning": (C.c_int, [_vp, C.POINTER(BatchTuning)]),
    "teno_batch_get_tuning": (C.c_int, [_vp, C.POINTER(BatchTuning)]),
    "teno_batch_max_dt": (C.c_int, [_vp, C.POINTER(_vp), C.c_double, _vp, _vp]),
    "teno_batch_rk_step": (C.c_int, [_vp, C.POINTER(_vp), _vp, _vp]),
    "teno_batch_set_flags": (C.c_int, [_vp, C.POINTER(_vp)]),
    "teno_batch_get_stats": (C.c_int, [_vp, C.POINTER(BatchStats)]),
    "teno_batch_destroy": (None, [_vp]),
}

KERNEL_KINDS = ("reconstruct", "flux_update", "dt", "adjoint")


class TenoError(RuntimeError):
    pass


def load():
    """Load libteno.so (raises if it has not been built).

    torch is imported first: its wheel carries its own HIP runtime with the
    same SONAME as the system one, so loading torch's copy first makes
    libteno bind to it and the process keeps a single HIP/HSA runtime (two
    runtimes in one process cannot share the device)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (must precede the CDLL, see above)
        if not os.path.exists(LIB_PATH):
            raise TenoError(f"{LIB_PATH} not found: build it with `python -m paper_2105_02127_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc is not None and rc < 0:
        raise TenoError(f"libteno error {rc}: {load().teno_last_error().decode()}")
    return rc


def default_params(**kw) -> Params:
    """The library's defaults with `kw` applied.  For the CWENO variant
    (variant=2) power and eps default to the paper's CWENO values, 4 and
    1e-14 (Sec. 2.4)."""
    p = Params()
    load().teno_default_params(C.byref(p))
    if kw.get("variant") == 2:
        kw.setdefault("power", 4)
        kw.setdefault("eps", 1e-14)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k}")
        setattr(p, k, v)
    return p


def _stream(stream):
    if stream is not None:
        return C.c_void_p(stream)
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t, shape=None, dtype=None, name="tensor", nullable=False):
    if t is None:
        if nullable:
            return None
        raise TenoError(f"{name} is required")
    import torch
    if not isinstance(t, torch.Tensor):
        raise TenoError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise TenoError(f"{name} must live on the GPU")
    if dtype is not None and t.dtype != dtype:
        raise TenoError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise TenoError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise TenoError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return C.c_void_p(t.data_ptr())


# boundary-condition kinds (teno_bc)
BC_TRANSMISSIVE, BC_REFLECTIVE, BC_PRESCRIBED = 1, 2, 3


class Mesh:
    """Triangle mesh plus (after `setup`) stencils and operators.  period:
    the period of each axis, 0 for an open axis (None: both open)."""

    def __init__(self, xy, tri, period=(1.0, 1.0)):
        L = load()
        xy = np.ascontiguousarray(xy, dtype=np.float64)
        tri = np.ascontiguousarray(tri, dtype=np.int32)
        per = None if period is None else np.ascontiguousarray(period, dtype=np.float64)
        h = C.c_void_p()
        _check(L.teno_mesh_create(xy.shape[0], xy.ctypes.data_as(_dp), tri.shape[0],
                                  tri.ctypes.data_as(_ip),
                                  None if per is None else per.ctypes.data_as(_dp), C.byref(h)))
        self.h = h
        self.n_cell = int(tri.shape[0])
        self.params = None
        self._perm = None

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.teno_mesh_destroy(self.h)
            self.h = None

    def setup(self, **kw):
        p = default_params(**kw)
        _check(load().teno_mesh_setup(self.h, C.byref(p)))
        self.params = p
        self._perm = None
        return self

    def info(self) -> Info:
        i = Info()
        _check(load().teno_mesh_info(self.h, C.byref(i)))
        return i

    @property
    def perm(self) -> np.ndarray:
        """perm[internal] = user cell id."""
        if self._perm is None:
            p = np.empty(self.n_cell, dtype=np.int32)
            _check(load().teno_mesh_permutation(self.h, p.ctypes.data_as(_ip)))
            self._perm = p
        return self._perm

    def to_internal(self, a):
        return a[self.perm] if isinstance(a, np.ndarray) else a[_torch_index(self.perm, a)]

    def to_user(self, a):
        inv = np.empty_like(self.perm)
        inv[self.perm] = np.arange(self.n_cell, dtype=np.int32)
        return a[inv] if isinstance(a, np.ndarray) else a[_torch_index(inv, a)]

    def stencil(self, cell: int, k: int) -> np.ndarray:
        i = self.info()
        n = i.rows_large if k == 3 else i.rows_small
        out = np.empty(n, dtype=np.int32)
        _check(load().teno_mesh_stencil(self.h, int(cell), int(k), out.ctypes.data_as(_ip)))
        return out

    def boundary_faces(self):
        """(verts [n_bface, 2], cell [n_bface]) of the boundary faces."""
        n = C.c_int32()
        _check(load().teno_mesh_boundary_count(self.h, C.byref(n)))
        v = np.empty((n.value, 2), dtype=np.int32)
        c = np.empty(n.value, dtype=np.int32)
        _check(load().teno_mesh_boundary_faces(self.h, v.ctypes.data_as(_ip), c.ctypes.data_as(_ip)))
        return v, c

    def set_boundary(self, kind, state=None):
        """kind: int [n_bface] of BC_*; state: [n_bface, 4] for prescribed faces."""
        k = np.ascontiguousarray(kind, dtype=np.int32)
        st = None if state is None else np.ascontiguousarray(state, dtype=np.float64)
        _check(load().teno_mesh_set_boundary(self.h, k.ctypes.data_as(_ip),
                                             None if st is None else st.ctypes.data_as(_dp)))
        return self

    def lsq_operator(self, cell: int, k: int) -> np.ndarray:
        i = self.info()
        rows = i.rows_large if k == 3 else i.rows_small
        nco = i.n_coef_large if k == 3 else i.n_coef_small
        out = np.empty((nco, rows))
        _check(load().teno_mesh_lsq_operator(self.h, int(cell), int(k), out.ctypes.data_as(_dp)))
        return out


def _torch_index(idx, like):
    import torch
    return torch.as_tensor(idx.astype(np.int64), device=like.device)


@dataclass
class ProfileReading:
    ms: dict
    launches: dict


class Solver:
    """Device data of one mesh and the per-stage calls (all asynchronous)."""

    def __init__(self, mesh: Mesh, device: int = 0):
        if mesh.params is None:
            raise TenoError("call Mesh.setup() first")
        h = C.c_void_p()
        _check(load().teno_solver_create(mesh.h, int(device), C.byref(h)))
        self.h = h
        self.mesh = mesh
        self.device = device
        info = mesh.info()
        self.n_cell = info.n_cell
        self.n_quad = info.n_quad
        self.order = info.order
        self.face_state_doubles = int(info.face_state_doubles)
        # flag words per cell: one, or one per local edge in characteristic
        # variables
        self.flag_words = 3 if mesh.params.characteristic else 1

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.teno_solver_destroy(self.h)
            self.h = None

    # -- helpers --
    def _state(self, t, name, nullable=False):
        import torch
        return _ptr(t, (self.n_cell, 4), torch.float64, name, nullable)

    def _flag_shape(self, n):
        base = (self.n_cell,) if self.flag_words == 1 else (self.flag_words, self.n_cell)
        return base if n == 1 else (n,) + base

    def _flags(self, t, n=1, name="flags", nullable=True):
        import torch
        # uint16 bit patterns carried in int16 tensors (view as uint16 on the host)
        return _ptr(t, self._flag_shape(n), torch.int16, name, nullable)

    def _dt(self, t):
        import torch
        return _ptr(t, (1,), torch.float64, "dt")

    def empty_state(self):
        import torch
        return torch.empty((self.n_cell, 4), dtype=torch.float64, device=f"cuda:{self.device}")

    def empty_flags(self, n=1):
        import torch
        return torch.zeros(self._flag_shape(n), dtype=torch.int16, device=f"cuda:{self.device}")

    # -- calls --
    def residual(self, U, R=None, flags=None, stream=None):
        R = self.empty_state() if R is None else R
        _check(load().teno_residual(self.h, self._state(U, "U"), self._state(R, "R"),
                                    self._flags(flags), _stream(stream)))
        return R

    def residual_frozen(self, U, flags, R=None, stream=None):
        R = self.empty_state() if R is None else R
        _check(load().teno_residual_frozen(self.h, self._state(U, "U"), self._state(R, "R"),
                                           self._flags(flags, nullable=False), _stream(stream)))
        return R

    def reconstruct(self, U, face_states=None, flags=None, stream=None):
        import torch
        if face_states is None:
            face_states = torch.empty((3 * self.n_quad, self.n_cell, 4), dtype=torch.float64,
                                      device=U.device)
        _check(load().teno_reconstruct(
            self.h, self._state(U, "U"),
            _ptr(face_states, (3 * self.n_quad, self.n_cell, 4), torch.float64, "face_states"),
            self._flags(flags), _stream(stream)))
        return face_states

    def max_dt(self, U, cfl=0.4, dt=None, stream=None):
        import torch
        dt = torch.empty(1, dtype=torch.float64, device=U.device) if dt is None else dt
        _check(load().teno_max_dt(self.h, self._state(U, "U"), float(cfl), self._dt(dt),
                                  _stream(stream)))
        return dt

    def rk_stage(self, k, Un, Uk, Uk1, dt, flags=None, frozen=False, stream=None):
        _check(load().teno_rk_stage(self.h, int(k), self._state(Un, "Un"), self._state(Uk, "Uk"),
                                    self._state(Uk1, "Uk1"), self._dt(dt), self._flags(flags),
                                    1 if frozen else 0, _stream(stream)))
        return Uk1

    def empty_face_states(self, n_steps=None):
        """Buffer for the face states rk_step can keep for vjp_rk_step:
        [3, face_state_doubles] float64 (or [n_steps, 3, ...])."""
        import torch
        shape = (3, self.face_state_doubles) if n_steps is None else \
            (n_steps, 3, self.face_state_doubles)
        return torch.empty(shape, dtype=torch.float64, device=f"cuda:{self.device}")

    def _face_states(self, t):
        import torch
        return _ptr(t, (3, self.face_state_doubles), torch.float64, "face_states", True)

    def rk_step(self, U, dt, flags3=None, frozen=False, stages=None, face_states=None,
                stream=None):
        import torch
        st = None if stages is None else _ptr(stages, (3, self.n_cell, 4), torch.float64, "stages")
        _check(load().teno_rk_step(self.h, self._state(U, "U"), self._dt(dt),
                                   self._flags(flags3, 3, "flags3"), 1 if frozen else 0, st,
                                   self._face_states(face_states), _stream(stream)))
        return U

    def rk_step_dt(self, U, dt, cfl=0.4, flags3=None, stream=None):
        """One SSP-RK3 step in place with dt; dt then holds the next step's
        CFL step (teno_rk_step_dt)."""
        _check(load().teno_rk_step_dt(self.h, self._state(U, "U"), self._dt(dt), float(cfl),
                                      self._flags(flags3, 3, "flags3"), _stream(stream)))
        return U

    def vjp_residual(self, U, flags, lam, U_bar=None, stream=None):
        U_bar = self.empty_state() if U_bar is None else U_bar
        _check(load().teno_vjp_residual(self.h, self._state(U, "U"),
                                        self._flags(flags, nullable=False),
                                        self._state(lam, "lam"), self._state(U_bar, "U_bar"),
                                        _stream(stream)))
        return U_bar

    def vjp_rk_step(self, stages, flags3, dt, lam_out, lam_in=None, face_states=None,
                    stream=None):
        import torch
        lam_in = self.empty_state() if lam_in is None else lam_in
        _check(load().teno_vjp_rk_step(
            self.h, _ptr(stages, (3, self.n_cell, 4), torch.float64, "stages"),
            self._flags(flags3, 3, "flags3", nullable=False), self._face_states(face_states),
            self._dt(dt), self._state(lam_out, "lam_out"), self._state(lam_in, "lam_in"),
            _stream(stream)))
        return lam_in

    def set_boundary_states(self, state, stream=None):
        """Replaces the prescribed boundary states: device float64 [n_bface, 4]."""
        import torch
        n = int(self.mesh.info().n_bface)
        _check(load().teno_solver_set_boundary_states(
            self.h, _ptr(state, (n, 4), torch.float64, "state"), _stream(stream)))

    def diagnostics(self, reset=False, stream=None) -> dict:
        d = Diag()
        _check(load().teno_diagnostics(self.h, C.byref(d), 1 if reset else 0, _stream(stream)))
        return {k: int(getattr(d, k)) for k, _ in Diag._fields_}

    def profile_enable(self, on=True, kinds=None):
        """Times the launches of `kinds` (names from KERNEL_KINDS; all when
        None) with HIP events while `on`."""
        if not on:
            mask = 0
        elif kinds is None:
            mask = 0xF
        else:
            mask = 0
            for k in kinds:
                mask |= 1 << KERNEL_KINDS.index(k)
        _check(load().teno_profile_enable(self.h, mask))

    def profile_read(self, reset=True) -> ProfileReading:
        ms = (C.c_double * 4)()
        n = (C.c_int64 * 4)()
        _check(load().teno_profile_read(self.h, ms, n, 1 if reset else 0))
        return ProfileReading(ms={k: ms[i] for i, k in enumerate(KERNEL_KINDS)},
                              launches={k: n[i] for i, k in enumerate(KERNEL_KINDS)})
