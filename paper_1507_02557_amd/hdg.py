"""Thin ctypes binding of the C ABI in include/hdg.h.

Argument marshalling only: every computation runs in the HIP library
``libhdg.so`` built in-tree by ``paper_1507_02557_amd.build``.  PyTorch supplies
device memory and the current stream.  Loading fails loudly if the library is
missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HEX, WEDGE, PYR, TET = 0, 1, 2, 3
BC_FREE_SURFACE, BC_RIGID_WALL = 0, 1
PREC_FP32, PREC_FP16X2, PREC_FP16X2_K16, PREC_BF16X2, PREC_BF16X3 = 0, 1, 2, 3, 4
PATH_AUTO, PATH_GENERIC = 0, 1
DT_REFERENCE, DT_ELEMENT = 0, 1
STEPPER_LSERK4, STEPPER_MRAB3 = 0, 1
PROJECT_SCRATCH_BYTES = 16 * 1024 * 1024  # HDG_PROJECT_SCRATCH_BYTES
OK, EINVAL, EMESH, ENOMEM, EHIP, ENONFINITE, ESTATE = 0, -1, -2, -3, -4, -5, -6

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhdg.so")

# (name, restype, argtypes) of every exported symbol
_P = ctypes.c_void_p
_SIGS = [
    ("hdg_create", ctypes.c_int, [ctypes.POINTER(_P), _P, ctypes.c_int, ctypes.c_int, _P]),
    ("hdg_destroy", None, [_P]),
    ("hdg_last_error", ctypes.c_char_p, [_P]),
    ("hdg_type_info", ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    ("hdg_dt", ctypes.c_int, [_P, ctypes.c_double, _P, ctypes.POINTER(ctypes.c_double)]),
    ("hdg_get_points", ctypes.c_int, [_P, ctypes.c_int, _P]),
    ("hdg_project", ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P]),
    ("hdg_project_noalloc", ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P]),
    ("hdg_set_state", ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P, _P]),
    ("hdg_get_field", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P, _P, _P, _P]),
    ("hdg_rhs", ctypes.c_int, [_P]),
    ("hdg_step", ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int64]),
    ("hdg_energy", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    ("hdg_get_time", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    ("hdg_set_time", ctypes.c_int, [_P, ctypes.c_double]),
    ("hdg_check_finite", ctypes.c_int, [_P]),
    ("hdg_advance", ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int64,
                                   ctypes.POINTER(ctypes.c_int64)]),
    ("hdg_checkpoint_size", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64)]),
    ("hdg_checkpoint_save", ctypes.c_int, [_P, _P, ctypes.c_int64]),
    ("hdg_checkpoint_load", ctypes.c_int, [_P, _P, ctypes.c_int64]),
    ("hdg_mrab_setup", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_double), _P, _P]),
    ("hdg_mrab_advance", ctypes.c_int, [_P, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]),
    ("hdg_mrab_level_info", ctypes.c_int, [_P, _P]),
    ("hdg_trace_constants", ctypes.c_int, [_P, _P]),
    ("hdg_step_graph", ctypes.c_int, [_P, ctypes.c_double, ctypes.c_int64]),
    ("hdg_autotune", ctypes.c_int, [_P, ctypes.c_int, _P]),
    ("hdg_set_dt_mode", ctypes.c_int, [_P, ctypes.c_int]),
    ("hdg_profile", ctypes.c_int, [_P, ctypes.c_int]),
    ("hdg_profile_read", ctypes.c_int, [_P, _P, _P]),
    ("hdg_set_path", ctypes.c_int, [_P, ctypes.c_int]),
    ("hdg_get_path", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
]
EXPORTS = [s[0] for s in _SIGS]


class HdgMesh(ctypes.Structure):
    _fields_ = [("n_vert", ctypes.c_int64), ("xyz", _P), ("n_elem", ctypes.c_int64), ("type", _P),
                ("verts", _P), ("kappa", _P), ("rho", _P), ("bc", ctypes.c_int32), ("bc_face", _P),
                ("n_hanging", ctypes.c_int64), ("hanging", _P)]


class HdgError(RuntimeError):
    def __init__(self, msg: str, code: int = 0):
        super().__init__(msg)
        self.code = code


_LIBS: dict = {}


def load_library(path: str | None = None) -> ctypes.CDLL:
    path = path or LIB_PATH
    if path in _LIBS:
        return _LIBS[path]
    if not os.path.exists(path):
        raise HdgError(f"HIP library not built: {path} (run paper_1507_02557_amd.build)")
    lib = ctypes.CDLL(path)
    for name, res, args in _SIGS:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIBS[path] = lib
    return lib


def _ptr(t: torch.Tensor) -> int:
    if not t.is_contiguous():
        raise HdgError("tensor must be contiguous")
    return t.data_ptr()


class Solver:
    """One solver context (mesh, order N) on one device.

    ``device`` is the torch device whose memory the library addresses; the
    HIP library requires a CUDA (HIP) device.
    """

    def __init__(self, mesh, N: int, bc: int = BC_RIGID_WALL, precision: int = PREC_FP32,
                 device: str | torch.device = "cuda", lib_path: str | None = None, path: int = PATH_AUTO):
        self.device = torch.device(device)
        self._lib = load_library(lib_path)
        if lib_path is None and (self.device.type != "cuda" or not torch.cuda.is_available()):
            raise HdgError("the HIP library needs a GPU device; none is available")
        self.N = N
        xyz = np.ascontiguousarray(mesh.xyz, dtype=np.float64)
        et = np.ascontiguousarray(mesh.etype, dtype=np.int8)
        ev = np.ascontiguousarray(mesh.everts, dtype=np.int64)
        ka = np.ascontiguousarray(mesh.kappa, dtype=np.float64)
        rh = np.ascontiguousarray(mesh.rho, dtype=np.float64)
        hg = np.ascontiguousarray(getattr(mesh, "hanging", np.zeros((0, 3))), dtype=np.int64).reshape(-1, 3)
        bf = getattr(mesh, "bc_face", None)
        bf = None if bf is None else np.ascontiguousarray(bf, dtype=np.int8).reshape(et.shape[0], 6)
        m = HdgMesh(xyz.shape[0], xyz.ctypes.data, et.shape[0], et.ctypes.data, ev.ctypes.data,
                    ka.ctypes.data, rh.ctypes.data, bc, None if bf is None else bf.ctypes.data,
                    hg.shape[0], hg.ctypes.data if hg.shape[0] else None)
        h = _P()
        rc = self._lib.hdg_create(ctypes.byref(h), ctypes.byref(m), N, precision, self._stream())
        if rc != 0:
            raise HdgError(f"hdg_create failed ({rc}): {self._lib.hdg_last_error(None).decode()}")
        self._h = h
        self.n_elem = et.shape[0]
        self.info = {}
        for t in (HEX, WEDGE, PYR, TET):
            K, Np, ns = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
            self._check(self._lib.hdg_type_info(h, t, ctypes.byref(K), ctypes.byref(Np), ctypes.byref(ns)))
            self.info[t] = (K.value, Np.value, ns.value)
        self.types = [t for t in (HEX, WEDGE, PYR, TET) if self.info[t][0] > 0]
        if path != PATH_AUTO:
            self.set_path(path)

    def _stream(self):
        if self.device.type == "cuda":
            return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        return None

    def _check(self, rc: int):
        if rc != 0:
            raise HdgError(f"hdg call failed ({rc}): {self._lib.hdg_last_error(self._h).decode()}", rc)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hdg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------
    def dt(self, cfl: float = 0.5):
        out = np.zeros(self.n_elem, dtype=np.float64)
        mn = ctypes.c_double()
        self._check(self._lib.hdg_dt(self._h, cfl, out.ctypes.data, ctypes.byref(mn)))
        return out, mn.value

    def points(self, t: int) -> torch.Tensor:
        K, _, ns = self.info[t]
        x = torch.empty((K, ns, 3), dtype=torch.float64, device=self.device)
        self._check(self._lib.hdg_get_points(self._h, t, _ptr(x)))
        return x

    def project(self, t: int, fields):
        f = [torch.as_tensor(v, dtype=torch.float64, device=self.device).contiguous() for v in fields]
        self._check(self._lib.hdg_project(self._h, t, *[_ptr(v) for v in f]))
        if self.device.type == "cuda":
            torch.cuda.current_stream(self.device).synchronize()

    def project_noalloc(self, t: int, fields):
        """hdg_project through the library's fixed work buffer (no device allocation, no sync)."""
        f = [torch.as_tensor(v, dtype=torch.float64, device=self.device).contiguous() for v in fields]
        self._check(self._lib.hdg_project_noalloc(self._h, t, *[_ptr(v) for v in f]))
        if self.device.type == "cuda":
            torch.cuda.current_stream(self.device).synchronize()

    def set_state(self, t: int, fields):
        f = [torch.as_tensor(v, dtype=torch.float32, device=self.device).contiguous() for v in fields]
        self._check(self._lib.hdg_set_state(self._h, t, *[_ptr(v) for v in f]))
        if self.device.type == "cuda":
            torch.cuda.current_stream(self.device).synchronize()

    def get_field(self, t: int, which: int = 0):
        K, Np, _ = self.info[t]
        out = [torch.empty((K, Np), dtype=torch.float32, device=self.device) for _ in range(4)]
        self._check(self._lib.hdg_get_field(self._h, which, t, *[_ptr(v) for v in out]))
        return torch.stack(out, 1)  # (K, 4, Np)

    def state(self):
        return {t: self.get_field(t, 0) for t in self.types}

    def rhs(self):
        self._check(self._lib.hdg_rhs(self._h))
        return {t: self.get_field(t, 1) for t in self.types}

    def step(self, dt: float, n_steps: int = 1):
        self._check(self._lib.hdg_step(self._h, float(dt), int(n_steps)))

    def step_graph(self, dt: float, n_steps: int):
        """n_steps LSERK4 steps replayed from a captured HIP graph (bitwise those of step)."""
        self._check(self._lib.hdg_step_graph(self._h, float(dt), int(n_steps)))

    def autotune(self, reps: int = 5):
        """Time every batch size of the hexahedron and wedge block kernels on this
        mesh and keep the fastest; returns the chosen elements per block per type
        (0: not tuned).  Overwrites the right-hand-side buffer."""
        out = (ctypes.c_int32 * 4)()
        self._check(self._lib.hdg_autotune(self._h, int(reps), ctypes.cast(out, ctypes.c_void_p)))
        return [int(v) for v in out]

    def energy(self) -> float:
        E = ctypes.c_double()
        self._check(self._lib.hdg_energy(self._h, ctypes.byref(E)))
        return E.value

    @property
    def time(self) -> float:
        t = ctypes.c_double()
        self._check(self._lib.hdg_get_time(self._h, ctypes.byref(t)))
        return t.value

    @time.setter
    def time(self, t: float):
        self._check(self._lib.hdg_set_time(self._h, float(t)))

    def check_finite(self):
        self._check(self._lib.hdg_check_finite(self._h))

    def advance(self, t_final: float, stepper: int = STEPPER_LSERK4, cfl: float = 0.5,
                check_every: int = 0) -> int:
        """Advance to t_final (step shortened to divide the interval); returns the steps taken."""
        n = ctypes.c_int64()
        rc = self._lib.hdg_advance(self._h, float(t_final), int(stepper), float(cfl), int(check_every),
                                   ctypes.byref(n))
        self.steps_done = n.value
        self._check(rc)
        return n.value

    def checkpoint(self) -> np.ndarray:
        """Checkpoint (time, state, multi-rate history) as a host byte array."""
        b = ctypes.c_int64()
        self._check(self._lib.hdg_checkpoint_size(self._h, ctypes.byref(b)))
        buf = np.empty(b.value, dtype=np.uint8)
        self._check(self._lib.hdg_checkpoint_save(self._h, buf.ctypes.data, b.value))
        return buf

    def restore(self, buf: np.ndarray):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self._lib.hdg_checkpoint_load(self._h, buf.ctypes.data, buf.size))

    def mrab_setup(self, n_levels: int, cfl: float = 0.5):
        """Multi-rate levels; returns (dt_min, elements per level, level per element)."""
        mn = ctypes.c_double()
        cnt = np.zeros(n_levels, dtype=np.int64)
        lev = np.zeros(self.n_elem, dtype=np.int8)
        self._check(self._lib.hdg_mrab_setup(self._h, n_levels, cfl, ctypes.byref(mn), cnt.ctypes.data,
                                             lev.ctypes.data))
        return mn.value, cnt, lev

    def trace_constants(self):
        """Per-element computed trace constants C_T(N, K) (n_elem,), mesh order."""
        out = np.zeros(self.n_elem, dtype=np.float64)
        self._check(self._lib.hdg_trace_constants(self._h, out.ctypes.data))
        return out

    def set_dt_mode(self, mode: int):
        """DT_REFERENCE (C_T(N) C_J^K) or DT_ELEMENT (per-element C_T(N, K))."""
        self._check(self._lib.hdg_set_dt_mode(self._h, int(mode)))

    def mrab_level_info(self, n_levels: int):
        """(4, n_levels, 2) int64: per type and level, the element count and the
        number of those that write mid-step traces."""
        out = np.zeros((4, n_levels, 2), dtype=np.int64)
        self._check(self._lib.hdg_mrab_level_info(self._h, out.ctypes.data))
        return out

    def mrab_advance(self, n_coarse: int) -> float:
        t = ctypes.c_double()
        self._check(self._lib.hdg_mrab_advance(self._h, int(n_coarse), ctypes.byref(t)))
        return t.value

    def profile(self, on: bool):
        self._check(self._lib.hdg_profile(self._h, 1 if on else 0))

    def set_path(self, path: int):
        self._check(self._lib.hdg_set_path(self._h, path))

    def get_path(self):
        """(requested path, 1 if lattice traces are in use else 0)."""
        p, lat = ctypes.c_int(), ctypes.c_int()
        self._check(self._lib.hdg_get_path(self._h, ctypes.byref(p), ctypes.byref(lat)))
        return p.value, lat.value

    def profile_read(self):
        """Kernel milliseconds and launch counts since the last reset, each (3, 4):
        [kind][type], kind 0 stage / right-hand side, 1 multi-rate update,
        2 non-conforming interface (type TET)."""
        ms = np.zeros(12, dtype=np.float64)
        cnt = np.zeros(12, dtype=np.int64)
        self._check(self._lib.hdg_profile_read(self._h, ms.ctypes.data, cnt.ctypes.data))
        return ms.reshape(3, 4), cnt.reshape(3, 4)

    def project_function(self, func, time: float = 0.0):
        """Sample func(x, y, z, t) -> (p, ux, uy, uz) at each type's points and project."""
        for t in self.types:
            x = self.points(t)
            vals = func(x[..., 0], x[..., 1], x[..., 2], time)
            self.project(t, [v.reshape(x.shape[0], -1) for v in vals])
