"""ctypes binding of the C ABI in ``include/esdg.h`` (argument marshalling only).

Every step of the method runs in the HIP library ``lib/libesdg.so``; this
module only converts arguments.  Device memory is supplied by torch tensors
(float64, contiguous, on the library's device) and the stream is torch's
current stream unless another one is given.  There is no CPU fallback: if
the library is missing the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libesdg.so")

OK, EINVAL, ENOMEM, EDEVICE, ENONPHYSICAL, ESTATE = 0, -1, -2, -3, -4, -5
FLUX = {"ranocha": 0, "shima": 1, "llf": 2, "central": 3}
PRECISION = {"fp64": 0, "fp32": 1}
HOST, DEVICE = 0, 1
KERNEL_STAGE, KERNEL_REDUCE = 1, 2
PMAX = 7


class EsdgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("esdg status %d: %s" % (status, message))
        self.status = status


class NonPhysicalState(EsdgError):
    pass


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("p", C.c_int32), ("n", C.c_int32 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("warp", C.c_double),
                ("coords", C.POINTER(C.c_double)), ("gamma", C.c_double),
                ("volume_flux", C.c_int32), ("surface_flux", C.c_int32),
                ("precision", C.c_int32), ("stream", C.c_void_p)]


_lib = None
_lock = threading.Lock()

EXPORTS = ["esdg_init_mesh", "esdg_destroy", "esdg_sizes", "esdg_set_stream", "esdg_get_coords",
           "esdg_set_state", "esdg_get_state", "esdg_rhs", "esdg_step", "esdg_entropy_rate",
           "esdg_totals", "esdg_max_dt", "esdg_sync", "esdg_timing_enable", "esdg_timing_read",
           "esdg_timing_reset", "esdg_operators", "esdg_last_error", "esdg_version"]


def load_library(path: str | None = None):
    """Load libesdg.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is not None and path is None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise RuntimeError("HIP library %s is not built: run __graft_entry__.build() or "
                               "python -m paper_2112_10517_amd.build" % p)
        # Share the process's HIP runtime with torch: importing torch first
        # makes its libamdhip64.so.7 the one this library binds to, so device
        # memory and streams handed over from torch are the same runtime's.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = C.CDLL(p)
        vp, dp, st = C.c_void_p, C.POINTER(C.c_double), C.c_int
        lib.esdg_init_mesh.argtypes = [C.POINTER(MeshDesc), C.POINTER(vp)]
        lib.esdg_destroy.argtypes = [vp]
        lib.esdg_destroy.restype = None
        lib.esdg_sizes.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        lib.esdg_set_stream.argtypes = [vp, vp]
        lib.esdg_get_coords.argtypes = [vp, dp]
        lib.esdg_set_state.argtypes = [vp, vp, C.c_int32]
        lib.esdg_get_state.argtypes = [vp, vp, C.c_int32]
        lib.esdg_rhs.argtypes = [vp, vp, C.c_int32]
        lib.esdg_step.argtypes = [vp, C.c_double, C.c_int32, C.c_double, dp]
        lib.esdg_entropy_rate.argtypes = [vp, dp]
        lib.esdg_totals.argtypes = [vp, dp]
        lib.esdg_max_dt.argtypes = [vp, C.c_double, dp]
        lib.esdg_sync.argtypes = [vp]
        lib.esdg_timing_enable.argtypes = [vp, C.c_int32]
        lib.esdg_timing_read.argtypes = [vp, C.c_int32, dp, C.POINTER(C.c_int64)]
        lib.esdg_timing_reset.argtypes = [vp]
        lib.esdg_last_error.argtypes = [vp]
        lib.esdg_last_error.restype = C.c_char_p
        lib.esdg_operators.argtypes = [C.c_int32, dp, dp, dp, dp]
        lib.esdg_version.argtypes = []
        lib.esdg_version.restype = C.c_char_p
        for name in EXPORTS:
            if name not in ("esdg_destroy", "esdg_last_error", "esdg_version"):
                getattr(lib, name).restype = st
        if path is None:
            _lib = lib
        return lib


def _check(lib, handle, status: int):
    if status != OK:
        msg = lib.esdg_last_error(handle)
        msg = msg.decode() if msg else ""
        cls = NonPhysicalState if status == ENONPHYSICAL else EsdgError
        raise cls(status, msg)


def _torch():
    import torch
    return torch


def _where_ptr(arr, shape, writable: bool):
    """(pointer, where, keepalive) for a numpy array or a CUDA/HIP torch tensor."""
    if isinstance(arr, np.ndarray):
        if arr.dtype != np.float64 or not arr.flags["C_CONTIGUOUS"] or arr.shape != shape:
            raise ValueError("expected a C-contiguous float64 array of shape %s" % (shape,))
        if writable and not arr.flags["WRITEABLE"]:
            raise ValueError("output array is read-only")
        return C.c_void_p(arr.ctypes.data), HOST, arr
    torch = _torch()
    if isinstance(arr, torch.Tensor):
        if arr.dtype != torch.float64 or not arr.is_contiguous() or tuple(arr.shape) != shape:
            raise ValueError("expected a contiguous float64 tensor of shape %s" % (shape,))
        if arr.is_cuda:
            return C.c_void_p(arr.data_ptr()), DEVICE, arr
        return C.c_void_p(arr.data_ptr()), HOST, arr
    raise TypeError("expected numpy.ndarray or torch.Tensor")


class Problem:
    """One periodic Euler problem on the GPU (handle of ``esdg_init_mesh``)."""

    def __init__(self, dim: int, p: int, n, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0),
                 warp: float = 0.0, gamma: float = 1.4, volume_flux: str = "ranocha",
                 surface_flux: str = "llf", precision: str = "fp64", coords=None, stream=None):
        self._lib = load_library()
        d = MeshDesc()
        d.dim, d.p = dim, p
        n = list(n) + [1] * (3 - len(n))
        lo = list(lo) + [0.0] * (3 - len(lo))
        hi = list(hi) + [1.0] * (3 - len(hi))
        for j in range(3):
            d.n[j], d.lo[j], d.hi[j] = int(n[j]), float(lo[j]), float(hi[j])
        d.warp, d.gamma = float(warp), float(gamma)
        d.volume_flux = FLUX[volume_flux] if isinstance(volume_flux, str) else int(volume_flux)
        d.surface_flux = FLUX[surface_flux] if isinstance(surface_flux, str) else int(surface_flux)
        d.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
        keep = None
        if coords is not None:
            keep = np.ascontiguousarray(coords, dtype=np.float64)
            d.coords = keep.ctypes.data_as(C.POINTER(C.c_double))
        d.stream = self._stream_ptr(stream)
        h = C.c_void_p()
        st = self._lib.esdg_init_mesh(C.byref(d), C.byref(h))
        _check(self._lib, None, st)
        self._h = h
        ne, nn, nv = C.c_int64(), C.c_int32(), C.c_int32()
        _check(self._lib, h, self._lib.esdg_sizes(h, C.byref(ne), C.byref(nn), C.byref(nv)))
        self.dim, self.p, self.N = dim, p, p + 1
        self.n_elem, self.nodes, self.n_var = ne.value, nn.value, nv.value
        self.shape = (self.n_elem, self.n_var, self.nodes)
        self.n_dof = self.n_elem * self.nodes

    @staticmethod
    def _stream_ptr(stream):
        if stream is None:
            try:
                torch = _torch()
                if torch.cuda.is_available():
                    return C.c_void_p(torch.cuda.current_stream().cuda_stream)
            except ImportError:
                pass
            return None
        if isinstance(stream, int):
            return C.c_void_p(stream)
        return C.c_void_p(stream.cuda_stream)

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.esdg_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _call(self, fn, *args):
        _check(self._lib, self._h, fn(self._h, *args))

    def set_stream(self, stream):
        self._call(self._lib.esdg_set_stream, self._stream_ptr(stream))

    def coords(self) -> np.ndarray:
        x = np.zeros((self.n_elem, self.dim, self.nodes))
        self._call(self._lib.esdg_get_coords, x.ctypes.data_as(C.POINTER(C.c_double)))
        return x

    def set_state(self, u):
        ptr, where, _keep = _where_ptr(u, self.shape, False)
        self._call(self._lib.esdg_set_state, ptr, where)

    def get_state(self, out=None):
        out = np.empty(self.shape) if out is None else out
        ptr, where, _keep = _where_ptr(out, self.shape, True)
        self._call(self._lib.esdg_get_state, ptr, where)
        return out

    def rhs(self, out=None):
        out = np.empty(self.shape) if out is None else out
        ptr, where, _keep = _where_ptr(out, self.shape, True)
        self._call(self._lib.esdg_rhs, ptr, where)
        return out

    def step(self, dt: float = 0.0, nsteps: int = 1, cfl: float = 0.0, t: float | None = None):
        """Advance nsteps RK4 steps; returns the new time if t is given."""
        tt = C.c_double(0.0 if t is None else t)
        self._call(self._lib.esdg_step, float(dt), int(nsteps), float(cfl),
                   C.byref(tt) if t is not None else None)
        return tt.value if t is not None else None

    def entropy_rate(self) -> float:
        r = C.c_double()
        self._call(self._lib.esdg_entropy_rate, C.byref(r))
        return r.value

    def totals(self) -> np.ndarray:
        t = np.zeros(self.n_var)
        self._call(self._lib.esdg_totals, t.ctypes.data_as(C.POINTER(C.c_double)))
        return t

    def max_dt(self, cfl: float) -> float:
        r = C.c_double()
        self._call(self._lib.esdg_max_dt, float(cfl), C.byref(r))
        return r.value

    def sync(self):
        self._call(self._lib.esdg_sync)

    def timing(self, enable: bool):
        self._call(self._lib.esdg_timing_enable, 1 if enable else 0)

    def timing_read(self, kernel: int):
        ms, cnt = C.c_double(), C.c_int64()
        self._call(self._lib.esdg_timing_read, int(kernel), C.byref(ms), C.byref(cnt))
        return ms.value, cnt.value

    def timing_reset(self):
        self._call(self._lib.esdg_timing_reset)


def operators(p: int):
    """(x, w, D, D~) of degree p as the library builds them (host only)."""
    lib = load_library()
    N = p + 1
    x, w, D, Dt = np.zeros(N), np.zeros(N), np.zeros((N, N)), np.zeros((N, N))
    dp = C.POINTER(C.c_double)
    _check(lib, None, lib.esdg_operators(int(p), x.ctypes.data_as(dp), w.ctypes.data_as(dp),
                                         D.ctypes.data_as(dp), Dt.ctypes.data_as(dp)))
    return x, w, D, Dt


def version() -> str:
    return load_library().esdg_version().decode()
