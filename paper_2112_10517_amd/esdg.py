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
KERNEL_STAGE, KERNEL_REDUCE, KERNEL_PROJECT, KERNEL_FACE = 1, 2, 3, 4
FACES_FUSED, FACES_ONCE = 0, 1
NODES = {"lgl": 0, "gauss": 1}
INTEGRATORS = {"rk4": 0, "ck45": 1}
PMAX = 7
TILE_VARIANTS = 5
BATCH_GRAPHS, BATCH_CONCURRENT = 1, 2
JOB_QUEUED, JOB_ACTIVE, JOB_DONE, JOB_FAILED = 0, 1, 2, 3


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
                ("precision", C.c_int32), ("stream", C.c_void_p), ("nodes", C.c_int32), ("pad", C.c_int32)]


class ServerConfig(C.Structure):
    _fields_ = [("hbm_budget", C.c_int64), ("max_active", C.c_int32), ("steps_per_tick", C.c_int32),
                ("flags", C.c_int32), ("pad", C.c_int32), ("cfl", C.c_double)]


class JobDesc(C.Structure):
    _fields_ = [("mesh", MeshDesc), ("u0", C.POINTER(C.c_double)), ("t0", C.c_double), ("t_end", C.c_double)]


_lib = None
_lib_path = None
_lock = threading.Lock()

_vp, _dp, _i32, _i64, _d = C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_int64, C.c_double
_pi32, _pi64 = C.POINTER(C.c_int32), C.POINTER(C.c_int64)
_st, _str = C.c_int, C.c_char_p

# name -> (restype, argtypes) of every exported symbol of include/esdg.h
SIGNATURES = {
    "esdg_init_mesh": (_st, [C.POINTER(MeshDesc), C.POINTER(_vp)]),
    "esdg_destroy": (None, [_vp]),
    "esdg_sizes": (_st, [_vp, _pi64, _pi32, _pi32]),
    "esdg_set_stream": (_st, [_vp, _vp]),
    "esdg_get_coords": (_st, [_vp, _dp]),
    "esdg_get_inv_jacobian": (_st, [_vp, _dp]),
    "esdg_set_state": (_st, [_vp, _vp, _i32]),
    "esdg_get_state": (_st, [_vp, _vp, _i32]),
    "esdg_rhs": (_st, [_vp, _vp, _i32]),
    "esdg_step": (_st, [_vp, _d, _i32, _d, _dp]),
    "esdg_set_time": (_st, [_vp, _d]),
    "esdg_set_integrator": (_st, [_vp, _i32]),
    "esdg_get_integrator": (_st, [_vp, _pi32]),
    "esdg_get_time": (_st, [_vp, _dp]),
    "esdg_entropy_rate": (_st, [_vp, _dp]),
    "esdg_totals": (_st, [_vp, _dp]),
    "esdg_totals_noalloc": (_st, [_vp, _vp]),
    "esdg_max_dt": (_st, [_vp, _d, _dp]),
    "esdg_sync": (_st, [_vp]),
    "esdg_timing_enable": (_st, [_vp, _i32]),
    "esdg_timing_read": (_st, [_vp, _i32, _dp, _pi64]),
    "esdg_timing_reset": (_st, [_vp]),
    "esdg_autotune": (_st, [_vp, _i32, _pi32, _dp]),
    "esdg_set_tile_variant": (_st, [_vp, _i32]),
    "esdg_get_tile_variant": (_st, [_vp, _pi32, _pi32]),
    "esdg_set_face_flux_mode": (_st, [_vp, _i32]),
    "esdg_get_face_flux_mode": (_st, [_vp, _pi32]),
    "esdg_footprint": (_st, [C.POINTER(MeshDesc), _pi64]),
    "esdg_batch_create": (_st, [C.POINTER(_vp), _i32, _dp, _vp, _i32, C.POINTER(_vp)]),
    "esdg_batch_destroy": (None, [_vp]),
    "esdg_batch_step": (_st, [_vp, _d, _i32, _d]),
    "esdg_batch_rhs": (_st, [_vp, C.POINTER(_vp), _i32]),
    "esdg_batch_times": (_st, [_vp, _dp]),
    "esdg_batch_sync": (_st, [_vp, _pi32]),
    "esdg_batch_autotune": (_st, [_vp, _i32]),
    "esdg_batch_info": (_st, [_vp, _pi32, _pi64]),
    "esdg_batch_timing_enable": (_st, [_vp, _i32]),
    "esdg_batch_timing_read": (_st, [_vp, _dp, _pi64]),
    "esdg_batch_last_error": (_str, [_vp]),
    "esdg_server_create": (_st, [C.POINTER(ServerConfig), C.POINTER(_vp)]),
    "esdg_server_destroy": (None, [_vp]),
    "esdg_server_submit": (_st, [_vp, C.POINTER(JobDesc), _pi64]),
    "esdg_server_tick": (_st, [_vp, _pi32, _pi32, _pi32]),
    "esdg_server_job": (_st, [_vp, _i64, _pi32, _dp, _pi64]),
    "esdg_server_finished": (_st, [_vp, _pi64, _i32, _pi32]),
    "esdg_server_fetch": (_st, [_vp, _i64, _dp]),
    "esdg_server_memory": (_st, [_vp, _pi64, _pi64]),
    "esdg_server_last_error": (_str, [_vp]),
    "esdg_server_plan": (_st, [_pi64, _i32, _i64, _i64, _i32, _i32, _pi32]),
    "esdg_operators": (_st, [_i32, _dp, _dp, _dp, _dp]),
    "esdg_last_error": (_str, [_vp]),
    "esdg_version": (_str, []),
}
EXPORTS = list(SIGNATURES)


def load_library(path: str | None = None):
    """Load libesdg.so (raises if it has not been built).  With a path, that
    build becomes the library every later call of this module uses (Problem,
    Batch, Server); a second, different path raises, since two builds of the
    library in one process would share no state."""
    global _lib, _lib_path
    with _lock:
        if _lib is not None and (path is None or os.path.realpath(path) == _lib_path):
            return _lib
        if _lib is not None:
            raise RuntimeError("libesdg is already loaded from %s; cannot load %s as well" % (_lib_path, path))
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
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib, _lib_path = lib, os.path.realpath(p)
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


def mesh_desc(dim: int, p: int, n, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0), warp: float = 0.0,
              gamma: float = 1.4, volume_flux="ranocha", surface_flux="llf", precision="fp64",
              nodes="lgl") -> MeshDesc:
    """esdg_mesh_desc of a periodic box (coords and stream unset)."""
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
    d.nodes = NODES[nodes] if isinstance(nodes, str) else int(nodes)
    return d


def server_plan(queued_bytes, used: int, budget: int, active: int = 0, max_active: int = 0) -> int:
    """How many of the queued jobs (device bytes, arrival order) the server's
    admission rule admits now (esdg_server_plan)."""
    lib = load_library()
    q = (C.c_int64 * max(1, len(queued_bytes)))(*[int(b) for b in queued_bytes])
    k = C.c_int32()
    _check(lib, None, lib.esdg_server_plan(q, len(queued_bytes), int(used), int(budget), int(active),
                                           int(max_active), C.byref(k)))
    return k.value


def footprint(dim: int, p: int, n, **kw) -> int:
    """Device bytes a problem of these parameters allocates (esdg_footprint)."""
    lib = load_library()
    b = C.c_int64()
    _check(lib, None, lib.esdg_footprint(C.byref(mesh_desc(dim, p, n, **kw)), C.byref(b)))
    return b.value


class Problem:
    """One periodic Euler problem on the GPU (handle of ``esdg_init_mesh``)."""

    def __init__(self, dim: int, p: int, n, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0),
                 warp: float = 0.0, gamma: float = 1.4, volume_flux: str = "ranocha",
                 surface_flux: str = "llf", precision: str = "fp64", coords=None, stream=None,
                 nodes: str = "lgl", integrator: str = "rk4"):
        self._lib = load_library()
        d = mesh_desc(dim, p, n, lo, hi, warp, gamma, volume_flux, surface_flux, precision, nodes)
        keep = None
        if coords is not None:
            keep = np.ascontiguousarray(coords, dtype=np.float64)
            d.coords = keep.ctypes.data_as(C.POINTER(C.c_double))
        d.stream = self._stream_ptr(stream)
        self._stream = d.stream or 0
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
        if integrator != "rk4":
            self.set_integrator(integrator)

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
        sp = self._stream_ptr(stream)
        self._call(self._lib.esdg_set_stream, sp)
        self._stream = (sp.value if sp is not None else None) or 0

    def stream_ptr(self) -> int:
        """The hipStream_t the problem's device work is enqueued on (0: default)."""
        return int(self._stream)

    def coords(self) -> np.ndarray:
        x = np.zeros((self.n_elem, self.dim, self.nodes))
        self._call(self._lib.esdg_get_coords, x.ctypes.data_as(C.POINTER(C.c_double)))
        return x

    def inv_jacobian(self) -> np.ndarray:
        """1/J per node [elem][node] as the kernels use it (host FP64 array)."""
        x = np.zeros((self.n_elem, self.nodes))
        self._call(self._lib.esdg_get_inv_jacobian, x.ctypes.data_as(C.POINTER(C.c_double)))
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

    def set_integrator(self, integrator):
        """Integrator of later steps: "rk4" (classical, default) or "ck45" (five-stage 2N-storage)."""
        k = INTEGRATORS[integrator] if isinstance(integrator, str) else int(integrator)
        self._call(self._lib.esdg_set_integrator, k)

    def integrator(self) -> str:
        k = C.c_int32()
        self._call(self._lib.esdg_get_integrator, C.byref(k))
        return {v: n for n, v in INTEGRATORS.items()}[k.value]

    def set_time(self, t: float):
        self._call(self._lib.esdg_set_time, float(t))

    def get_time(self) -> float:
        r = C.c_double()
        self._call(self._lib.esdg_get_time, C.byref(r))
        return r.value

    def autotune(self, reps: int = 20):
        """Time every tile variant on the current state; (best variant, us per variant)."""
        best = C.c_int32()
        us = (C.c_double * TILE_VARIANTS)()
        self._call(self._lib.esdg_autotune, int(reps), C.byref(best), us)
        return best.value, list(us)

    def tile_variant(self):
        """(variant in use for this problem's parameters, elements per workgroup)."""
        v, e = C.c_int32(), C.c_int32()
        self._call(self._lib.esdg_get_tile_variant, C.byref(v), C.byref(e))
        return v.value, e.value

    def set_tile_variant(self, variant: int):
        self._call(self._lib.esdg_set_tile_variant, int(variant))

    def face_flux_mode(self) -> int:
        """FACES_FUSED (each element evaluates its faces) or FACES_ONCE."""
        m = C.c_int32()
        self._call(self._lib.esdg_get_face_flux_mode, C.byref(m))
        return m.value

    def set_face_flux_mode(self, mode: int):
        self._call(self._lib.esdg_set_face_flux_mode, int(mode))

    def entropy_rate(self) -> float:
        r = C.c_double()
        self._call(self._lib.esdg_entropy_rate, C.byref(r))
        return r.value

    def totals(self) -> np.ndarray:
        t = np.zeros(self.n_var)
        self._call(self._lib.esdg_totals, t.ctypes.data_as(C.POINTER(C.c_double)))
        return t

    def totals_noalloc(self, out):
        """esdg_totals_noalloc: the totals into `out`, a float64 CUDA tensor of
        n_var entries, in stream order (no wait; no allocation by the library)."""
        import torch
        if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64
                and out.is_contiguous() and out.numel() >= self.n_var):
            raise TypeError("totals_noalloc needs a contiguous float64 CUDA tensor of n_var entries")
        self._call(self._lib.esdg_totals_noalloc, C.c_void_p(out.data_ptr()))
        return out

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


class Batch:
    """Problems advanced together (handle of ``esdg_batch_create``).

    The batch references its members: keep the Problem objects alive while it
    exists."""

    def __init__(self, problems, t_end=None, stream=None, graphs: bool = True, concurrent: bool = False):
        self._lib = load_library()
        self.problems = list(problems)
        arr = (C.c_void_p * len(self.problems))(*[q._h.value for q in self.problems])
        te = None
        if t_end is not None:
            te = np.ascontiguousarray(t_end, dtype=np.float64)
            if te.shape != (len(self.problems),):
                raise ValueError("t_end needs one entry per problem")
        flags = (BATCH_GRAPHS if graphs else 0) | (BATCH_CONCURRENT if concurrent else 0)
        sp = None if stream is None else (C.c_void_p(stream) if isinstance(stream, int) else C.c_void_p(stream.cuda_stream))
        h = C.c_void_p()
        st = self._lib.esdg_batch_create(arr, len(self.problems), None if te is None else te.ctypes.data_as(_dp),
                                         sp, flags, C.byref(h))
        _check(self._lib, None, st)
        self._h = h

    def _call(self, fn, *args):
        st = fn(self._h, *args)
        if st != OK:
            msg = self._lib.esdg_batch_last_error(self._h)
            cls = NonPhysicalState if st == ENONPHYSICAL else EsdgError
            raise cls(st, msg.decode() if msg else "")

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.esdg_batch_destroy(h)
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

    def step(self, dt: float = 0.0, nsteps: int = 1, cfl: float = 0.0):
        self._call(self._lib.esdg_batch_step, float(dt), int(nsteps), float(cfl))

    def rhs(self, outs=None):
        """RHS of every member; outs: list of arrays/tensors (or None entries), or None."""
        if outs is None:
            self._call(self._lib.esdg_batch_rhs, None, HOST)
            return None
        ptrs, wheres, keep = [], set(), []
        for q, o in zip(self.problems, outs):
            if o is None:
                ptrs.append(None)
                continue
            ptr, where, k = _where_ptr(o, q.shape, True)
            ptrs.append(ptr.value)
            wheres.add(where)
            keep.append(k)
        if len(wheres) > 1:
            raise ValueError("outputs must all be host or all be device memory")
        arr = (C.c_void_p * len(ptrs))(*ptrs)
        self._call(self._lib.esdg_batch_rhs, arr, wheres.pop() if wheres else HOST)
        return outs

    def times(self) -> np.ndarray:
        t = np.zeros(len(self.problems))
        self._call(self._lib.esdg_batch_times, t.ctypes.data_as(_dp))
        return t

    def sync(self):
        bad = C.c_int32()
        self._call(self._lib.esdg_batch_sync, C.byref(bad))

    def autotune(self, reps: int = 10):
        self._call(self._lib.esdg_batch_autotune, int(reps))

    def info(self):
        g, t = C.c_int32(), C.c_int64()
        self._call(self._lib.esdg_batch_info, C.byref(g), C.byref(t))
        return g.value, t.value

    def timing(self, enable: bool):
        self._call(self._lib.esdg_batch_timing_enable, 1 if enable else 0)

    def timing_read(self):
        ms, n = C.c_double(), C.c_int64()
        self._call(self._lib.esdg_batch_timing_read, C.byref(ms), C.byref(n))
        return ms.value, n.value


class Server:
    """Continuous-batching request loop (handle of ``esdg_server_create``)."""

    def __init__(self, cfl: float, steps_per_tick: int = 8, hbm_budget: int = 0, max_active: int = 0,
                 graphs: bool = True, concurrent: bool = False):
        self._lib = load_library()
        c = ServerConfig()
        c.hbm_budget, c.max_active, c.steps_per_tick = int(hbm_budget), int(max_active), int(steps_per_tick)
        c.flags = (BATCH_GRAPHS if graphs else 0) | (BATCH_CONCURRENT if concurrent else 0)
        c.cfl = float(cfl)
        h = C.c_void_p()
        st = self._lib.esdg_server_create(C.byref(c), C.byref(h))
        if st != OK:
            raise EsdgError(st, "esdg_server_create failed")
        self._h = h
        self._shapes = {}

    def _call(self, fn, *args):
        st = fn(self._h, *args)
        if st != OK:
            msg = self._lib.esdg_server_last_error(self._h)
            raise EsdgError(st, msg.decode() if msg else "")

    def close(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.esdg_server_destroy(h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, u0: np.ndarray, t_end: float, t0: float = 0.0, **mesh) -> int:
        """Queue a job: u0 (host FP64 state), end time, mesh keywords of mesh_desc()."""
        j = JobDesc()
        j.mesh = mesh_desc(**mesh)
        u = np.ascontiguousarray(u0, dtype=np.float64)
        j.u0 = u.ctypes.data_as(_dp)
        j.t0, j.t_end = float(t0), float(t_end)
        jid = C.c_int64()
        self._call(self._lib.esdg_server_submit, C.byref(j), C.byref(jid))
        self._shapes[jid.value] = u.shape
        return jid.value

    def tick(self):
        """One tick; returns (finished ids, active, queued)."""
        f, a, q = C.c_int32(), C.c_int32(), C.c_int32()
        self._call(self._lib.esdg_server_tick, C.byref(f), C.byref(a), C.byref(q))
        ids = (C.c_int64 * max(1, f.value))()
        n = C.c_int32()
        self._call(self._lib.esdg_server_finished, ids, f.value, C.byref(n))
        return [ids[i] for i in range(n.value)], a.value, q.value

    def job(self, jid: int):
        """(status, time, steps) of a job."""
        s, t, n = C.c_int32(), C.c_double(), C.c_int64()
        self._call(self._lib.esdg_server_job, int(jid), C.byref(s), C.byref(t), C.byref(n))
        return s.value, t.value, n.value

    def fetch(self, jid: int, want_state: bool = True):
        """Final state of a finished job (host array, or None) and release of the job."""
        shape = self._shapes.get(jid)
        u = np.empty(shape) if want_state and shape is not None else None
        self._call(self._lib.esdg_server_fetch, int(jid), None if u is None else u.ctypes.data_as(_dp))
        self._shapes.pop(jid, None)
        return u

    def memory(self):
        used, budget = C.c_int64(), C.c_int64()
        self._call(self._lib.esdg_server_memory, C.byref(used), C.byref(budget))
        return used.value, budget.value
