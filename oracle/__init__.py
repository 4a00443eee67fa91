"""CPU oracle for the flux-differencing LGL-DGSEM and the Legendre-Gauss
collocation scheme with entropy projection (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``esdg_oracle.c`` (plain C,
FP64, OpenMP across elements) through ctypes and shares no code with the HIP
library in ``paper_2112_10517_amd``.

Every function follows the definitions of Ranocha et al. (arXiv:2112.10517):
the flux-differencing DG form of Sec. 2, the Euler fluxes and log means of
Sec. 3, the metric terms of Sec. 2.3, the hybridised Gauss collocation form of
Sec. 6.  See the header of ``esdg_oracle.c`` for
the readings taken where the paper is silent.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "esdg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

RANOCHA, SHIMA, LLF, CENTRAL = 0, 1, 2, 3
FLUX_NAMES = {"ranocha": RANOCHA, "shima": SHIMA, "llf": LLF, "central": CENTRAL}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("p", C.c_int32), ("n", C.c_int32 * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("warp", C.c_double), ("gamma", C.c_double),
                ("vol_flux", C.c_int32), ("surf_flux", C.c_int32), ("nodes", C.c_int32)]


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        build()
        lib = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        lib.orc_lgl.argtypes = [C.c_int, dp, dp, dp]
        lib.orc_lgl.restype = C.c_int
        lib.orc_gauss.argtypes = [C.c_int, dp, dp, dp, dp, dp]
        lib.orc_gauss.restype = C.c_int
        lib.orc_cons_from_entropy.argtypes = [C.c_int, C.c_double, dp, dp]
        lib.orc_logmean.argtypes = [C.c_double, C.c_double]
        lib.orc_logmean.restype = C.c_double
        lib.orc_inv_logmean.argtypes = [C.c_double, C.c_double]
        lib.orc_inv_logmean.restype = C.c_double
        lib.orc_phys_flux.argtypes = [C.c_int, C.c_double, dp, dp, dp]
        lib.orc_two_point.argtypes = [C.c_int, C.c_int, C.c_double, dp, dp, dp, dp]
        lib.orc_entropy_vars.argtypes = [C.c_int, C.c_double, dp, dp]
        lib.orc_entropy.argtypes = [C.c_int, C.c_double, dp, dp, dp, dp]
        lib.orc_mesh_new.argtypes = [C.POINTER(_Desc), dp]
        lib.orc_mesh_new.restype = C.c_void_p
        lib.orc_mesh_free.argtypes = [C.c_void_p]
        lib.orc_mesh_sizes.argtypes = [C.c_void_p, C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        lib.orc_mesh_geometry.argtypes = [C.c_void_p, dp, dp, dp]
        lib.orc_mesh_operators.argtypes = [C.c_void_p, dp, dp, dp]
        lib.orc_rhs.argtypes = [C.c_void_p, dp, dp]
        lib.orc_rhs_scale.argtypes = [C.c_void_p, dp, dp]
        lib.orc_rhs_elements.argtypes = [C.c_void_p, dp, dp, C.POINTER(C.c_int64), C.c_int64]
        lib.orc_rhs_scale_elements.argtypes = [C.c_void_p, dp, dp, C.POINTER(C.c_int64), C.c_int64]
        lib.orc_totals.argtypes = [C.c_void_p, dp, dp]
        lib.orc_entropy_rate.argtypes = [C.c_void_p, dp, dp]
        lib.orc_entropy_rate.restype = C.c_double
        lib.orc_max_dt.argtypes = [C.c_void_p, dp, C.c_double]
        lib.orc_max_dt.restype = C.c_double
        lib.orc_rk4.argtypes = [C.c_void_p, dp, C.c_double, C.c_int, C.c_double, dp]
        lib.orc_ck45.argtypes = [C.c_void_p, dp, C.c_double, C.c_int, C.c_double, dp]
        lib.orc_ck45_coefficients.argtypes = [dp, dp]
        lib.orc_num_threads.argtypes = []
        lib.orc_num_threads.restype = C.c_int
        lib.orc_set_num_threads.argtypes = [C.c_int]
        lib.orc_set_num_threads.restype = None
        _lib = lib
        return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def num_threads() -> int:
    """OpenMP threads the oracle's element loops use."""
    return _load().orc_num_threads()


def ck45_coefficients():
    """(A, B) of the oracle's 2N-storage scheme (Carpenter and Kennedy)."""
    A, B = np.zeros(5), np.zeros(5)
    _load().orc_ck45_coefficients(_ptr(A), _ptr(B))
    return A, B


def set_num_threads(n: int) -> None:
    """Set the OpenMP threads of the oracle's element loops (for timing)."""
    _load().orc_set_num_threads(int(n))


# --------------------------------------------------------------------------
# point functions
# --------------------------------------------------------------------------

def lgl(p: int):
    """LGL nodes, weights and derivative matrix D (N x N) for degree p."""
    lib = _load()
    N = p + 1
    xi, w, D = np.zeros(N), np.zeros(N), np.zeros((N, N))
    if lib.orc_lgl(p, _ptr(xi), _ptr(w), _ptr(D)) != 0:
        raise ValueError("degree out of range")
    return xi, w, D


def gauss(p: int):
    """Legendre-Gauss nodes, weights, derivative matrix D (N x N) and the
    Lagrange basis values at -1 and +1 (rL, rR) for degree p (N = p+1 nodes)."""
    lib = _load()
    N = p + 1
    xi, w, D, rL, rR = np.zeros(N), np.zeros(N), np.zeros((N, N)), np.zeros(N), np.zeros(N)
    if lib.orc_gauss(p, _ptr(xi), _ptr(w), _ptr(D), _ptr(rL), _ptr(rR)) != 0:
        raise ValueError("degree out of range")
    return xi, w, D, rL, rR


def cons_from_entropy(dim: int, gamma: float, w) -> np.ndarray:
    """Conservative variables of entropy variables w (inverse of entropy_vars)."""
    w = _f64(w)
    u = np.zeros(dim + 2)
    _load().orc_cons_from_entropy(dim, gamma, _ptr(w), _ptr(u))
    return u


def logmean(a, b) -> float:
    """Algorithm 2 of Sec. 3.1, arguments (a_-, a_+)."""
    return _load().orc_logmean(float(a), float(b))


def inv_logmean(a, b) -> float:
    """Algorithm 3 of Sec. 3.1, arguments (a_-, a_+)."""
    return _load().orc_inv_logmean(float(a), float(b))


def phys_flux(dim: int, gamma: float, u, n) -> np.ndarray:
    u, nn = _f64(u), _f64(list(n) + [0.0] * (3 - len(n)))
    f = np.zeros(dim + 2)
    _load().orc_phys_flux(dim, gamma, _ptr(u), _ptr(nn), _ptr(f))
    return f


def two_point(kind, dim: int, gamma: float, um, up, n) -> np.ndarray:
    """Directional two-point flux f(u_-, u_+, n); kind in FLUX_NAMES."""
    k = FLUX_NAMES[kind] if isinstance(kind, str) else int(kind)
    um, up = _f64(um), _f64(up)
    nn = _f64(list(n) + [0.0] * (3 - len(n)))
    f = np.zeros(dim + 2)
    _load().orc_two_point(k, dim, gamma, _ptr(um), _ptr(up), _ptr(nn), _ptr(f))
    return f


def entropy_vars(dim: int, gamma: float, u) -> np.ndarray:
    u = _f64(u)
    w = np.zeros(dim + 2)
    _load().orc_entropy_vars(dim, gamma, _ptr(u), _ptr(w))
    return w


def entropy(dim: int, gamma: float, u, n):
    """(U, F.n) for the entropy U = -rho s/(gamma-1)."""
    u = _f64(u)
    nn = _f64(list(n) + [0.0] * (3 - len(n)))
    U, F = C.c_double(), C.c_double()
    _load().orc_entropy(dim, gamma, _ptr(u), _ptr(nn), C.byref(U), C.byref(F))
    return U.value, F.value


# --------------------------------------------------------------------------
# mesh-level oracle
# --------------------------------------------------------------------------

class Mesh:
    """Periodic box mesh of n[0] x ... elements of degree p (plain CPU);
    nodes = "lgl" (Sec. 2) or "gauss" (Sec. 6, affine meshes only)."""

    def __init__(self, dim, p, n, lo=(-1.0, -1.0, -1.0), hi=(1.0, 1.0, 1.0), warp=0.0,
                 gamma=1.4, vol_flux="ranocha", surf_flux="llf", coords=None, nodes="lgl"):
        lib = _load()
        d = _Desc()
        d.dim, d.p = dim, p
        n = list(n) + [1] * (3 - len(n))
        lo = list(lo) + [0.0] * (3 - len(lo))
        hi = list(hi) + [1.0] * (3 - len(hi))
        for j in range(3):
            d.n[j], d.lo[j], d.hi[j] = n[j], lo[j], hi[j]
        d.warp, d.gamma = warp, gamma
        d.vol_flux = FLUX_NAMES[vol_flux] if isinstance(vol_flux, str) else vol_flux
        d.surf_flux = FLUX_NAMES[surf_flux] if isinstance(surf_flux, str) else surf_flux
        d.nodes = {"lgl": 0, "gauss": 1}[nodes]
        self.node_kind = nodes
        self._coords = None if coords is None else _f64(coords)
        h = lib.orc_mesh_new(C.byref(d), None if coords is None else _ptr(self._coords))
        if not h:
            raise ValueError("invalid mesh description")
        self._h = h
        self._lib = lib
        ne, nn, nv = C.c_int64(), C.c_int32(), C.c_int32()
        lib.orc_mesh_sizes(h, C.byref(ne), C.byref(nn), C.byref(nv))
        self.dim, self.p, self.N, self.gamma = dim, p, p + 1, gamma
        self.n_elem, self.nodes, self.n_var = ne.value, nn.value, nv.value
        self.shape = (self.n_elem, self.n_var, self.nodes)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.orc_mesh_free(h)
            self._h = None

    # geometry -----------------------------------------------------------
    def coords(self) -> np.ndarray:
        x = np.zeros((self.n_elem, self.dim, self.nodes))
        self._lib.orc_mesh_geometry(self._h, _ptr(x), None, None)
        return x

    def metrics(self):
        Ja = np.zeros((self.n_elem, 3, 3, self.nodes))
        J = np.zeros((self.n_elem, self.nodes))
        self._lib.orc_mesh_geometry(self._h, None, _ptr(Ja), _ptr(J))
        return Ja, J

    def operators(self):
        xi, w, D = np.zeros(self.N), np.zeros(self.N), np.zeros((self.N, self.N))
        self._lib.orc_mesh_operators(self._h, _ptr(xi), _ptr(w), _ptr(D))
        return xi, w, D

    def weights(self) -> np.ndarray:
        """tensor-product quadrature weights W_i per node."""
        _, w, _ = self.operators()
        W = np.ones(self.nodes)
        idx = np.arange(self.nodes)
        for j in range(self.dim):
            W *= w[(idx // self.N ** j) % self.N]
        return W

    # method -------------------------------------------------------------
    def _state(self, u) -> np.ndarray:
        u = _f64(u)
        if u.shape != self.shape:
            raise ValueError("state shape %s != %s" % (u.shape, self.shape))
        return u

    def rhs(self, u) -> np.ndarray:
        u = self._state(u)
        du = np.empty_like(u)
        self._lib.orc_rhs(self._h, _ptr(u), _ptr(du))
        return du

    def rhs_scale(self, u) -> np.ndarray:
        """Per-node rounding scale of RHS: the same sums over term magnitudes."""
        u = self._state(u)
        sc = np.empty_like(u)
        self._lib.orc_rhs_scale(self._h, _ptr(u), _ptr(sc))
        return sc

    def rhs_elements(self, u, elems):
        """(RHS, rounding scale) of the listed elements only: arrays [len(elems), var, node]."""
        u = self._state(u)
        el = np.ascontiguousarray(np.asarray(elems, dtype=np.int64))
        du = np.zeros_like(u)
        sc = np.zeros_like(u)
        ep = el.ctypes.data_as(C.POINTER(C.c_int64))
        self._lib.orc_rhs_elements(self._h, _ptr(u), _ptr(du), ep, len(el))
        self._lib.orc_rhs_scale_elements(self._h, _ptr(u), _ptr(sc), ep, len(el))
        return du[el], sc[el]

    def totals(self, u) -> np.ndarray:
        u = self._state(u)
        t = np.zeros(self.n_var)
        self._lib.orc_totals(self._h, _ptr(u), _ptr(t))
        return t

    def entropy_rate(self, u, du=None) -> float:
        u = self._state(u)
        du = self.rhs(u) if du is None else self._state(du)
        return self._lib.orc_entropy_rate(self._h, _ptr(u), _ptr(du))

    def max_dt(self, u, cfl: float) -> float:
        return self._lib.orc_max_dt(self._h, _ptr(self._state(u)), cfl)

    def rk4(self, u, dt: float, nsteps: int, cfl: float = 0.0, t: float = 0.0):
        """Return (u_new, t_new) after nsteps classical RK4 steps."""
        u = self._state(u).copy()
        tt = C.c_double(t)
        self._lib.orc_rk4(self._h, _ptr(u), dt, nsteps, cfl, C.byref(tt))
        return u, tt.value

    def ck45(self, u, dt: float, nsteps: int, cfl: float = 0.0, t: float = 0.0):
        """Return (u_new, t_new) after nsteps steps of the five-stage, fourth-order
        2N-storage scheme of Carpenter and Kennedy (Williamson form)."""
        u = self._state(u).copy()
        tt = C.c_double(t)
        self._lib.orc_ck45(self._h, _ptr(u), dt, nsteps, cfl, C.byref(tt))
        return u, tt.value
