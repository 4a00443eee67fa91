"""Seeded synthetic initial states for the Euler workloads (numpy only).

This module holds no part of the discretisation: it only turns node
coordinates ``x`` (layout ``[elem][dim][node]``) into conservative states
``u`` (layout ``[elem][var][node]``, variables rho, rho v_1..rho v_d, rho e)
with the ideal-gas relation rho e = p/(gamma-1) + rho |v|^2 / 2 of Sec. 3.
Both the HIP library and the CPU oracle consume the arrays it returns.

Workloads:
  * density wave: rho = 1 + A sin(pi (x_1+...+x_d)), constant v and p
    (exact solution: translation with v);
  * smooth random Fourier modes (rho, p in [0.8, 1.2], |v_j| <= 0.1, |k| <= 4);
  * Taylor-Green vortex on [0, 2 pi]^3 at a given Mach number;
  * isentropic vortex of Sec. 4.1 (vortex strength 20, context workload);
  * sinusoidal state of Sec. 7.2.
"""
from __future__ import annotations

import math

import numpy as np


def prim_to_cons(rho, v, p, gamma: float) -> np.ndarray:
    """rho [E,n], v [E,d,n], p [E,n] -> u [E,d+2,n]."""
    rho = np.asarray(rho, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    E, d, n = v.shape
    u = np.empty((E, d + 2, n))
    u[:, 0] = rho
    u[:, 1:d + 1] = rho[:, None, :] * v
    u[:, d + 1] = p / (gamma - 1.0) + 0.5 * rho * np.sum(v * v, axis=1)
    return u


def cons_to_prim(u, gamma: float):
    u = np.asarray(u, dtype=np.float64)
    d = u.shape[1] - 2
    rho = u[:, 0]
    v = u[:, 1:d + 1] / rho[:, None, :]
    p = (gamma - 1.0) * (u[:, d + 1] - 0.5 * rho * np.sum(v * v, axis=1))
    return rho, v, p


DENSITY_WAVE_V = (0.1, 0.2, 0.3)


def density_wave(x, gamma: float = 1.4, amp: float = 0.98, p0: float = 20.0,
                 t: float = 0.0, v=None) -> np.ndarray:
    """rho = 1 + amp sin(pi (sum_j x_j - t sum_j v_j)), v = (0.1, 0.2, 0.3)[:d], p = p0."""
    x = np.asarray(x, dtype=np.float64)
    E, d, n = x.shape
    vel = np.asarray(DENSITY_WAVE_V[:d] if v is None else v, dtype=np.float64)
    phase = np.sum(x, axis=1) - t * float(np.sum(vel))
    rho = 1.0 + amp * np.sin(np.pi * phase)
    vv = np.broadcast_to(vel[None, :, None], (E, d, n))
    return prim_to_cons(rho, vv, np.full((E, n), p0), gamma)


def fourier_modes(rng, d: int, modes: int = 8, kmax: float = 4.0):
    """`modes` draws (k, a, phi): integer k with 1 <= |k| <= kmax, a = U[0.5,1]/|k|, phi = U[0,2pi]."""
    K = int(math.floor(kmax))
    out = []
    for _ in range(modes):
        while True:
            k = rng.integers(-K, K + 1, size=d)
            nk = float(np.sqrt(np.sum(k * k)))
            if 1.0 <= nk <= kmax:
                break
        a = rng.uniform(0.5, 1.0) / nk
        phi = rng.uniform(0.0, 2.0 * np.pi)
        out.append((k.astype(np.float64), a, phi))
    return out


def random_fourier_modes(seed: int, d: int):
    """Mode lists of the fields rho, p, v_1..v_d of random_fourier(seed)."""
    return [fourier_modes(np.random.Generator(np.random.PCG64(seed * 16 + idx)), d) for idx in range(2 + d)]


def _fourier_field(rng, s: np.ndarray, modes: int = 8, kmax: float = 4.0) -> np.ndarray:
    """sum of `modes` sines sin(pi k.s + phi), 1 <= |k| <= kmax, amplitude U[0.5,1]/|k|."""
    E, d, n = s.shape
    g = np.zeros((E, n))
    for k, a, phi in fourier_modes(rng, d, modes, kmax):
        g += a * np.sin(np.pi * np.einsum("j,ejn->en", k, s) + phi)
    return g


def random_fourier(x, seed: int, gamma: float = 1.4, lo=None, hi=None) -> np.ndarray:
    """Smooth random state: rho, p in [0.8, 1.2] and v_j in [-0.1, 0.1].

    Each field (rho, p, v_1..v_d) draws 8 Fourier modes with integer wave
    vector 1 <= |k| <= 4 (periodic on the box scaled to [-1,1]^d) from its own
    PCG64 stream (seed*16 + field), and is scaled so that its extreme value
    over the given nodes hits the interval end exactly.
    """
    x = np.asarray(x, dtype=np.float64)
    E, d, n = x.shape
    lo = np.full(d, -1.0) if lo is None else np.asarray(lo[:d], dtype=np.float64)
    hi = np.full(d, 1.0) if hi is None else np.asarray(hi[:d], dtype=np.float64)
    s = 2.0 * (x - lo[None, :, None]) / (hi - lo)[None, :, None] - 1.0

    def field(idx):
        g = _fourier_field(np.random.Generator(np.random.PCG64(seed * 16 + idx)), s)
        return g / np.max(np.abs(g))

    rho = 1.0 + 0.2 * field(0)
    p = 1.0 + 0.2 * field(1)
    v = np.stack([0.1 * field(2 + j) for j in range(d)], axis=1)
    return prim_to_cons(rho, v, p, gamma)


def taylor_green(x, gamma: float = 1.4, mach: float = 0.1) -> np.ndarray:
    """Taylor-Green vortex on [0, 2 pi]^3: rho = 1, p0 = 1/(gamma Ma^2)."""
    x = np.asarray(x, dtype=np.float64)
    E, d, n = x.shape
    if d != 3:
        raise ValueError("Taylor-Green vortex is three-dimensional")
    X, Y, Z = x[:, 0], x[:, 1], x[:, 2]
    v = np.stack([np.sin(X) * np.cos(Y) * np.cos(Z),
                  -np.cos(X) * np.sin(Y) * np.cos(Z),
                  np.zeros_like(X)], axis=1)
    p0 = 1.0 / (gamma * mach * mach)
    p = p0 + (np.cos(2 * X) + np.cos(2 * Y)) * (np.cos(2 * Z) + 2.0) / 16.0
    return prim_to_cons(np.ones_like(X), v, p, gamma)


def isentropic_vortex(x, gamma: float = 1.4, eps: float = 20.0, t: float = 0.0) -> np.ndarray:
    """Isentropic vortex of Sec. 4.1 (rho0 = 1, v0 = (1,1,0), p0 = 10, periodic
    domain [-5,5]^d), centred at v0 t (wrapped into the domain).

    r is the distance from the centre over all d coordinates, as the paper
    states it; in 2D the state at time t is the exact solution (the initial
    vortex translated with v0), in 3D the field is only a test state.
    """
    x = np.asarray(x, dtype=np.float64)
    E, d, n = x.shape
    rho0, p0 = 1.0, 10.0
    T0 = p0 / rho0
    v0 = np.array([1.0, 1.0, 0.0][:d])
    xs = x - (v0 * t)[None, :, None]
    xs = np.mod(xs + 5.0, 10.0) - 5.0
    r2 = np.sum(xs * xs, axis=1)
    T = T0 - (gamma - 1.0) * eps ** 2 / (8.0 * gamma * np.pi ** 2) * np.exp(1.0 - r2)
    rho = rho0 * (T / T0) ** (1.0 / (gamma - 1.0))
    amp = eps / (2.0 * np.pi) * np.exp(0.5 * (1.0 - r2))
    v = np.zeros((E, d, n))
    v[:, 0] = 1.0 - amp * xs[:, 1]
    v[:, 1] = 1.0 + amp * xs[:, 0]
    return prim_to_cons(rho, v, rho * T, gamma)


def sinusoidal(x, gamma: float = 1.4) -> np.ndarray:
    """rho = 2 + prod_j sin(pi x_j / 5), v = 0, p = rho^gamma (Sec. 7.2)."""
    x = np.asarray(x, dtype=np.float64)
    E, d, n = x.shape
    rho = 2.0 + np.prod(np.sin(np.pi * x / 5.0), axis=1)
    return prim_to_cons(rho, np.zeros((E, d, n)), rho ** gamma, gamma)
