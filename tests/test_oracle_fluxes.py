"""Pins of the oracle's Euler fluxes (Sec. 2 definitions of numerical fluxes and
entropy conservation; Sec. 3.2 fluxes of Shima et al. and Ranocha).

Checks: consistency with the physical flux, symmetry, the n -> -n
antisymmetry, linearity in n, Tadmor's entropy-conservation condition for
the Ranocha flux (with entropy variables pinned to a finite-difference
gradient of the entropy), the pressure-equilibrium form of both fluxes and
entropy dissipation of the local Lax-Friedrichs flux for small jumps."""
import numpy as np
import pytest

G = 1.4
EPS = np.finfo(np.float64).eps


def cons(rho, v, p):
    v = np.asarray(v, dtype=float)
    return np.concatenate([[rho], rho * v, [p / (G - 1) + 0.5 * rho * v @ v]])


def rand_state(rng, dim):
    return cons(rng.uniform(0.5, 2.0), rng.uniform(-1, 1, dim), rng.uniform(0.5, 3.0))


def rand_normal(rng, dim):
    return rng.uniform(-1.5, 1.5, dim)


def euler_flux_n(u, n):
    # physical flux sum_j n_j f^j(u) written out from the Euler equations (Sec. 3)
    dim = len(u) - 2
    rho, m, E = u[0], u[1:dim + 1], u[dim + 1]
    v = m / rho
    p = (G - 1) * (E - 0.5 * rho * v @ v)
    vn = v @ n
    return np.concatenate([[rho * vn], rho * v * vn + p * np.asarray(n), [(E + p) * vn]])


@pytest.mark.parametrize("dim", [1, 2, 3])
def test_physical_flux(orc, dim):
    rng = np.random.default_rng(1)
    for _ in range(50):
        u, n = rand_state(rng, dim), rand_normal(rng, dim)
        assert np.allclose(orc.phys_flux(dim, G, u, n), euler_flux_n(u, n), rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("kind", ["ranocha", "shima", "llf", "central"])
@pytest.mark.parametrize("dim", [2, 3])
def test_consistency_and_antisymmetry(orc, kind, dim):
    rng = np.random.default_rng(2)
    for _ in range(200):
        u1, u2, n = rand_state(rng, dim), rand_state(rng, dim), rand_normal(rng, dim)
        f_uu = orc.two_point(kind, dim, G, u1, u1, n)
        ref = euler_flux_n(u1, n)
        assert np.allclose(f_uu, ref, rtol=1e-14, atol=1e-14 * np.abs(ref).max())
        f12 = orc.two_point(kind, dim, G, u1, u2, n)
        f21m = orc.two_point(kind, dim, G, u2, u1, -n)
        assert np.allclose(f12, -f21m, rtol=1e-13, atol=1e-13 * np.abs(f12).max())


@pytest.mark.parametrize("kind", ["ranocha", "shima", "central"])
@pytest.mark.parametrize("dim", [2, 3])
def test_symmetry_and_linearity(orc, kind, dim):
    rng = np.random.default_rng(3)
    for _ in range(200):
        u1, u2 = rand_state(rng, dim), rand_state(rng, dim)
        n1, n2 = rand_normal(rng, dim), rand_normal(rng, dim)
        a, b = rng.uniform(-2, 2, 2)
        f12 = orc.two_point(kind, dim, G, u1, u2, n1)
        f21 = orc.two_point(kind, dim, G, u2, u1, n1)
        sc = np.abs(f12).max()
        assert np.allclose(f12, f21, rtol=0, atol=1e-14 * sc)
        lin = a * f12 + b * orc.two_point(kind, dim, G, u1, u2, n2)
        assert np.allclose(orc.two_point(kind, dim, G, u1, u2, a * n1 + b * n2), lin,
                           rtol=0, atol=1e-13 * max(1.0, np.abs(lin).max()))


def entropy_vars_ref(u):
    # w = dU/du of U = -rho s/(gamma-1), s = ln p - gamma ln rho
    dim = len(u) - 2
    rho, v = u[0], u[1:dim + 1] / u[0]
    p = (G - 1) * (u[dim + 1] - 0.5 * rho * v @ v)
    s = np.log(p) - G * np.log(rho)
    return np.concatenate([[(G - s) / (G - 1) - 0.5 * rho * v @ v / p], rho * v / p, [-rho / p]])


@pytest.mark.parametrize("dim", [2, 3])
def test_entropy_variables_are_gradient(orc, dim):
    rng = np.random.default_rng(4)
    for _ in range(20):
        u = rand_state(rng, dim)
        w = orc.entropy_vars(dim, G, u)
        fd = np.zeros_like(u)
        for k in range(len(u)):
            h = 1e-6 * max(1.0, abs(u[k]))
            up, um = u.copy(), u.copy()
            up[k] += h
            um[k] -= h
            fd[k] = (orc.entropy(dim, G, up, [0] * dim)[0] - orc.entropy(dim, G, um, [0] * dim)[0]) / (2 * h)
        assert np.allclose(w, fd, rtol=1e-7, atol=1e-7)
        assert np.allclose(w, entropy_vars_ref(u), rtol=1e-14, atol=1e-14)
        # entropy flux F.n = U v.n
        n = rand_normal(rng, dim)
        U, F = orc.entropy(dim, G, u, n)
        assert abs(F - U * (u[1:dim + 1] / u[0]) @ n) <= 1e-14 * abs(F) + 1e-15


@pytest.mark.parametrize("dim", [2, 3])
def test_ranocha_entropy_conservative(orc, dim):
    # Sec. 2, EC condition: (w(u+) - w(u-)).f - sum_j n_j (psi^j(u+) - psi^j(u-)) = 0
    # with psi^j = w.f^j - F^j = rho v_j for this entropy
    rng = np.random.default_rng(5)
    worst = 0.0
    for trial in range(2000):
        um, n = rand_state(rng, dim), rand_normal(rng, dim)
        if trial % 2:
            up = rand_state(rng, dim)
        else:  # near-equal states exercise the series branch of the log means
            up = um * (1 + rng.uniform(-1e-3, 1e-3, len(um)))
        f = orc.two_point("ranocha", dim, G, um, up, n)
        wp, wm = entropy_vars_ref(up), entropy_vars_ref(um)
        dpsi = (up[1:dim + 1] - um[1:dim + 1]) @ n
        # rounding scale: w(u+) - w(u-) cancels for near-equal states
        scale = np.abs(wp * f).sum() + np.abs(wm * f).sum() + np.abs(up[1:dim + 1] @ n) + np.abs(um[1:dim + 1] @ n)
        worst = max(worst, abs((wp - wm) @ f - dpsi) / scale)
    assert worst < 1e-13, worst
    # the Shima flux is not entropy conservative (no logarithmic mean)
    um, up, n = cons(1.0, [0.1] * dim, 1.0), cons(2.0, [-0.2] * dim, 0.5), np.ones(dim)
    f = orc.two_point("shima", dim, G, um, up, n)
    assert abs((entropy_vars_ref(up) - entropy_vars_ref(um)) @ f - (up[1:dim + 1] - um[1:dim + 1]) @ n) > 1e-3


@pytest.mark.parametrize("kind", ["ranocha", "shima"])
@pytest.mark.parametrize("dim", [2, 3])
def test_pressure_equilibrium_form(orc, kind, dim):
    # both fluxes are PEP (Sec. 3.2): for equal v and p,
    # f = (m, v m + p n, |v|^2 m / 2 + gamma/(gamma-1) p v.n) with m = f_rho
    rng = np.random.default_rng(6)
    for _ in range(200):
        v, p, n = rng.uniform(-1, 1, dim), rng.uniform(0.5, 3), rand_normal(rng, dim)
        r1, r2 = rng.uniform(0.3, 3, 2)
        f = orc.two_point(kind, dim, G, cons(r1, v, p), cons(r2, v, p), n)
        m = f[0]
        rho_mean = (r2 - r1) / (np.log(r2) - np.log(r1)) if kind == "ranocha" else 0.5 * (r1 + r2)
        assert abs(m - rho_mean * (v @ n)) <= 1e-13 * max(1, abs(m))
        ref = np.concatenate([[m], v * m + p * n, [0.5 * (v @ v) * m + G / (G - 1) * p * (v @ n)]])
        assert np.allclose(f, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("dim", [2, 3])
def test_llf_dissipative_and_closed_form(orc, dim):
    rng = np.random.default_rng(8)
    for _ in range(500):
        um, n = rand_state(rng, dim), rand_normal(rng, dim)
        up = um * (1 + rng.uniform(-0.05, 0.05, len(um)))
        f = orc.two_point("llf", dim, G, um, up, n)
        dw = entropy_vars_ref(up) - entropy_vars_ref(um)
        dpsi = (up[1:dim + 1] - um[1:dim + 1]) @ n
        assert dw @ f - dpsi <= 1e-13 * np.abs(dw * f).sum()
    # resting contact: v = 0, equal p -> (-lam/2 [rho], p n, -lam/2 [rho e])
    n = np.array([0.3, -0.4, 1.2][:dim])
    p = 1.7
    um, up = cons(1.0, np.zeros(dim), p), cons(2.5, np.zeros(dim), p)
    lam = np.sqrt(G * p / 1.0) * np.linalg.norm(n)
    f = orc.two_point("llf", dim, G, um, up, n)
    ref = np.concatenate([[-0.5 * lam * 1.5], p * n, [0.0]])
    assert np.allclose(f, ref, rtol=1e-14, atol=1e-14)
