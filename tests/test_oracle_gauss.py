"""Pins of the oracle's Legendre-Gauss collocation scheme (Sec. 6: hybridised
SBP operators with the entropy projection), each against something other than
the oracle: numpy's Gauss-Legendre rule, polynomial exactness, the
generalised SBP identity, the entropy-variable round trip, free-stream
preservation, discrete conservation, zero entropy production of the
entropy-conservative flux pair (the property the entropy projection exists
for), entropy dissipation with LLF, and design-order convergence to the exact
density wave."""
import numpy as np
import pytest

from paper_2112_10517_amd import inputs

GAMMA = 1.4


@pytest.mark.parametrize("p", range(0, 11))
def test_gauss_rule_matches_numpy(orc, p):
    xi, w, D, rL, rR = orc.gauss(p)
    xg, wg = np.polynomial.legendre.leggauss(p + 1)
    assert np.abs(xi - xg).max() < 4e-16 * (p + 1)
    assert np.abs(w - wg).max() < 4e-16 * (p + 1)
    # exact for polynomials of degree 2p+1
    for k in range(2 * p + 2):
        exact = (1.0 - (-1.0) ** (k + 1)) / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 1e-14 * (p + 1)


@pytest.mark.parametrize("p", range(1, 9))
def test_gauss_operators(orc, p):
    xi, w, D, rL, rR = orc.gauss(p)
    N = p + 1
    for k in range(N):
        deriv = k * xi ** (k - 1) if k else np.zeros(N)
        assert np.abs(D @ xi ** k - deriv).max() < 2e-13 * N * N
        assert abs(rL @ xi ** k - (-1.0) ** k) < 1e-13 * N
        assert abs(rR @ xi ** k - 1.0) < 1e-13 * N
    # generalised SBP: M D + (M D)^T = R^T B R
    M = np.diag(w)
    R = np.stack([rL, rR])
    B = np.diag([-1.0, 1.0])
    assert np.abs(M @ D + (M @ D).T - R.T @ B @ R).max() < 1e-13 * N * N


def test_entropy_variable_round_trip(orc):
    rng = np.random.default_rng(3)
    for dim in (2, 3):
        for _ in range(20):
            rho, p = rng.uniform(0.2, 3.0, 2)
            v = rng.uniform(-2, 2, dim)
            u = np.concatenate([[rho], rho * v, [p / (GAMMA - 1) + 0.5 * rho * v @ v]])
            w = orc.entropy_vars(dim, GAMMA, u)
            assert np.abs(orc.cons_from_entropy(dim, GAMMA, w) - u).max() < 1e-13 * np.abs(u).max()


CASES = [(2, 2, (4, 3)), (2, 4, (3, 2)), (3, 1, (3, 2, 2)), (3, 3, (2, 3, 2))]


@pytest.mark.parametrize("dim,p,n", CASES)
def test_free_stream(orc, dim, p, n):
    m = orc.Mesh(dim, p, n, vol_flux="ranocha", surf_flux="llf", nodes="gauss")
    v = np.array([0.3, -0.2, 0.1][:dim])
    u0 = np.concatenate([[1.3], 1.3 * v, [2.5 / (GAMMA - 1) + 0.5 * 1.3 * v @ v]])
    u = np.broadcast_to(u0[None, :, None], m.shape).copy()
    scale = m.rhs_scale(u)
    assert np.all(np.abs(m.rhs(u)) <= 1e-13 * scale.max())


@pytest.mark.parametrize("dim,p,n", CASES)
@pytest.mark.parametrize("vol,surf", [("ranocha", "ranocha"), ("shima", "llf")])
def test_conservation(orc, dim, p, n, vol, surf):
    m = orc.Mesh(dim, p, n, vol_flux=vol, surf_flux=surf, nodes="gauss")
    u = inputs.random_fourier(m.coords(), 4)
    du = m.rhs(u)
    _, J = m.metrics()
    JW = J * m.weights()[None, :]
    scale = np.einsum("en,evn->v", JW, m.rhs_scale(u))
    assert np.all(np.abs(np.einsum("en,evn->v", JW, du)) <= 1e-14 * scale)


@pytest.mark.parametrize("dim,p,n", CASES)
def test_entropy_conservative_pair(orc, dim, p, n):
    # Ranocha volume and surface fluxes with the entropy projection: zero
    # entropy production up to round-off; LLF at the surface dissipates
    m = orc.Mesh(dim, p, n, vol_flux="ranocha", surf_flux="ranocha", nodes="gauss")
    u = inputs.random_fourier(m.coords(), 5)
    du = m.rhs(u)
    _, J = m.metrics()
    JW = J * m.weights()[None, :]
    w = np.stack([orc.entropy_vars(dim, GAMMA, u[e, :, i]) for e in range(m.n_elem) for i in range(m.nodes)])
    w = w.reshape(m.n_elem, m.nodes, dim + 2).transpose(0, 2, 1)
    escale = np.sum(JW[:, None, :] * np.abs(w * du))
    assert abs(m.entropy_rate(u, du)) <= 1e-13 * escale
    m2 = orc.Mesh(dim, p, n, vol_flux="ranocha", surf_flux="llf", nodes="gauss")
    assert m2.entropy_rate(u) < -1e-6 * escale


@pytest.mark.parametrize("p", [2, 3])
def test_density_wave_convergence(orc, p):
    # rho = 1 + A sin(pi(x+y-2t)), v = (1,1), p = 1, one period (the setup of
    # the LGL convergence pin); LLF surface flux
    amp, t_end, v, p0 = 0.5, 1.0, (1.0, 1.0), 1.0
    errs = []
    for n in (4, 8, 16):
        m = orc.Mesh(2, p, (n, n), vol_flux="ranocha", surf_flux="llf", nodes="gauss")
        x = m.coords()
        u0 = inputs.density_wave(x, amp=amp, p0=p0, v=v)
        steps = int(np.ceil(t_end / m.max_dt(u0, 0.5)))
        u, t = m.rk4(u0, t_end / steps, steps)
        ex = inputs.density_wave(x, amp=amp, t=t, p0=p0, v=v)
        _, J = m.metrics()
        JW = J * m.weights()[None, :]
        errs.append(np.sqrt(np.sum(JW * (u[:, 0] - ex[:, 0]) ** 2) / np.sum(JW)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > p + 0.5, (errs, rates)


def test_gauss_rejects_curved_mesh(orc):
    with pytest.raises(ValueError):
        orc.Mesh(2, 2, (2, 2), warp=0.1, nodes="gauss")
