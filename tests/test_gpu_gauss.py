"""Legendre-Gauss collocation with entropy projection (Sec. 6) on the GPU
against the oracle: right-hand sides to the FP64 parity bar of the LGL path
(and the FP32 bar for FP32 bulk), RK4 states, the zero entropy production of
the entropy-conservative flux pair, and Gauss problems in a batch
(bit-identical alone)."""
import numpy as np
import pytest

from paper_2112_10517_amd import inputs

import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def esdg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2112_10517_amd import esdg as E
    E.load_library()
    return E


CASES = [
    (2, 1, (4, 3), "ranocha", "llf"),
    (2, 3, (3, 2), "shima", "ranocha"),
    (2, 5, (2, 3), "central", "central"),
    (2, 7, (2, 2), "ranocha", "shima"),
    (3, 2, (3, 2, 3), "ranocha", "llf"),
    (3, 3, (2, 3, 2), "ranocha", "ranocha"),
    (3, 4, (2, 2, 3), "shima", "llf"),
    (3, 6, (2, 2, 2), "ranocha", "llf"),
    (3, 7, (2, 1, 2), "ranocha", "ranocha"),
    (3, 3, (1, 1, 1), "ranocha", "llf"),  # element is its own neighbour
]


def pair(orc, esdg, dim, p, n, vol, surf, prec="fp64", lo=None, hi=None):
    kw = {}
    if lo is not None:
        kw = dict(lo=lo, hi=hi)
    m = orc.Mesh(dim, p, n, vol_flux=vol, surf_flux=surf, nodes="gauss", **kw)
    g = esdg.Problem(dim, p, n, volume_flux=vol, surface_flux=surf, nodes="gauss", precision=prec, **kw)
    return m, g


def fp64_parity(d, ref, sigma, label, u=None):
    assert parity.rhs64(d, ref, sigma, label=label, u=u) <= 1.0


@pytest.mark.parametrize("dim,p,n,vol,surf", CASES)
def test_gauss_rhs_parity(orc, esdg, dim, p, n, vol, surf):
    lo = tuple([-1.0, -0.5, 0.0][:dim])
    hi = tuple([1.0, 1.5, 1.0][:dim])
    m, g = pair(orc, esdg, dim, p, n, vol, surf, lo=lo, hi=hi)
    x = m.coords()
    assert np.abs(g.coords() - x).max() < 1e-15
    u = inputs.random_fourier(x, 7, lo=lo, hi=hi)
    g.set_state(u)
    fp64_parity(g.rhs(), m.rhs(u), m.rhs_scale(u), "gauss %dD p=%d %s %s/%s" % (dim, p, n, vol, surf), u=u)


@pytest.mark.parametrize("dim,p,n,vol,surf", [CASES[1], CASES[5], CASES[7]])
def test_gauss_fp32_rhs(orc, esdg, dim, p, n, vol, surf):
    m, g = pair(orc, esdg, dim, p, n, vol, surf, prec="fp32")
    u = inputs.random_fourier(m.coords(), 8)
    g.set_state(u)
    ref, sigma = m.rhs(u), m.rhs_scale(u)
    d = g.rhs()
    ws = parity.rhs32(d, ref, sigma, label="gauss fp32 %dD p=%d" % (dim, p))
    assert ws <= parity.SIGMA32


def test_gauss_steps_parity(orc, esdg):
    m, g = pair(orc, esdg, 3, 3, (3, 2, 3), "ranocha", "llf")
    u = inputs.random_fourier(m.coords(), 9)
    g.set_state(u)
    dt = 0.5 * m.max_dt(u, 0.5)
    g.step(dt=dt, nsteps=10)
    uo, _ = m.rk4(u, dt, 10)
    ug = g.get_state()
    sigma0 = m.rhs_scale(u)
    assert parity.state64(ug, uo, sigma0, 10 * dt, label="gauss 3D p=3 10 steps", u0=u) <= 1.0
    # CFL steps advance with the Gauss weights' CFL value of the oracle
    g.set_state(u)
    t = g.step(dt=0.0, nsteps=3, cfl=0.4, t=0.0)
    uo, to = m.rk4(u, 0.0, 3, cfl=0.4)
    assert abs(t - to) <= 1e-13 * to
    assert parity.state64(g.get_state(), uo, sigma0, to, label="gauss 3D p=3 3 CFL steps", u0=u) <= 1.0


@pytest.mark.parametrize("dim,p,n", [(2, 3, (3, 3)), (3, 4, (2, 2, 2))])
def test_gauss_entropy_conservation(orc, esdg, dim, p, n):
    m, g = pair(orc, esdg, dim, p, n, "ranocha", "ranocha")
    u = inputs.random_fourier(m.coords(), 10)
    g.set_state(u)
    du = m.rhs(u)
    _, J = m.metrics()
    JW = J * m.weights()[None, :]
    w = np.stack([orc.entropy_vars(dim, 1.4, u[e, :, i]) for e in range(m.n_elem) for i in range(m.nodes)])
    w = w.reshape(m.n_elem, m.nodes, dim + 2).transpose(0, 2, 1)
    escale = np.sum(JW[:, None, :] * np.abs(w * du))
    rate = g.entropy_rate()
    print("gauss EC entropy rate %.3e (relative %.3e)" % (rate, abs(rate) / escale))
    assert abs(rate) <= 1e-12 * escale
    assert np.all(np.abs(g.totals() - m.totals(u)) <= 1e-13 * np.abs(m.totals(np.abs(u))))


def test_gauss_in_batch_matches_alone(esdg):
    specs = [dict(dim=3, p=3, n=(3, 2, 3), nodes="gauss"), dict(dim=3, p=3, n=(3, 2, 3)),
             dict(dim=3, p=5, n=(2, 2, 2), nodes="gauss", precision="fp32"), dict(dim=2, p=4, n=(3, 3), nodes="gauss")]
    a, b = [], []
    for i, s in enumerate(specs):
        for lst in (a, b):
            q = esdg.Problem(**s)
            q.set_state(inputs.random_fourier(q.coords(), 20 + i))
            lst.append(q)
    with esdg.Batch(a, graphs=True) as B:
        assert B.info()[0] == 4
        B.step(nsteps=3, cfl=0.3)
        t = B.times()
    for q, r, tq in zip(a, b, t):
        tr = r.step(nsteps=3, cfl=0.3, t=0.0)
        assert tr == tq
        assert np.array_equal(q.get_state(), r.get_state())


def test_gauss_rejects_curved_mesh(esdg):
    with pytest.raises(esdg.EsdgError) as ei:
        esdg.Problem(3, 3, (2, 2, 2), warp=0.1, nodes="gauss")
    assert "affine" in str(ei.value)
