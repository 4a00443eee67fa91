"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

The bars (tests/parity.py): FP64 right-hand sides per conserved variable
max|gpu - oracle| <= max(1e-12 max|RHS_v|, 3e-14 max sigma_v), sigma_i the
oracle's sum of the magnitudes of the terms of RHS_i (Mesh.rhs_scale);
states after steps 1e-12 max|u_v| plus 3e-14 sigma times the integrated
time.  Every check records its R20 figure (max|d|/max|RHS| per variable),
printed in the session summary.  Inputs are seeded and synthetic; the oracle
never sees a GPU output.
"""
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


def rhs_parity(gpu, m, u, ref=None, label=""):
    """worst ratio of |gpu - oracle| to the FP64 bar over the variables (must be <= 1)."""
    ref = m.rhs(u) if ref is None else ref
    return parity.rhs64(gpu, ref, m.rhs_scale(u), label=label, u=u)


def state_parity(gpu, uo, m, u0, t_span, label=""):
    """worst ratio of |gpu - oracle| to the FP64 state bar after steps (must be <= 1)."""
    return parity.state64(gpu, uo, m.rhs_scale(u0), t_span, label=label, u0=u0)


def make_pair(orc, E, dim, p, n, warp=0.0, vol="ranocha", surf="llf", lo=None, hi=None):
    lo = lo or (-1.0,) * dim
    hi = hi or (1.0,) * dim
    m = orc.Mesh(dim, p, n, lo=lo, hi=hi, warp=warp, vol_flux=vol, surf_flux=surf)
    g = E.Problem(dim, p, n, lo=lo, hi=hi, warp=warp, volume_flux=vol, surface_flux=surf)
    return m, g


def noisy(u, seed, rel=0.01):
    rng = np.random.default_rng(seed)
    return u * (1 + rel * rng.standard_normal(u.shape))


def test_density_wave_2d_rhs_and_steps(orc, esdg):
    # 2D Euler, periodic affine [-1,1]^2, 8x8 elements, p=3, density wave,
    # Ranocha volume + LLF surface: one RHS and 10 RK4 steps with dt = 1e-3
    m, g = make_pair(orc, esdg, 2, 3, (8, 8))
    x = m.coords()
    assert np.abs(g.coords() - x).max() < 1e-14
    u = inputs.density_wave(x)
    g.set_state(u)
    assert rhs_parity(g.rhs(), m, u, label="2D density wave 8^2 p=3 rhs") <= 1.0
    t = g.step(dt=1e-3, nsteps=10, t=0.0)
    assert abs(t - 0.01) < 1e-15
    ug = g.get_state()
    uo, _ = m.rk4(u, 1e-3, 10)
    assert state_parity(ug, uo, m, u, 0.01, label="2D density wave 8^2 p=3 10 steps") <= 1.0
    g.sync()
    # positivity after the steps (rho_min = 0.02 initially)
    assert ug[:, 0].min() > 0


@pytest.mark.parametrize("vol", ["ranocha", "shima"])
def test_warped_3d_16cubed_rhs(orc, esdg, vol):
    # 3D Euler, warped periodic 16^3 on [-1,1]^3, p=3, smooth random state (seed 2)
    m, g = make_pair(orc, esdg, 3, 3, (16, 16, 16), warp=0.1, vol=vol)
    u = inputs.random_fourier(m.coords(), 2)
    g.set_state(u)
    du = g.rhs()
    assert rhs_parity(du, m, u, label="warped 16^3 p=3 %s rhs (headline)" % vol) <= 1.0
    # bitwise reproducible
    assert np.array_equal(du, g.rhs())


def test_warped_3d_16cubed_steps(orc, esdg):
    m, g = make_pair(orc, esdg, 3, 3, (16, 16, 16), warp=0.1, vol="ranocha")
    u = inputs.random_fourier(m.coords(), 2)
    g.set_state(u)
    dt = 0.5 * m.max_dt(u, 1.0)
    g.step(dt=dt, nsteps=3)
    uo, _ = m.rk4(u, dt, 3)
    assert state_parity(g.get_state(), uo, m, u, 3 * dt, label="warped 16^3 p=3 3 steps") <= 1.0


CASES = [
    # dim, p, n, warp, vol, surf
    (2, 1, (5, 3), 0.0, "ranocha", "llf"),
    (2, 2, (4, 4), 0.1, "shima", "llf"),
    (2, 4, (3, 5), 0.1, "ranocha", "ranocha"),
    (2, 5, (2, 3), 0.0, "central", "central"),
    (2, 6, (3, 2), 0.1, "ranocha", "shima"),
    (2, 7, (2, 2), 0.1, "shima", "central"),
    (3, 1, (3, 4, 2), 0.1, "ranocha", "llf"),
    (3, 2, (2, 3, 4), 0.0, "shima", "ranocha"),
    (3, 3, (3, 2, 5), 0.1, "central", "llf"),
    (3, 4, (2, 2, 3), 0.1, "ranocha", "llf"),
    (3, 5, (2, 3, 2), 0.0, "ranocha", "ranocha"),
    (3, 6, (2, 2, 2), 0.1, "shima", "shima"),
    (3, 7, (2, 1, 2), 0.1, "ranocha", "llf"),
    (3, 7, (2, 2, 1), 0.0, "ranocha", "ranocha"),
    (3, 7, (1, 2, 2), 0.1, "central", "central"),
    (3, 7, (2, 2, 2), 0.0, "shima", "llf"),
    (3, 3, (1, 1, 1), 0.0, "ranocha", "llf"),   # element is its own neighbour
    (2, 3, (1, 7), 0.1, "ranocha", "llf"),
]


@pytest.mark.parametrize("dim,p,n,warp,vol,surf", CASES)
def test_rhs_parity_matrix(orc, esdg, dim, p, n, warp, vol, surf):
    lo = tuple([-1.0, -0.5, 0.0][:dim])
    hi = tuple([1.0, 1.5, 1.0][:dim])
    m, g = make_pair(orc, esdg, dim, p, n, warp=warp, vol=vol, surf=surf, lo=lo, hi=hi)
    u = noisy(inputs.random_fourier(m.coords(), 7, lo=lo, hi=hi), 3)
    g.set_state(u)
    assert rhs_parity(g.rhs(), m, u, label="matrix %dD p=%d %s warp %.1f %s/%s" % (dim, p, n, warp, vol, surf)) <= 1.0


@pytest.mark.parametrize("warp", [0.0, 0.1])
def test_reductions(orc, esdg, warp):
    m, g = make_pair(orc, esdg, 3, 3, (4, 3, 5), warp=warp, vol="ranocha", surf="ranocha")
    u = noisy(inputs.random_fourier(m.coords(), 4), 5)
    g.set_state(u)
    tot = g.totals()
    ref = m.totals(u)
    _, J = m.metrics()
    JW = J * m.weights()[None, :]
    scale = np.einsum("en,evn->v", JW, np.abs(u))
    assert np.all(np.abs(tot - ref) <= 1e-13 * scale)
    # entropy conservative volume + surface flux: dS/dt = 0 to round-off
    du = m.rhs(u)
    w = np.stack([orc.entropy_vars(3, 1.4, u[e, :, i]) for e in range(m.n_elem) for i in range(m.nodes)])
    w = w.reshape(m.n_elem, m.nodes, 5).transpose(0, 2, 1)
    escale = np.sum(JW[:, None, :] * np.abs(w * du))
    rate = g.entropy_rate()
    assert abs(rate) < 1e-13 * escale
    assert abs(rate - m.entropy_rate(u, du)) < 1e-13 * escale
    assert abs(g.max_dt(0.7) - m.max_dt(u, 0.7)) < 1e-13 * m.max_dt(u, 0.7)


def test_llf_entropy_dissipation_and_cfl_steps(orc, esdg):
    m, g = make_pair(orc, esdg, 2, 3, (6, 5), warp=0.1, vol="ranocha", surf="llf")
    u = noisy(inputs.random_fourier(m.coords(), 8), 9)
    g.set_state(u)
    rate = g.entropy_rate()
    ref = m.entropy_rate(u)
    assert rate < 0 and abs(rate - ref) < 1e-12 * abs(ref)
    t = g.step(dt=0.0, nsteps=4, cfl=0.5, t=1.0)
    uo, to = m.rk4(u, 0.0, 4, cfl=0.5, t=1.0)
    assert abs(t - to) < 1e-13
    assert state_parity(g.get_state(), uo, m, u, to - 1.0, label="2D warped LLF 4 CFL steps") <= 1.0


@pytest.mark.parametrize("p", [3, 5])
def test_cfl_steps_across_calls(orc, esdg, p):
    # the CFL step of a step's start state is carried over between calls and
    # recomputed after set_state; both paths must equal the oracle's CFL steps
    # (p = 3: line layout; p = 5: node layout, by default)
    m, g = make_pair(orc, esdg, 3, p, (3, 4, 2), warp=0.1, vol="ranocha", surf="llf")
    u = noisy(inputs.random_fourier(m.coords(), 12), 13)
    g.set_state(u)
    t = g.step(dt=0.0, nsteps=2, cfl=0.4, t=0.0)
    t = g.step(dt=0.0, nsteps=3, cfl=0.4, t=t)
    uo, to = m.rk4(u, 0.0, 5, cfl=0.4)
    assert abs(t - to) < 1e-13 * to
    assert state_parity(g.get_state(), uo, m, u, to, label="p=%d CFL steps across calls" % p) <= 1.0
    # fixed-dt step in between, then CFL again (state changed: recomputed)
    g.step(dt=1e-4, nsteps=1)
    uo, _ = m.rk4(uo, 1e-4, 1)
    t2 = g.step(dt=0.0, nsteps=2, cfl=0.3, t=0.0)
    uo, to2 = m.rk4(uo, 0.0, 2, cfl=0.3)
    assert abs(t2 - to2) < 1e-13 * to2
    assert state_parity(g.get_state(), uo, m, u, to + 1e-4 + to2, label="p=%d CFL, fixed, CFL steps" % p) <= 1.0
    # a new state invalidates the carried CFL value
    g.set_state(u)
    t3 = g.step(dt=0.0, nsteps=1, cfl=0.4, t=0.0)
    assert abs(t3 - m.max_dt(u, 0.4)) < 1e-13 * t3


def test_free_stream_gpu(esdg):
    g = esdg.Problem(3, 4, (4, 3, 5), warp=0.1, volume_flux="ranocha", surface_flux="llf")
    u = np.zeros(g.shape)
    u[:, 0] = 1.3
    u[:, 1], u[:, 2], u[:, 3] = 1.3 * 0.3, -1.3 * 0.2, 1.3 * 0.1
    u[:, 4] = 2.0 / 0.4 + 0.5 * 1.3 * 0.14
    g.set_state(u)
    du = g.rhs()
    # flux scale (rho e + p)|v| |Ja|/J (p+1)^2 ~ 1e3 on this mesh
    assert np.abs(du).max() < 1e-10


def test_device_pointers(orc, esdg):
    import torch
    m, g = make_pair(orc, esdg, 3, 2, (3, 3, 3), warp=0.1)
    u = inputs.random_fourier(m.coords(), 1)
    ud = torch.from_numpy(u).cuda()
    g.set_state(ud)
    out = torch.empty_like(ud)
    g.rhs(out)
    torch.cuda.synchronize()
    assert rhs_parity(out.cpu().numpy(), m, u, label="device pointers 3^3 p=2") <= 1.0
    back = torch.empty_like(ud)
    g.get_state(back)
    torch.cuda.synchronize()
    assert np.array_equal(back.cpu().numpy(), u)


def test_error_paths(esdg):
    g = esdg.Problem(2, 3, (2, 2))
    with pytest.raises(esdg.EsdgError) as ei:
        g.rhs()
    assert ei.value.status == esdg.ESTATE
    with pytest.raises(esdg.EsdgError) as ei:
        esdg.Problem(2, 9, (2, 2))
    assert ei.value.status == esdg.EINVAL
    good = inputs.density_wave(g.coords())
    u = good.copy()
    u[0, 0, 3] = -1.0  # negative density
    g.set_state(u)
    g.rhs()
    with pytest.raises(esdg.NonPhysicalState):
        g.sync()
    g.sync()  # flag cleared by reporting it
    # esdg_step reports a flag raised by earlier work and enqueues nothing
    g.rhs()
    with pytest.raises(esdg.NonPhysicalState):
        g.step(dt=1e-4, nsteps=1)
    assert np.array_equal(g.get_state(), u)
    g.sync()
    # ... and its own kernels' flag when it synchronises (t given)
    with pytest.raises(esdg.NonPhysicalState):
        g.step(dt=1e-4, nsteps=1, t=0.0)
    g.sync()
    # the reductions report it after writing their result
    with pytest.raises(esdg.NonPhysicalState):
        g.entropy_rate()
    g.sync()
    # a good state again: nothing to report
    g.set_state(good)
    g.step(dt=1e-4, nsteps=2, t=0.0)
    g.totals()
    g.sync()
    # a batch refuses to step while a member is flagged; sync names the member
    h = esdg.Problem(2, 3, (2, 2))
    h.set_state(good)
    g.set_state(u)
    g.rhs()
    with esdg.Batch([h, g]) as B:
        with pytest.raises(esdg.NonPhysicalState):
            B.step(dt=1e-4, nsteps=1)
        with pytest.raises(esdg.NonPhysicalState) as ei:
            B.sync()
        assert "member 1" in str(ei.value)
        B.sync()
    g.close()
    h.close()


@pytest.mark.parametrize("dim,warp,vol", [(2, 0.0, "ranocha"), (2, 0.1, "shima"), (3, 0.0, "ranocha"),
                                          (3, 0.1, "ranocha"), (3, 0.1, "shima")])
def test_isentropic_vortex_parity(orc, esdg, dim, warp, vol):
    # the timing workload of Sec. 4.1: vortex of strength 20 on [-5,5]^d, 8
    # elements per direction, p = 3, the same flux in the volume and at the
    # faces; its log means take both branches
    lo, hi = (-5.0,) * dim, (5.0,) * dim
    m, g = make_pair(orc, esdg, dim, 3, (8,) * dim, warp=warp, vol=vol, surf=vol, lo=lo, hi=hi)
    u = inputs.isentropic_vortex(m.coords())
    g.set_state(u)
    assert rhs_parity(g.rhs(), m, u, label="vortex %dD warp %.1f %s" % (dim, warp, vol)) <= 1.0
    if vol == "ranocha":
        # entropy conservative in the volume and at the faces: dS/dt = 0 to
        # round-off, on the scale sum J W |w . du|
        du = m.rhs(u)
        nv = dim + 2
        w = np.stack([orc.entropy_vars(dim, 1.4, u[e, :, i]) for e in range(m.n_elem) for i in range(m.nodes)])
        w = w.reshape(m.n_elem, m.nodes, nv).transpose(0, 2, 1)
        _, J = m.metrics()
        escale = np.sum((J * m.weights()[None, :])[:, None, :] * np.abs(w * du))
        rate = g.entropy_rate()
        assert abs(rate) < 1e-13 * escale and abs(rate - m.entropy_rate(u, du)) < 1e-13 * escale


@pytest.mark.parametrize("p,n,warp,variant", [(5, (2, 3, 2), 0.1, 3), (7, (2, 2, 2), 0.0, 3), (7, (2, 1, 2), 0.1, 3),
                                               (7, (2, 2, 2), 0.0, 4), (7, (2, 1, 2), 0.1, 4), (4, (3, 2, 1), 0.1, 4),
                                               (5, (1, 2, 3), 0.1, 4), (6, (2, 1, 2), 0.0, 4), (6, (1, 2, 2), 0.1, 4)])
def test_entropy_conservation_node_layout(orc, esdg, p, n, warp, variant):
    """Entropy-conservative volume and surface fluxes in the node layout
    (tile variant 3, one lane per node; every pair evaluated from both of its
    nodes) and the pair layout (variant 4; each pair evaluated by one lane and
    handed to its partner): the right-hand side matches the oracle and
    dS/dt = 0 to round-off on the scale sum J W |w . du| -- the pair fluxes
    of the two ends must cancel as exactly as the line layout's."""
    m, g = make_pair(orc, esdg, 3, p, n, warp=warp, vol="ranocha", surf="ranocha")
    u = noisy(inputs.random_fourier(m.coords(), 8), 6)
    g.set_state(u)
    v_before = g.tile_variant()[0]
    try:
        g.set_tile_variant(variant)
        assert rhs_parity(g.rhs(), m, u, label="variant %d EC p=%d warp %.1f" % (variant, p, warp)) <= 1.0
        du = m.rhs(u)
        w = np.stack([orc.entropy_vars(3, 1.4, u[e, :, i]) for e in range(m.n_elem) for i in range(m.nodes)])
        w = w.reshape(m.n_elem, m.nodes, 5).transpose(0, 2, 1)
        _, J = m.metrics()
        escale = np.sum((J * m.weights()[None, :])[:, None, :] * np.abs(w * du))
        rate = g.entropy_rate()
        print("p=%d warp=%.1f variant %d: entropy rate %.3e (relative %.3e)"
              % (p, warp, variant, rate, abs(rate) / escale))
        assert abs(rate) < 1e-13 * escale and abs(rate - m.entropy_rate(u, du)) < 1e-13 * escale
    finally:
        g.set_tile_variant(v_before)


PAIR_CASES = [
    # below p = 7 the last workgroup is partly filled where the element
    # count is not a multiple of the tile's (p = 1: 16, 2: 7, 3: 4, 4: 2)
    (1, (3, 2, 3), 0.1, "ranocha", "llf"),
    (2, (2, 5, 1), 0.1, "ranocha", "ranocha"),
    (3, (3, 1, 2), 0.0, "shima", "llf"),
    (4, (3, 1, 1), 0.1, "ranocha", "llf"),
    (5, (2, 1, 2), 0.1, "ranocha", "ranocha"),
    (6, (1, 2, 2), 0.0, "central", "llf"),
    (6, (2, 1, 1), 0.1, "ranocha", "llf"),     # FP64 curved at p = 6: one z-plane per wave
    (6, (1, 1, 3), 0.1, "shima", "ranocha"),
    (7, (2, 1, 2), 0.1, "ranocha", "llf"),
    (7, (2, 2, 1), 0.0, "ranocha", "ranocha"),
    (7, (1, 2, 2), 0.1, "central", "central"),
    (7, (2, 2, 2), 0.0, "shima", "llf"),
    (7, (3, 1, 1), 0.1, "shima", "ranocha"),
]


@pytest.mark.parametrize("p,n,warp,vol,surf", PAIR_CASES)
def test_pair_layout_parity(orc, esdg, p, n, warp, vol, surf):
    """Pair layout (tile variant 4): right-hand side and three CFL steps
    against the oracle (FP64 bars), on seams of periodic boxes one to five
    elements wide in each direction, degrees 1 to 7."""
    m, g = make_pair(orc, esdg, 3, p, n, warp=warp, vol=vol, surf=surf)
    u = noisy(inputs.random_fourier(m.coords(), 12), 13)
    g.set_state(u)
    v_before = g.tile_variant()[0]
    try:
        g.set_tile_variant(4)
        assert g.tile_variant()[0] == 4
        assert rhs_parity(g.rhs(), m, u, label="pair layout p=%d %s %s/%s" % (p, n, vol, surf)) <= 1.0
        t = g.step(nsteps=3, cfl=0.3, t=0.0)
        uo, to = m.rk4(u, 0.0, 3, cfl=0.3)
        assert abs(t - to) <= 1e-14 * to
        assert state_parity(g.get_state(), uo, m, u, to, label="pair layout p=%d %s 3 CFL steps" % (p, n)) <= 1.0
    finally:
        g.set_tile_variant(v_before)


@pytest.mark.parametrize("prec,cfl", [("fp64", False), ("fp32", False), ("fp64", True), ("fp32", True)])
def test_checkpoint_resume_bitwise(esdg, prec, cfl):
    # the state and time read through the ABI (FP64, canonical layout) are the
    # checkpoint: 10 steps equal 5 steps, checkpoint, a new handle restored
    # from it, 5 more steps -- bit for bit, with fixed dt and in CFL mode
    kw = dict(warp=0.1, volume_flux="ranocha", surface_flux="llf", precision=prec)
    a = esdg.Problem(3, 3, (3, 4, 2), **kw)
    u = noisy(inputs.random_fourier(a.coords(), 3), 4)
    a.set_state(u)
    dt = 0.0 if cfl else 0.5 * a.max_dt(0.5)
    a.step(dt=dt, nsteps=10, cfl=0.5, t=0.0)
    u10, t10 = a.get_state(), a.get_time()
    b = esdg.Problem(3, 3, (3, 4, 2), **kw)
    b.set_state(u)
    b.step(dt=dt, nsteps=5, cfl=0.5, t=0.0)
    ck_u, ck_t = b.get_state(), b.get_time()
    b.close()
    c = esdg.Problem(3, 3, (3, 4, 2), **kw)
    c.set_state(ck_u)
    c.set_time(ck_t)
    c.step(dt=dt, nsteps=5, cfl=0.5)
    assert c.get_time() == t10
    assert np.array_equal(c.get_state(), u10)


@pytest.mark.parametrize("dim,p,n,warp,prec", [(3, 3, (2, 3, 2), 0.1, "fp64"), (3, 7, (2, 1, 2), 0.1, "fp64"),
                                               (3, 4, (3, 2, 2), 0.1, "fp32"), (2, 5, (3, 4), 0.1, "fp64"),
                                               (3, 3, (2, 3, 4), 0.0, "fp64")])
def test_inv_jacobian(orc, esdg, dim, p, n, warp, prec):
    """esdg_get_inv_jacobian returns the 1/J the kernels use: against the
    oracle's independent geometry (own LGL construction and metric
    evaluation, R1 and R10); FP32 mode returns the FP32-rounded values; an
    affine box the constant 1 / prod(h/2).  Independently of the oracle,
    sum_i W_i J_i is the box volume 2^dim to round-off: the warp adds one
    scalar phi to every coordinate, so the collocation Jacobian is
    prod(h/2) (1 + sum_k D_k phi), and by the SBP property the weighted sum of
    D_k phi over an element is a difference of face values, which cancels
    over the periodic mesh."""
    m = orc.Mesh(dim, p, n, warp=warp)
    g = esdg.Problem(dim, p, n, warp=warp, precision=prec)
    try:
        inv_j = g.inv_jacobian()
        _, J = m.metrics()
        assert inv_j.shape == J.shape
        tol = 1e-12 if prec == "fp64" else 2.0 ** -23
        np.testing.assert_allclose(inv_j * J, 1.0, rtol=0, atol=tol)
        vol = np.sum(m.weights()[None, :] / inv_j)
        assert abs(vol - 2.0 ** dim) < (1e-12 if prec == "fp64" else 1e-6) * 2.0 ** dim, vol
        if warp == 0.0:
            h = [2.0 / k for k in n]
            assert np.all(inv_j == 1.0 / np.prod([0.5 * x for x in h]))
    finally:
        g.close()
