"""FP32 bulk precision and full-size (32^3, p = 4 and 7) FP64 parity on the GPU.

FP32 bar: per conserved variable, max|gpu32 - oracle64| <= 1e-6 max sigma_v,
with sigma the oracle's per-node sum of term magnitudes (Mesh.rhs_scale): the
FP32 analogue of the FP64 bar, about 17 units of FP32 round-off of the sums
(measured 0.5e-7 .. 1.2e-7 sigma).  Reductions stay FP64 on the device.  The
measured L2 / Linf errors against the FP64 oracle are printed (`-s`) for
every case.
"""
import numpy as np
import pytest

from paper_2112_10517_amd import inputs

import parity

pytestmark = pytest.mark.gpu

TOL32 = parity.SIGMA32


@pytest.fixture(scope="module")
def esdg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2112_10517_amd import esdg as E
    E.load_library()
    return E


def errors(gpu, ref, sigma, label=""):
    """(max over v of max|d| / max sigma_v, L2 relative, Linf relative per variable max)."""
    d = np.asarray(gpu) - ref
    worst_sigma = parity.rhs32(gpu, ref, sigma, label=label)
    l2 = np.sqrt(np.mean(d ** 2)) / np.sqrt(np.mean(ref ** 2))
    linf = max(np.abs(d[:, v]).max() / np.abs(ref[:, v]).max() for v in range(ref.shape[1]))
    return worst_sigma, l2, linf


CASES32 = [
    (2, 3, (8, 8), 0.0, "ranocha", "llf", "density_wave"),
    (3, 3, (16, 16, 16), 0.1, "ranocha", "llf", "random"),
    (3, 3, (6, 5, 4), 0.1, "shima", "llf", "random"),
    (3, 4, (8, 8, 8), 0.1, "ranocha", "ranocha", "density_wave"),
    (3, 7, (4, 4, 4), 0.1, "ranocha", "llf", "density_wave"),
    (3, 7, (3, 4, 2), 0.0, "shima", "shima", "random"),
]


@pytest.mark.parametrize("dim,p,n,warp,vol,surf,state", CASES32)
def test_fp32_rhs_vs_fp64_oracle(orc, esdg, dim, p, n, warp, vol, surf, state):
    m = orc.Mesh(dim, p, n, warp=warp, vol_flux=vol, surf_flux=surf)
    x = m.coords()
    u = inputs.density_wave(x) if state == "density_wave" else inputs.random_fourier(x, 5)
    ref, sigma = m.rhs(u), m.rhs_scale(u)
    g = esdg.Problem(dim, p, n, warp=warp, volume_flux=vol, surface_flux=surf, precision="fp32")
    g.set_state(u)
    ws, l2, linf = errors(g.rhs(), ref, sigma, "fp32 %dD p=%d %s %s/%s %s" % (dim, p, n, vol, surf, state))
    print("fp32 %dD p=%d %s %s/%s %s: err/sigma %.2e  L2 %.2e  Linf %.2e" % (dim, p, n, vol, surf, state, ws, l2, linf))
    assert ws <= TOL32
    # the FP32 state round-trips through the FP64 ABI to FP32 rounding
    assert np.abs(g.get_state() - u).max() <= 2 ** -23 * np.abs(u).max()


def test_fp32_reductions_are_fp64(orc, esdg):
    m = orc.Mesh(3, 4, (4, 3, 5), warp=0.1, vol_flux="ranocha", surf_flux="ranocha")
    u = inputs.random_fourier(m.coords(), 6)
    u32 = u.astype(np.float32).astype(np.float64)  # the state the FP32 problem holds
    g = esdg.Problem(3, 4, (4, 3, 5), warp=0.1, volume_flux="ranocha", surface_flux="ranocha", precision="fp32")
    g.set_state(u)
    _, J = m.metrics()
    JW = J * m.weights()[None, :]
    scale = np.einsum("en,evn->v", JW, np.abs(u32))
    # totals of the FP32 state, summed in FP64 (metric weights J in FP32 -> 1e-7)
    assert np.all(np.abs(g.totals() - m.totals(u32)) <= 2e-7 * scale)
    # discrete entropy-rate residual of the EC discretisation in FP32
    du = m.rhs(u32)
    w = np.stack([orc.entropy_vars(3, 1.4, u32[e, :, i]) for e in range(m.n_elem) for i in range(m.nodes)])
    w = w.reshape(m.n_elem, m.nodes, 5).transpose(0, 2, 1)
    escale = np.sum(JW[:, None, :] * np.abs(w * du))
    rate = g.entropy_rate()
    print("fp32 EC entropy-rate residual %.3e (relative %.3e)" % (rate, abs(rate) / escale))
    assert abs(rate) <= 1e-5 * escale


def test_fp32_density_wave_error(esdg):
    # solution error against the exact density wave after RK4 steps:
    # FP32 bulk must not be dominated by round-off at this resolution
    dim, p, n, warp = 3, 4, (6, 6, 6), 0.1
    errs = {}
    for prec in ("fp64", "fp32"):
        g = esdg.Problem(dim, p, n, warp=warp, volume_flux="ranocha", surface_flux="llf", precision=prec)
        x = g.coords()
        u0 = inputs.density_wave(x, amp=0.5)
        g.set_state(u0)
        t = g.step(dt=0.0, nsteps=20, cfl=0.5, t=0.0)
        ex = inputs.density_wave(x, amp=0.5, t=t)
        errs[prec] = np.abs(g.get_state()[:, 0] - ex[:, 0]).max()
    print("density wave rho Linf error after 20 CFL-0.5 steps: fp64 %.3e fp32 %.3e" % (errs["fp64"], errs["fp32"]))
    assert errs["fp32"] <= 1.5 * errs["fp64"] + 1e-6


def sampled_elements(n, count, seed):
    E = n ** 3
    rng = np.random.default_rng(seed)
    corners = [0, n - 1, n * (n - 1), E - 1, E // 2]  # seams and corners of the periodic box
    return np.unique(np.concatenate([corners, rng.choice(E, count, replace=False)]))


@pytest.mark.parametrize("p", [4, 7])
def test_precision_sweep_32cubed(orc, esdg, p):
    """3D density wave on the warped 32^3 mesh: FP64 parity on sampled
    elements at full size, FP32 errors against it, FP32 entropy residual."""
    n = 32
    g64 = esdg.Problem(3, p, (n, n, n), warp=0.1, volume_flux="ranocha", surface_flux="llf")
    x = g64.coords()
    u = inputs.density_wave(x)
    g64.set_state(u)
    d64 = g64.rhs()
    m = orc.Mesh(3, p, (n, n, n), warp=0.1, vol_flux="ranocha", surf_flux="llf")
    el = sampled_elements(n, 40, p)
    ref, sigma = m.rhs_elements(u, el)
    del m
    assert parity.rhs64(d64[el], ref, sigma, label="32^3 p=%d density wave, %d sampled elements" % (p, len(el)),
                        u=u) <= 1.0
    g32 = esdg.Problem(3, p, (n, n, n), warp=0.1, volume_flux="ranocha", surface_flux="llf", precision="fp32")
    g32.set_state(u)
    d32 = g32.rhs()
    ws, l2, linf = errors(d32[el], ref, sigma, "fp32 32^3 p=%d density wave, sampled elements" % p)
    l2_full = np.sqrt(np.mean((d32 - d64) ** 2)) / np.sqrt(np.mean(d64 ** 2))
    print("32^3 p=%d density wave: fp32 err/sigma %.2e, L2 (full mesh vs fp64) %.2e, Linf %.2e"
          % (p, ws, l2_full, linf))
    assert ws <= TOL32
    # ten RK4 steps in both precisions from the same state
    dt = 0.5 * g64.max_dt(0.5)
    g64.step(dt=dt, nsteps=10)
    g32.step(dt=dt, nsteps=10)
    s64, s32 = g64.get_state(), g32.get_state()
    serr = max(np.abs(s32[:, v] - s64[:, v]).max() / np.abs(s64[:, v]).max() for v in range(5))
    print("32^3 p=%d: state after 10 steps fp32 vs fp64, max relative %.2e" % (p, serr))
    assert serr <= 1e-5
    g64.close()
    g32.close()


@pytest.mark.parametrize("dim,warp", [(2, 0.0), (3, 0.1)])
def test_fp32_isentropic_vortex(orc, esdg, dim, warp):
    # Sec. 4.1 vortex (both log-mean branches) in FP32 bulk against the FP64 oracle
    lo, hi = (-5.0,) * dim, (5.0,) * dim
    n = (8,) * dim
    m = orc.Mesh(dim, 3, n, lo=lo, hi=hi, warp=warp, vol_flux="ranocha", surf_flux="ranocha")
    u = inputs.isentropic_vortex(m.coords())
    ref, sigma = m.rhs(u), m.rhs_scale(u)
    g = esdg.Problem(dim, 3, n, lo=lo, hi=hi, warp=warp, volume_flux="ranocha", surface_flux="ranocha",
                     precision="fp32")
    g.set_state(u)
    ws, l2, linf = errors(g.rhs(), ref, sigma, "fp32 vortex %dD warp %.1f" % (dim, warp))
    print("fp32 vortex %dD warp %.1f: err/sigma %.2e  L2 %.2e  Linf %.2e" % (dim, warp, ws, l2, linf))
    assert ws <= TOL32
