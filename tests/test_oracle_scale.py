"""Pins of the oracle's rounding scale sigma (Mesh.rhs_scale).

sigma_i is the flux-differencing right-hand side of Sec. 2 with every term
replaced by its magnitude:

  sigma_i = (1/|J_i|) [ sum_n sum_k |2 D_{i_n k} f_vol(u_i, u_k, (Ja^n_i + Ja^n_k)/2)|
                        + sum_n (|f*| + |f^n(u_i) . Ja^n_i|) / w_end ]

(the face sum only over the faces node i lies on).  Every FP64 parity bound
of the GPU tests is a multiple of it, so a mistake in it (a dropped 1/J, a
face counted twice, a lost factor 2, a wrong weight) would loosen or tighten
every bound unseen.  It is pinned here against

  * a closed form: a constant state on an affine box with different element
    widths per direction, where every two-point flux reduces to the physical
    flux f^n(u) (consistency) and sigma_i = sum_n (2/h_n) |f^n(u)|
    (sum_k 2 |D_{i_n k}| + [i_n = p] 2/w_p + [i_n = 0] 2/w_0);
  * an independent numpy evaluation of the definition on warped 2D and 3D
    meshes (own LGL operators, own two-point fluxes written from Sec. 3.2,
    own neighbour and node indexing; only the metric terms come from the
    oracle, and those are pinned in test_oracle_mesh.py);
  * the triangle inequality |RHS_i| <= sigma_i node by node (RHS is the signed
    sum of the same terms), for every flux pairing, affine and warped, and
    for the Gauss collocation scheme of Sec. 6;
  * 1/h scaling under uniform refinement.
"""
import numpy as np
import pytest

from paper_2112_10517_amd import inputs

from test_oracle_rhs import lgl_numpy

G = 1.4


# ---------------------------------------------------------------------------
# numpy two-point fluxes (Sec. 3.2), arrays [..., var] and normals [..., dim]
# ---------------------------------------------------------------------------

def prim(u, dim):
    rho = u[..., 0]
    v = u[..., 1:dim + 1] / rho[..., None]
    p = (G - 1) * (u[..., dim + 1] - 0.5 * rho * np.sum(v * v, axis=-1))
    return rho, v, p


def phys_flux(u, n, dim):
    """f(u) . n"""
    rho, v, p = prim(u, dim)
    vn = np.sum(v * n, axis=-1)
    f = np.empty_like(u)
    f[..., 0] = rho * vn
    f[..., 1:dim + 1] = rho[..., None] * v * vn[..., None] + p[..., None] * n
    f[..., dim + 1] = (u[..., dim + 1] + p) * vn
    return f


def inv_log_mean(x, y):
    """(ln y - ln x)/(y - x), written with log1p; 1/x where y == x."""
    d = y - x
    safe = np.where(d == 0, 1.0, d)
    return np.where(d == 0, 1.0 / x, np.log1p(d / x) / safe)


def two_point(kind, um, up, n, dim):
    if kind in ("central", "llf"):
        f = 0.5 * (phys_flux(um, n, dim) + phys_flux(up, n, dim))
        if kind == "llf":
            rm, vm, pm = prim(um, dim)
            rp, vp, pp = prim(up, dim)
            lam = (np.maximum(np.abs(np.sum(vm * n, -1)), np.abs(np.sum(vp * n, -1))) +
                   np.maximum(np.sqrt(G * pm / rm), np.sqrt(G * pp / rp)) * np.sqrt(np.sum(n * n, -1)))
            f = f - 0.5 * lam[..., None] * (up - um)
        return f
    rm, vm, pm = prim(um, dim)
    rp, vp, pp = prim(up, dim)
    vnm, vnp = np.sum(vm * n, -1), np.sum(vp * n, -1)
    vn_avg = 0.5 * (vnm + vnp)
    p_avg = 0.5 * (pm + pp)
    f = np.empty_like(um)
    if kind == "shima":
        f[..., 0] = 0.5 * (rm + rp) * vn_avg
        e_int = p_avg * vn_avg / (G - 1)
    else:  # ranocha: log mean of rho, p- p+ times the inverse log mean of (rho- p+, rho+ p-)
        f[..., 0] = vn_avg / inv_log_mean(rm, rp)
        e_int = f[..., 0] * pm * pp * inv_log_mean(rm * pp, rp * pm) / (G - 1)
    f[..., 1:dim + 1] = f[..., 0][..., None] * 0.5 * (vm + vp) + p_avg[..., None] * n
    f[..., dim + 1] = (0.5 * f[..., 0] * np.sum(vm * vp, -1) + e_int + 0.5 * (pp * vnm + pm * vnp))
    return f


def sigma_numpy(m, u, vol, surf):
    """The definition of sigma evaluated with numpy on the oracle's mesh."""
    dim, N, p = m.dim, m.N, m.p
    nn, nv = m.nodes, m.n_var
    _, w, D = lgl_numpy(p)
    Ja, J = m.metrics()
    ut = np.ascontiguousarray(u.transpose(0, 2, 1))  # [E][node][var]
    idx = np.arange(nn)
    dig = [(idx // N ** j) % N for j in range(dim)]
    nel = [int(round(x)) for x in m._nel]
    E = m.n_elem
    eidx = np.arange(E)
    edig = [(eidx // int(np.prod(nel[:j]))) % nel[j] for j in range(dim)]
    acc = np.zeros((E, nn, nv))
    for n in range(dim):
        a = np.ascontiguousarray(Ja[:, n, :dim, :].transpose(0, 2, 1))  # [E][node][dim]
        for k in range(N):
            j = idx + (k - dig[n]) * N ** n
            f = two_point(vol, ut, ut[:, j], 0.5 * (a + a[:, j]), dim)
            acc += np.abs(2.0 * D[dig[n], k][None, :, None] * f)
        for side in (0, 1):
            at, other = (p, 0) if side else (0, p)
            step = 1 if side else -1
            en_dig = list(edig)
            en_dig[n] = (edig[n] + step) % nel[n]
            eo = sum(en_dig[j] * int(np.prod(nel[:j])) for j in range(dim))
            io = idx + (other - dig[n]) * N ** n
            uo, ao = ut[eo][:, io], a[eo][:, io]
            nf = 0.5 * (a + ao)
            fstar = two_point(surf, ut, uo, nf, dim) if side else two_point(surf, uo, ut, nf, dim)
            term = (np.abs(fstar) + np.abs(phys_flux(ut, a, dim))) / w[at]
            acc += np.where((dig[n] == at)[None, :, None], term, 0.0)
    return (acc / np.abs(J)[:, :, None]).transpose(0, 2, 1)


def mesh(orc, dim, p, n, lo, hi, warp=0.0, vol="ranocha", surf="llf", nodes="lgl"):
    m = orc.Mesh(dim, p, n, lo=lo, hi=hi, warp=warp, vol_flux=vol, surf_flux=surf, nodes=nodes)
    m._nel = list(n)
    return m


# ---------------------------------------------------------------------------

@pytest.mark.parametrize("p", [2, 4])
@pytest.mark.parametrize("vol,surf", [("ranocha", "llf"), ("shima", "ranocha"), ("central", "central")])
def test_sigma_closed_form_constant_state(orc, p, vol, surf):
    lo, hi, n = (-1.0, -0.5, 0.0), (1.0, 1.5, 1.0), (2, 3, 4)
    h = [(b - a) / k for a, b, k in zip(lo, hi, n)]
    m = mesh(orc, 3, p, n, lo, hi, vol=vol, surf=surf)
    rho, vel, pr = 1.3, np.array([0.3, -0.2, 0.1]), 2.0
    u = np.zeros(m.shape)
    u[:, 0] = rho
    u[:, 1:4] = rho * vel[None, :, None]
    u[:, 4] = pr / (G - 1) + 0.5 * rho * vel @ vel
    x, w, D = lgl_numpy(p)
    N = p + 1
    idx = np.arange(N ** 3)
    expect = np.zeros((5, N ** 3))
    for a in range(3):
        e_a = np.eye(3)[a]
        f = phys_flux(u[0, :, 0], e_a, 3)  # f^a(u)
        d = (idx // N ** a) % N
        row = 2.0 * np.abs(D).sum(axis=1)[d] + np.where(d == p, 2.0 / w[p], 0.0) + np.where(d == 0, 2.0 / w[0], 0.0)
        expect += (2.0 / h[a]) * np.abs(f)[:, None] * row[None, :]
    sc = m.rhs_scale(u)
    np.testing.assert_allclose(sc, np.broadcast_to(expect, sc.shape), rtol=1e-13, atol=0)


@pytest.mark.parametrize("dim,p,n,warp,vol,surf", [
    (3, 3, (2, 3, 2), 0.1, "ranocha", "llf"),
    (3, 2, (3, 2, 2), 0.1, "shima", "central"),
    (3, 4, (2, 2, 2), 0.0, "ranocha", "ranocha"),
    (2, 5, (3, 4), 0.1, "shima", "llf"),
    (2, 3, (1, 3), 0.1, "ranocha", "shima"),   # an element that is its own x-neighbour
])
def test_sigma_numpy_definition(orc, dim, p, n, warp, vol, surf):
    lo, hi = (-1.0,) * dim, (1.0,) * dim
    m = mesh(orc, dim, p, n, lo, hi, warp=warp, vol=vol, surf=surf)
    rng = np.random.default_rng(11)
    u = inputs.random_fourier(m.coords(), 5) * (1 + 0.01 * rng.standard_normal(m.shape))
    sc = m.rhs_scale(u)
    ref = sigma_numpy(m, u, vol, surf)
    assert np.all(sc > 0)
    np.testing.assert_allclose(sc, ref, rtol=1e-12, atol=0)


@pytest.mark.parametrize("dim,p,n,warp,vol,surf,nodes", [
    (3, 3, (3, 2, 2), 0.1, "ranocha", "llf", "lgl"),
    (3, 7, (1, 2, 1), 0.1, "shima", "ranocha", "lgl"),
    (3, 5, (2, 2, 2), 0.0, "central", "central", "lgl"),
    (2, 4, (4, 3), 0.1, "ranocha", "ranocha", "lgl"),
    (3, 3, (2, 2, 3), 0.0, "ranocha", "llf", "gauss"),
    (2, 5, (3, 3), 0.0, "shima", "ranocha", "gauss"),
])
def test_sigma_bounds_rhs(orc, dim, p, n, warp, vol, surf, nodes):
    # |RHS_i| <= sigma_i: RHS_i is the signed sum of the terms sigma_i sums in
    # magnitude (slack: the rounding of the two sums)
    lo, hi = (-1.0,) * dim, (1.0,) * dim
    m = mesh(orc, dim, p, n, lo, hi, warp=warp, vol=vol, surf=surf, nodes=nodes)
    rng = np.random.default_rng(3)
    u = inputs.random_fourier(m.coords(), 9) * (1 + 0.02 * rng.standard_normal(m.shape))
    du, sc = m.rhs(u), m.rhs_scale(u)
    assert np.all(np.abs(du) <= sc * (1 + 1e-12))
    # and sigma is no gross over-estimate: on a random state some node of
    # every variable keeps at least 1% of its terms' magnitude
    assert np.all(np.max(np.abs(du) / sc, axis=(0, 2)) > 0.01)


def test_sigma_scales_with_inverse_width(orc):
    # the same reference-element state on a box refined by two: every term
    # of sigma carries one factor 2/h
    rho, vel, pr = 0.9, np.array([0.2, 0.1, -0.3]), 1.1
    out = []
    for k in (2, 4):
        m = mesh(orc, 3, 3, (k, k, k), (-1.0,) * 3, (1.0,) * 3)
        u = np.zeros(m.shape)
        u[:, 0] = rho
        u[:, 1:4] = rho * vel[None, :, None]
        u[:, 4] = pr / (G - 1) + 0.5 * rho * vel @ vel
        out.append(m.rhs_scale(u)[0])
    np.testing.assert_allclose(out[1], 2.0 * out[0], rtol=1e-13, atol=0)
