"""Pins of the oracle's mesh and metric terms (Sec. 2.3).

* affine boxes: Ja^n = prod_{j != n}(h_j/2) e_n and J = prod_j h_j/2 exactly;
* warped boxes: the discrete metric identities sum_i D_i (Ja)^i = 0 hold to
  round-off, the two sides of every face see the same normal, J > 0, and at
  high degree the metrics converge to the analytic cofactors of the map;
* warped boxes: sum W J is the box volume to round-off (rank-one Jacobian of
  the warp, SBP)."""
import numpy as np
import pytest


def ref_derivative(field, D, N, dim, axis):
    # field [E, nodes] with x fastest; apply D along reference direction `axis`
    E = field.shape[0]
    f = field.reshape((E,) + (N,) * dim)  # axes (E, [z], [y], x)
    ax = dim - axis  # numpy axis of reference direction `axis`
    return np.moveaxis(np.tensordot(D, np.moveaxis(f, ax, 0), axes=(1, 0)), 0, ax).reshape(E, -1)


@pytest.mark.parametrize("dim", [2, 3])
def test_affine_metrics_exact(orc, dim):
    lo, hi, n = [-1.0, 0.5, -2.0], [3.0, 1.5, 2.0], [3, 5, 2]
    m = orc.Mesh(dim, 3, n[:dim], lo=lo[:dim], hi=hi[:dim])
    Ja, J = m.metrics()
    h = [(hi[j] - lo[j]) / n[j] for j in range(dim)]
    Jex = np.prod([hj / 2 for hj in h])
    assert np.allclose(J, Jex, rtol=1e-13, atol=0)
    for a in range(dim):
        for b in range(dim):
            ex = np.prod([h[j] / 2 for j in range(dim) if j != a]) if a == b else 0.0
            assert np.allclose(Ja[:, a, b], ex, rtol=0, atol=1e-13 * Jex)
    x = m.coords()
    # element corners on the uniform grid, nodes at the LGL points
    xi, _, _ = m.operators()
    assert np.isclose(x[0, 0, 0], lo[0]) and np.isclose(x[0, 0, 1], lo[0] + (xi[1] + 1) / 2 * h[0])


@pytest.mark.parametrize("dim,p", [(2, 3), (3, 3), (3, 5)])
def test_metric_identities_and_faces(orc, dim, p):
    n = [5, 4, 3][:dim]
    m = orc.Mesh(dim, p, n, warp=0.1)
    Ja, J = m.metrics()
    _, _, D = m.operators()
    N = p + 1
    assert np.all(J > 0)
    scale = np.abs(Ja).max()
    for comp in range(dim):
        div = sum(ref_derivative(Ja[:, i, comp], D, N, dim, i) for i in range(dim))
        assert np.abs(div).max() < 1e-13 * scale * N * N
    # the normal (Ja)^a on a shared face agrees from both sides (periodic seam included)
    E = m.n_elem
    grid = np.arange(E).reshape(tuple(reversed(n)))
    shp = (E,) + (N,) * dim
    for a in range(dim):
        ax = dim - a  # numpy axis of direction a within (E, [z], [y], x)
        right = np.roll(grid, -1, axis=dim - 1 - a).reshape(-1)
        for comp in range(dim):
            f = Ja[:, a, comp].reshape(shp)
            L = np.take(f, N - 1, axis=ax)
            R = np.take(f, 0, axis=ax)[right]
            assert np.abs(L - R).max() < 1e-14 * N * N * scale


def test_warped_metrics_converge_to_map(orc):
    # x = xh + w prod sin(pi xh_j): Ja^n_m = J * d xi^n / d x_m (cofactors of dx/dxi)
    w, p, n = 0.1, 9, 3
    m = orc.Mesh(3, p, (n, n, n), warp=w)
    Ja, J = m.metrics()
    x = m.coords()
    xi, _, _ = m.operators()
    N = p + 1
    h = 2.0 / n
    idx = np.arange(N ** 3)
    ij = np.stack([idx % N, (idx // N) % N, idx // (N * N)])
    worst_J, worst_Ja = 0.0, 0.0
    for e in range(m.n_elem):
        ie = [e % n, (e // n) % n, e // (n * n)]
        xh = np.stack([-1 + (ie[j] + (xi[ij[j]] + 1) / 2) * h for j in range(3)])  # [3, nodes]
        s = np.sin(np.pi * xh)
        c = np.cos(np.pi * xh)
        grad = w * np.pi * np.stack([c[0] * s[1] * s[2], s[0] * c[1] * s[2], s[0] * s[1] * c[2]])
        assert np.allclose(x[e], xh + w * np.prod(s, axis=0), atol=1e-14)
        for q in range(N ** 3):
            A = (np.eye(3) + np.outer(np.ones(3), grad[:, q])) * (h / 2)  # A[m, j] = dx_m/dxi_j
            det = np.linalg.det(A)
            cof = det * np.linalg.inv(A)  # cof[n, m] = J dxi^n/dx_m
            worst_J = max(worst_J, abs(J[e, q] - det) / det)
            worst_Ja = max(worst_Ja, np.abs(Ja[e, :, :, q] - cof).max() / np.abs(cof).max())
    assert worst_J < 1e-4 and worst_Ja < 1e-4, (worst_J, worst_Ja)


@pytest.mark.parametrize("dim,p,n,warp", [(2, 3, (3, 4), 0.1), (2, 6, (2, 3), 0.15), (3, 3, (2, 3, 2), 0.1),
                                          (3, 5, (3, 2, 2), 0.1), (3, 7, (2, 1, 2), 0.05)])
def test_warped_volume_is_exact(orc, dim, p, n, warp):
    """sum_i W_i J_i over a warped periodic box is its volume to round-off at
    any degree: the map adds one scalar phi to every coordinate, so the
    collocation Jacobian is prod(h/2) (1 + sum_k D_k phi) (a rank-one update of
    the identity), and by the SBP property 1^T M D = 1^T B the weighted sum of
    D_k phi over an element is a difference of its face values, which cancels
    over the periodic mesh.  A wrong D, a dropped term of the determinant or
    a wrong scale breaks it."""
    m = orc.Mesh(dim, p, n, warp=warp, lo=(-1.0, -2.0, 0.0)[:dim] + (0.0,) * (3 - dim),
                 hi=(1.0, 2.0, 3.0)[:dim] + (1.0,) * (3 - dim))
    _, J = m.metrics()
    vol = float(np.prod([(2.0, 4.0, 3.0)[j] for j in range(dim)]))
    assert J.min() > 0
    assert abs(np.sum(m.weights()[None, :] * J) - vol) < 1e-13 * vol
