"""Pins of the oracle's second time integrator: the five-stage, fourth-order
2N-storage Runge-Kutta scheme of Carpenter and Kennedy that the paper's FLUXO
runs use (Sec. 4.1), in Williamson's form du <- A_i du + h RHS(u),
u <- u + B_i du.

  * the stored coefficients, turned into the equivalent Butcher tableau,
    satisfy the eight order conditions of order four (and c_1 = 0);
  * self-convergence at order four in time on a smooth problem;
  * it agrees with classical RK4 to the difference of two fourth-order
    schemes; totals are conserved; CFL mode advances the time.
"""
import numpy as np

from paper_2112_10517_amd import inputs


def butcher(A, B):
    """(a, b, c) of the 2N scheme: stage i evaluates RHS at u_{i-1}."""
    s = len(A)

    def weight(i, j):  # coefficient of h k_j in u_i (after i stages), j < i
        tot = 0.0
        for m in range(j, i):
            tot += B[m] * np.prod([A[l] for l in range(j + 1, m + 1)])
        return tot

    a = np.array([[weight(i, j) if j < i else 0.0 for j in range(s)] for i in range(s)])
    b = np.array([weight(s, j) for j in range(s)])
    return a, b, a.sum(axis=1)


def test_ck45_order_conditions(orc):
    A, B = orc.ck45_coefficients()
    assert A[0] == 0.0
    a, b, c = butcher(A, B)
    conds = [
        (b.sum(), 1.0), (b @ c, 1 / 2), (b @ c ** 2, 1 / 3), (b @ (a @ c), 1 / 6),
        (b @ c ** 3, 1 / 4), (b @ (c * (a @ c)), 1 / 8), (b @ (a @ c ** 2), 1 / 12), (b @ (a @ (a @ c)), 1 / 24),
    ]
    for got, want in conds:
        assert abs(got - want) < 1e-14, conds
    # not fifth order: one fifth-order condition fails clearly
    assert abs(b @ c ** 4 - 1 / 5) > 1e-6 or abs(b @ (a @ (a @ (a @ c))) - 1 / 120) > 1e-6
    assert np.all(np.diff(c) > 0) and c[-1] < 1.0


def test_ck45_fourth_order_in_time(orc):
    m = orc.Mesh(2, 3, (3, 3), vol_flux="ranocha", surf_flux="llf")
    u0 = inputs.density_wave(m.coords(), amp=0.3)
    T = 0.02
    sols = [m.ck45(u0, T / s, s)[0] for s in (8, 16, 32, 64)]
    d = [np.abs(sols[i] - sols[i + 1]).max() for i in range(3)]
    ratios = [d[i] / d[i + 1] for i in range(2)]
    assert all(14 < r < 18 for r in ratios), ratios
    # both schemes converge to the same solution of the semi-discretisation
    ref, _ = m.rk4(u0, T / 256, 256)
    assert np.abs(sols[-1] - ref).max() < 1e-3 * d[0]


def test_ck45_conservation_and_cfl_time(orc):
    m = orc.Mesh(2, 4, (4, 3), warp=0.1, vol_flux="ranocha", surf_flux="llf")
    u0 = inputs.random_fourier(m.coords(), 3)
    tot0 = m.totals(u0)
    u1, t1 = m.ck45(u0, 0.0, 5, cfl=0.5, t=2.0)
    scale = np.abs(m.totals(np.abs(u0)))
    assert np.all(np.abs(m.totals(u1) - tot0) <= 1e-13 * scale)
    h0 = m.max_dt(u0, 0.5)
    assert 2.0 + 4.5 * h0 < t1 < 2.0 + 5.5 * h0
