"""Pins of the oracle's 1D LGL operators (Sec. 2: derivative matrix, SBP
property, LGL-DGSEM example; Sec. 2.1-2.2: flux-differencing operator).

Every check compares against mathematics fixed independently of the oracle:
textbook closed forms, numpy's Legendre roots, polynomial exactness and the
SBP identity."""
import math

import numpy as np
import pytest
from numpy.polynomial import legendre as L


def test_closed_forms(orc):
    # p = 1..4 nodes and weights: textbook closed forms of LGL quadrature
    s5, s37 = 1.0 / math.sqrt(5.0), math.sqrt(3.0 / 7.0)
    expect = {
        1: ([-1, 1], [1, 1]),
        2: ([-1, 0, 1], [1 / 3, 4 / 3, 1 / 3]),
        3: ([-1, -s5, s5, 1], [1 / 6, 5 / 6, 5 / 6, 1 / 6]),
        4: ([-1, -s37, 0, s37, 1], [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10]),
    }
    for p, (x, w) in expect.items():
        xi, ww, D = orc.lgl(p)
        assert np.allclose(xi, x, atol=1e-15, rtol=0)
        assert np.allclose(ww, w, atol=1e-15, rtol=0)
    _, _, D2 = orc.lgl(2)
    assert np.allclose(D2, [[-1.5, 2, -0.5], [-0.5, 0, 0.5], [0.5, -2, 1.5]], atol=1e-15, rtol=0)
    _, _, D1 = orc.lgl(1)
    assert np.allclose(D1, [[-0.5, 0.5], [-0.5, 0.5]], atol=1e-16, rtol=0)


@pytest.mark.parametrize("p", range(1, 16))
def test_nodes_are_legendre_derivative_roots(orc, p):
    xi, w, D = orc.lgl(p)
    inner = np.sort(L.Legendre.basis(p).deriv().roots().real) if p > 1 else np.array([])
    assert np.allclose(xi[1:-1], inner, atol=2e-14, rtol=0)
    assert xi[0] == -1.0 and xi[-1] == 1.0
    assert np.all(np.diff(xi) > 0)


@pytest.mark.parametrize("p", range(1, 16))
def test_quadrature_exactness(orc, p):
    # LGL quadrature integrates degree 2p-1 exactly
    xi, w, _ = orc.lgl(p)
    for k in range(2 * p):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, xi ** k) - exact) < 5e-15 * max(1, p)


@pytest.mark.parametrize("p", range(1, 16))
def test_derivative_exactness(orc, p):
    # Sec. 2, definition of a p-th order derivative matrix: D x^k = k x^(k-1)
    xi, _, D = orc.lgl(p)
    for k in range(p + 1):
        lhs = D @ xi ** k
        rhs = k * xi ** (k - 1) if k > 0 else np.zeros_like(xi)
        assert np.max(np.abs(lhs - rhs)) < 2e-14 * (1 + k) * p ** 2


@pytest.mark.parametrize("p", range(1, 16))
def test_sbp_property(orc, p):
    # Sec. 2, SBP identity M D + D^T M = R^T B N R = diag(-1, 0, ..., 0, 1)
    xi, w, D = orc.lgl(p)
    M = np.diag(w)
    B = np.zeros((p + 1, p + 1))
    B[0, 0], B[-1, -1] = -1.0, 1.0
    assert np.max(np.abs(M @ D + D.T @ M - B)) < 1e-14 * p


@pytest.mark.parametrize("p", range(1, 16))
def test_flux_differencing_operator_skew(orc, p):
    # Sec. 2.1-2.2: D~ = 2D - M^-1 B is skew-symmetric w.r.t. M, zero diagonal
    xi, w, D = orc.lgl(p)
    B = np.zeros((p + 1, p + 1))
    B[0, 0], B[-1, -1] = -1.0, 1.0
    Dt = 2 * D - np.diag(1 / w) @ B
    MDt = np.diag(w) @ Dt
    assert np.max(np.abs(MDt + MDt.T)) < 2e-14 * p
    assert np.max(np.abs(np.diag(Dt))) < 1e-13 * p


def test_bad_degree(orc):
    with pytest.raises(ValueError):
        orc.lgl(0)
    with pytest.raises(ValueError):
        orc.lgl(16)
