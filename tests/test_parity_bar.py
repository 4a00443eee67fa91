"""Pin of the state-dependent part of the FP64 parity bar (CPU).

The library evaluates the log means of Sec. 3.1 from per-node logarithms
(the precomputation of Sec. 7.2): in the logarithmic branch, taken when
|a+ - a-| >= 0.01 (a+ + a-), the difference ln a+ - ln a- of two rounded
FP64 logarithms is at least ln(1.01/0.99) ~ 0.02 in magnitude and, with
each logarithm within one unit in the last place, carries an absolute error
of at most eps (|ln a+| + |ln a-|)/2 + eps |ln a+ - ln a-|/2, eps = 2^-52.
Its relative error is then bounded by eps (1 + 100 L), L = max(|ln a+|,
|ln a-|), the term the bar adds to the sigma factor (tests/parity.py).
Checked here against 50-digit logarithms on seeded pairs over the ranges of
the test states (beta = rho/p from 1e-3 to 10), including pairs at the
branch cut, where the bound is tightest.
"""
import mpmath
import numpy as np

import parity

mpmath.mp.dps = 50
EPS = 2.0 ** -52


def pairs(seed, count):
    rng = np.random.default_rng(seed)
    a = np.exp(rng.uniform(np.log(1e-3), np.log(10.0), count))
    # relative gaps from the branch cut (0.01) up to a factor of three
    r = np.where(rng.random(count) < 0.5, 0.01 * (1 + rng.random(count) * 1e-6), rng.uniform(0.01, 0.5, count))
    b = a * (1 + r) / (1 - r)
    return a, b


def test_log_difference_error_within_bar_term():
    a, b = pairs(3, 4000)
    worst = 0.0
    for x, y in zip(a, b):
        assert abs(y - x) >= 0.01 * (x + y) * (1 - 1e-12)  # logarithmic branch
        got = np.log(y) - np.log(x)
        exact = mpmath.log(mpmath.mpf(float(y))) - mpmath.log(mpmath.mpf(float(x)))
        rel = abs(float((mpmath.mpf(float(got)) - exact) / exact))
        L = max(abs(np.log(x)), abs(np.log(y)))
        bound = EPS * (1 + 100 * L)
        assert rel <= bound, (x, y, rel, bound)
        worst = max(worst, rel / bound)
    print("log-difference error: worst fraction of eps (1 + 100 L) %.3f" % worst)
    assert worst > 0.05  # the bound is not vacuous on these ranges


def test_log_range_of_the_test_states():
    """L of the states the GPU tests use: the random Fourier states (rho, p in
    [0.8, 1.2]) and the density wave (p = 20, rho in [0.02, 1.98])."""
    from paper_2112_10517_amd import inputs
    import oracle
    m = oracle.Mesh(3, 3, (3, 3, 3), warp=0.1)
    L_rand = parity.log_range(inputs.random_fourier(m.coords(), 2))
    L_dw = parity.log_range(inputs.density_wave(m.coords()))
    assert L_rand <= np.log(1.2 / 0.8) + 1e-12
    assert 5.0 < L_dw < 7.0
    assert abs(parity.sigma_factor(None) - parity.SIGMA64) == 0.0
    assert 1.5e-13 < parity.sigma_factor(inputs.density_wave(m.coords())) < 1.9e-13
