"""Pins of the oracle's logarithmic means (Sec. 3.1, Algorithms 2 and 3).

The reference value is the definition (a_+ - a_-)/(log a_+ - log a_-) evaluated
with mpmath at 50 digits; the identities (tie, homogeneity, mean bounds,
reciprocity) hold for the exact log mean."""
import mpmath
import numpy as np
import pytest

mpmath.mp.dps = 50
EPS = np.finfo(np.float64).eps


def exact_logmean(a, b):
    a, b = mpmath.mpf(a), mpmath.mpf(b)
    if a == b:
        return a
    return (b - a) / (mpmath.log(b) - mpmath.log(a))


def ratios():
    # dense near 1 (series branch, u < 1e-4 <=> |r-1| < ~0.02) and both sides
    r = np.concatenate([1 + np.linspace(-0.5, 3.0, 301),
                        1 + np.geomspace(1e-12, 0.05, 120),
                        1 - np.geomspace(1e-12, 0.05, 120),
                        [1 + 0.0200, 1 + 0.0201, 1 - 0.0198, 1 - 0.0199]])
    return r[r > 0]


@pytest.mark.parametrize("scale", [1e-3, 1.0, 37.5, 1e4])
def test_logmean_vs_mpmath(orc, scale):
    worst = 0.0
    branches = set()
    for r in ratios():
        a, b = scale, scale * float(r)
        u = (a - b) ** 2 / (a + b) ** 2
        branches.add(u < 1e-4)
        ex = exact_logmean(a, b)
        lm = orc.logmean(a, b)
        ilm = orc.inv_logmean(a, b)
        e1 = abs(float((mpmath.mpf(lm) - ex) / ex))
        e2 = abs(float((mpmath.mpf(ilm) - 1 / ex) * ex))
        worst = max(worst, e1, e2)
    assert branches == {True, False}
    assert worst < 64 * EPS, worst


def test_tie_is_exact(orc):
    for a in [1e-8, 0.3, 1.0, 2.0, 123.456, 1e8]:
        assert orc.logmean(a, a) == a
        assert abs(orc.inv_logmean(a, a) * a - 1.0) <= EPS


def test_homogeneity_bounds_reciprocity(orc):
    rng = np.random.default_rng(7)
    for _ in range(2000):
        a = rng.uniform(0.1, 10.0)
        b = a * rng.choice([rng.uniform(0.5, 3.0), 1 + rng.uniform(-0.02, 0.02)])
        c = rng.uniform(0.01, 100.0)
        lm = orc.logmean(a, b)
        # rounding of c*a, c*b is amplified by 1/|b-a| in the log branch
        amp = 1.0 + (a + b) / max(abs(b - a), 1e-300)
        assert abs(orc.logmean(c * a, c * b) - c * lm) <= 4 * EPS * c * lm * min(amp, 1e3)
        assert np.sqrt(a * b) * (1 - 4 * EPS) <= lm <= 0.5 * (a + b) * (1 + 4 * EPS)
        assert abs(lm * orc.inv_logmean(a, b) - 1) < 8 * EPS
        # the log mean is symmetric (Alg. 2 is up to rounding)
        assert abs(orc.logmean(b, a) - lm) <= 4 * EPS * lm * min(amp, 1e3)
