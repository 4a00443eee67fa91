"""The oracle against the fixtures in tests/golden/ (CPU): the log-mean
series branch and cutoff printed in Algorithms 2 and 3 of Sec. 3.1, and the
textbook closed forms of the LGL rule of the DGSEM (Sec. 2).  Each fixture
names its source; the values are written out there, not computed by the
oracle."""
import json
import os
from fractions import Fraction
from math import sqrt

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def value(s: str) -> float:
    s = s.strip()
    neg = s.startswith("-")
    s = s.lstrip("-")
    if s.startswith("sqrt(") and s.endswith(")"):
        v = sqrt(float(Fraction(s[5:-1])))
    else:
        v = float(Fraction(s))
    return -v if neg else v


def test_logmean_series_branch_matches_the_printed_algorithm(orc):
    g = load("logmean_series.json")
    c = g["series_coefficients"]
    assert [float(Fraction(x)) for x in g["series_coefficients_exact"]] == pytest.approx(c, rel=1e-16)
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(2000):
        a = float(rng.uniform(0.1, 10.0))
        b = a * (1.0 + float(rng.uniform(-0.019, 0.019)))  # u below the cutoff
        u = (a * (a - 2 * b) + b * b) / (a * (a + 2 * b) + b * b)
        if not u < g["cutoff_fp64"]:
            continue
        P = c[0] + u * (c[1] + u * (c[2] + u * c[3]))
        assert orc.logmean(a, b) == pytest.approx((a + b) / P, rel=4e-16, abs=0)
        assert orc.inv_logmean(a, b) == pytest.approx(P / (a + b), rel=4e-16, abs=0)
        checked += 1
    assert checked > 1000
    # above the cutoff the logarithmic branch of the algorithms
    a, b = 1.0, 1.5
    assert orc.logmean(a, b) == pytest.approx((b - a) / np.log(b / a), rel=1e-15)
    assert orc.inv_logmean(a, b) == pytest.approx(np.log(b / a) / (b - a), rel=1e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_lgl_rules_match_the_closed_forms(orc, p):
    g = load("lgl_closed_forms.json")["rules"][str(p)]
    xi, w, D = orc.lgl(p)
    assert np.allclose(xi, [value(s) for s in g["nodes"]], rtol=0, atol=1e-15)
    assert np.allclose(w, [value(s) for s in g["weights"]], rtol=0, atol=1e-15)
    if p == 2:
        rows = load("lgl_closed_forms.json")["derivative_p2"]["rows"]
        assert np.allclose(D, [[value(s) for s in r] for r in rows], rtol=0, atol=1e-14)
