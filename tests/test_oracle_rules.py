"""Pins for the oracle's quadrature rules: exactness on every monomial up to the
rule's degree against the textbook closed forms (Beta integrals), which the
rules' derivation (symmetric invariants only) never uses directly."""

from math import factorial

import numpy as np
import pytest

from oracle import rules


@pytest.mark.parametrize("n", range(1, 16))
def test_gauss_legendre_exact(n):
    t, w = rules.gauss_legendre01(n)
    assert np.all(np.diff(t) > 0) and np.all(w > 0)
    for k in range(2 * n):
        assert abs(np.dot(w, t ** k) - 1.0 / (k + 1)) < 2e-15
    # nodes are the roots of P_n, so the degree-2n integrand P_n^2 (exact 1/(2n+1)) is missed
    pn = np.polynomial.legendre.legval(2 * t - 1, [0] * n + [1])
    assert np.max(np.abs(pn)) < 1e-13
    assert abs(np.dot(w, pn ** 2) - 1.0 / (2 * n + 1)) > 0.5 / (2 * n + 1)


def test_gauss_legendre_matches_numpy():
    for n in range(1, 16):
        x, w = np.polynomial.legendre.leggauss(n)
        t, w2 = rules.gauss_legendre01(n)
        assert np.allclose(t, 0.5 * (x + 1), atol=1e-15, rtol=0)
        assert np.allclose(w2, 0.5 * w, atol=1e-15, rtol=0)


@pytest.mark.parametrize("deg,npts", [(4, 6), (6, 12), (8, 16)])
def test_triangle_rule_exact(deg, npts):
    bary, w = rules.triangle_rule(deg)
    assert bary.shape == (npts, 3) and np.all(bary > 0)
    assert np.allclose(bary.sum(1), 1.0, atol=1e-15)
    # reference triangle (0,0),(1,0),(0,1): x = l1, y = l2, area 1/2
    x, y = bary[:, 1], bary[:, 2]
    worst = 0.0
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            exact = factorial(a) * factorial(b) / factorial(a + b + 2)
            worst = max(worst, abs(0.5 * np.dot(w, x ** a * y ** b) - exact) / exact)
    assert worst < 1e-14
    # degree is not higher than claimed
    errs = [abs(0.5 * np.dot(w, x ** a * y ** (deg + 1 - a)) - factorial(a) * factorial(deg + 1 - a) / factorial(deg + 3))
            for a in range(deg + 2)]
    assert max(errs) > 1e-10


def test_tet_rule_exact():
    bary, w = rules.tet_rule(4)
    assert bary.shape == (11, 4)
    assert abs(w.sum() - 1) < 1e-15
    x, y, z = bary[:, 1], bary[:, 2], bary[:, 3]
    worst = 0.0
    for a in range(5):
        for b in range(5 - a):
            for c in range(5 - a - b):
                exact = factorial(a) * factorial(b) * factorial(c) / factorial(a + b + c + 3)
                worst = max(worst, abs(np.dot(w, x ** a * y ** b * z ** c) / 6.0 - exact) / exact)
    assert worst < 1e-14


@pytest.mark.parametrize("deg", [4, 6, 8])
def test_triangle_rule_exact_in_rational_arithmetic(deg):
    """The rule as stored (doubles) against the exact moments, summed exactly
    (Fractions): residuals at the rounding level of the data, so the rule is the
    double rule nearest the exact one (a double-precision fit leaves ~1e-14)."""
    from fractions import Fraction as Fr
    bary, w = rules.triangle_rule(deg)
    B = [[Fr(float(v)) for v in row] for row in bary]
    W = [Fr(float(v)) for v in w]
    worst = 0.0
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            s = sum(wi * q[1] ** a * q[2] ** b for wi, q in zip(W, B))
            exact = Fr(2 * factorial(a) * factorial(b), factorial(a + b + 2))
            worst = max(worst, abs(float(s - exact)) / float(exact))
    assert worst < 1e-15
