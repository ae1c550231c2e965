"""Exact polynomial integration used by the pin tests (independent of oracle/ and
of the GPU path).

* Bounding-box Legendre basis functions expanded as power-series polynomials in
  (x, y) with numpy's Legendre -> power conversion.
* Integrals of x^a y^b over a simple polygon by the divergence theorem:
  int_P x^a y^b dA = 1/(a+1) oint x^(a+1) y^b n_x ds = 1/(a+1) sum_edges int x(t)^(a+1) y(t)^b y'(t) dt,
  evaluated with a Gauss rule exact for the edge polynomial (numpy.leggauss).
"""

import numpy as np
from numpy.polynomial import legendre as L
from numpy.polynomial import polynomial as P


def basis_exponents(dim, p):
    out = []
    for k in range(p + 1):
        for a in range(k, -1, -1):
            if dim == 2:
                out.append((a, k - a))
            else:
                for b in range(k - a, -1, -1):
                    out.append((a, b, k - a - b))
    return out


def legendre_in_x(n, lo, hi):
    """Coefficients (ascending powers of x) of P_n((2x - lo - hi)/(hi - lo))."""
    c = L.leg2poly([0] * n + [1])
    alpha, beta = 2.0 / (hi - lo), -(lo + hi) / (hi - lo)
    out = np.zeros(1)
    lin = np.array([beta, alpha])
    powk = np.array([1.0])
    for k, ck in enumerate(c):
        out = P.polyadd(out, ck * powk)
        powk = P.polymul(powk, lin)
    return out


def basis_polys_2d(p, lo, hi):
    """Basis functions as 2D coefficient arrays C[a, b] of xi^a eta^b in the box
    coordinates xi = (2x - lo - hi)/(hi - lo) (well conditioned)."""
    box = (hi[0] - lo[0]) * (hi[1] - lo[1])
    out = []
    for a, b in basis_exponents(2, p):
        s = np.sqrt((2 * a + 1) * (2 * b + 1) / box)
        out.append(s * np.outer(L.leg2poly([0] * a + [1]), L.leg2poly([0] * b + [1])))
    return out


def to_box(xy, lo, hi):
    """Polygon vertices in box coordinates, and the Jacobian dx dy = J dxi deta."""
    lo, hi = np.asarray(lo)[:2], np.asarray(hi)[:2]
    return (2 * xy - lo - hi) / (hi - lo), np.prod(hi - lo) / 4.0


def dx(c):
    return P.polyder(c, axis=0) if c.shape[0] > 1 else np.zeros((1, c.shape[1]))


def dy(c):
    return P.polyder(c, axis=1) if c.shape[1] > 1 else np.zeros((c.shape[0], 1))


def mul(a, b):
    out = np.zeros((a.shape[0] + b.shape[0] - 1, a.shape[1] + b.shape[1] - 1))
    for i in range(a.shape[0]):
        for j in range(a.shape[1]):
            if a[i, j] != 0.0:
                out[i:i + b.shape[0], j:j + b.shape[1]] += a[i, j] * b
    return out


def polygon_monomial(xy, a, b):
    """int over the CCW polygon xy[n,2] of x^a y^b."""
    deg = a + b + 1
    t, w = np.polynomial.legendre.leggauss(deg // 2 + 2)
    t = 0.5 * (t + 1)
    w = 0.5 * w
    s = 0.0
    n = xy.shape[0]
    for k in range(n):
        p0, p1 = xy[k], xy[(k + 1) % n]
        x = p0[0] + t * (p1[0] - p0[0])
        y = p0[1] + t * (p1[1] - p0[1])
        s += np.dot(w, x ** (a + 1) * y ** b) * (p1[1] - p0[1])
    return s / (a + 1)


def polygon_integral(xy, c):
    """int over the polygon of the 2D polynomial with coefficients c[a, b]."""
    s = 0.0
    for a in range(c.shape[0]):
        for b in range(c.shape[1]):
            if c[a, b] != 0.0:
                s += c[a, b] * polygon_monomial(xy, a, b)
    return s
