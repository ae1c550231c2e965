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


# ----------------------------------------------------------------- 3D
def basis_polys_3d(p, lo, hi):
    """Basis functions as coefficient arrays C[a, b, c] of xi^a eta^b zeta^c in
    the box coordinates."""
    box = np.prod(np.asarray(hi)[:3] - np.asarray(lo)[:3])
    out = []
    for a, b, c in basis_exponents(3, p):
        s = np.sqrt((2 * a + 1) * (2 * b + 1) * (2 * c + 1) / box)
        pa, pb, pc = (L.leg2poly([0] * k + [1]) for k in (a, b, c))
        out.append(s * pa[:, None, None] * pb[None, :, None] * pc[None, None, :])
    return out


def d3(c, axis):
    """Derivative along a box axis of a 3D coefficient array."""
    if c.shape[axis] == 1:
        return np.zeros_like(c)
    return P.polyder(c, axis=axis)


def mul3(a, b):
    out = np.zeros(tuple(a.shape[k] + b.shape[k] - 1 for k in range(3)))
    for idx in np.ndindex(*a.shape):
        if a[idx] != 0.0:
            i, j, k = idx
            out[i:i + b.shape[0], j:j + b.shape[1], k:k + b.shape[2]] += a[idx] * b
    return out


def triangle_rule_collapsed(n):
    """n^2-point rule on the unit triangle from a Gauss product on the square
    collapsed onto it (Duffy map); exact for total degree 2n - 2.  Returns
    barycentric points [n^2, 3] and weights summing to 1."""
    t, w = np.polynomial.legendre.leggauss(n)
    u, wu = 0.5 * (t + 1), 0.5 * w
    pts, wts = [], []
    for i in range(n):
        for j in range(n):
            s = u[i]
            r = (1 - s) * u[j]
            pts.append((1 - s - r, s, r))
            wts.append(wu[i] * wu[j] * (1 - s))
    wts = np.array(wts)
    return np.array(pts), wts / wts.sum()


def cell_triangles_outward(m, c):
    """The boundary triangles of polyhedral cell c as [k, 3, 3] vertex
    coordinates, each ordered so that its normal points out of the cell."""
    xyz = np.stack([m.x, m.y, m.z], 1)
    out = []
    for f in m.cell_face[m.cell_face_ptr[c]:m.cell_face_ptr[c + 1]]:
        v = xyz[m.face_vtx[3 * f:3 * f + 3]]
        o = xyz[m.face_opp[f]]
        nrm = np.cross(v[1] - v[0], v[2] - v[0])
        away_from_opp = np.dot(nrm, o - v[0]) < 0
        left = m.face_cell[2 * f] == c
        if away_from_opp != left:
            v = v[[0, 2, 1]]
        out.append(v)
    return np.array(out)


def polyhedron_integral_box(tris_xi, c, n_rule=6):
    """int over the polyhedron (triangles given in box coordinates, outward) of
    the polynomial c[a, b, c] in (xi, eta, zeta), by the divergence theorem with
    the xi-antiderivative, in box coordinates (multiply by the box Jacobian)."""
    G = P.polyint(c, axis=0)
    bary, w = triangle_rule_collapsed(n_rule)
    s = 0.0
    for v in tris_xi:
        S1 = 0.5 * np.cross(v[1] - v[0], v[2] - v[0])[0]
        if S1 == 0.0:
            continue
        x = bary @ v
        vals = P.polyval3d(x[:, 0], x[:, 1], x[:, 2], G)
        s += S1 * np.dot(w, vals)
    return s
