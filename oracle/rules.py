"""Quadrature rules for the oracle (test infrastructure; FP64).

The method applies standard quadrature rules on every simplex of a simplicial
subdivision of each element and on every simplicial sub-face (Section 3,
"Implementation on Graphics Processing Units").  The paper does not name the
rules, so this module derives the standard ones itself from their defining
moment equations:

* Gauss-Legendre on [0, 1]: Newton's method on the roots of P_n (three-term
  recurrence), weights 1 / ((1 - x^2) P_n'(x)^2) mapped to [0, 1].
* Fully symmetric triangle rules of degree 4 (6 points), 6 (12) and 8 (16)
  (the Dunavant families) and the 11-point degree-4 tetrahedron rule (the
  Keast family): Newton's method on the moment equations of the symmetric
  invariants e2^i e3^j (e4^k) of the barycentric coordinates, whose exact means
  come from the simplex moment formula  mean(lambda^alpha) =
  d! alpha! / (|alpha| + d)!  evaluated in exact rational arithmetic.
  The published point/weight values are only used as Newton starting guesses.

Rules are returned as (bary, w): barycentric points [n, d+1] and weights [n]
summing to 1 (multiply by the simplex measure).
"""

from fractions import Fraction
from functools import lru_cache
from itertools import combinations, permutations
from math import factorial

import numpy as np


# --------------------------------------------------------------------------- 1D
@lru_cache(maxsize=None)
def gauss_legendre01(n: int):
    """n-point Gauss-Legendre rule on [0, 1] (points ascending, weights sum to 1)."""
    if n < 1:
        raise ValueError("n >= 1")
    xs = np.empty(n)
    ws = np.empty(n)
    for i in range(n):
        x = np.cos(np.pi * (i + 0.75) / (n + 0.5))
        for _ in range(100):
            p0, p1 = 1.0, x
            for k in range(2, n + 1):
                p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
            if n == 1:
                p0, p1 = 1.0, x
            dp = n * (x * p1 - p0) / (x * x - 1.0)
            dx = p1 / dp
            x -= dx
            if abs(dx) < 1e-16:
                break
        p0, p1 = 1.0, x
        for k in range(2, n + 1):
            p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
        dp = n * (x * p1 - p0) / (x * x - 1.0)
        xs[i] = x
        ws[i] = 2.0 / ((1.0 - x * x) * dp * dp)
    # polish each root by Newton on P_n in 50-digit arithmetic (mpmath), then round once
    import mpmath as mp
    with mp.workdps(50):
        for i in range(n):
            x = mp.mpf(float(xs[i]))
            for _ in range(6):
                p0, p1 = mp.mpf(1), x
                for k in range(2, n + 1):
                    p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
                if n == 1:
                    p0, p1 = mp.mpf(1), x
                dp = n * (x * p1 - p0) / (x * x - 1)
                x = x - p1 / dp
            p0, p1 = mp.mpf(1), x
            for k in range(2, n + 1):
                p0, p1 = p1, ((2 * k - 1) * x * p1 - (k - 1) * p0) / k
            if n == 1:
                p0, p1 = mp.mpf(1), x
            dp = n * (x * p1 - p0) / (x * x - 1)
            xs[i] = float(x)
            ws[i] = float(2 / ((1 - x * x) * dp * dp))
    order = np.argsort(xs)
    t = (xs[order] + 1.0) / 2
    w = ws[order] / 2
    return t, w


# ---------------------------------------------------------------- exact moments
def _poly_mul(a, b):
    out = {}
    for ea, ca in a.items():
        for eb, cb in b.items():
            e = tuple(x + y for x, y in zip(ea, eb))
            out[e] = out.get(e, 0) + ca * cb
    return out


def _elem_sym(d1: int, k: int):
    """Elementary symmetric polynomial e_k in d1 variables as {exponents: coeff}."""
    out = {}
    for idx in combinations(range(d1), k):
        e = tuple(1 if i in idx else 0 for i in range(d1))
        out[e] = Fraction(1)
    return out


def _exact_mean(poly, d: int) -> float:
    """Mean over a d-simplex of a polynomial in barycentric coordinates."""
    s = Fraction(0)
    for e, c in poly.items():
        num = factorial(d)
        for a in e:
            num *= factorial(a)
        s += c * Fraction(num, factorial(sum(e) + d))
    return float(s)


def _invariant_exponents(d: int, degree: int):
    """Exponent tuples (of e2, e3[, e4]) of the symmetric invariants up to ``degree``."""
    degs = list(range(2, d + 2))
    out = []

    def rec(i, cur, tot):
        if i == len(degs):
            out.append(tuple(cur))
            return
        k = 0
        while tot + k * degs[i] <= degree:
            rec(i + 1, cur + [k], tot + k * degs[i])
            k += 1

    rec(0, [], 0)
    return out


def _invariants_numeric(bary: np.ndarray, exps):
    d1 = bary.shape[1]
    es = []
    for k in range(2, d1 + 1):
        v = np.zeros(bary.shape[0])
        for idx in combinations(range(d1), k):
            v = v + np.prod(bary[:, idx], axis=1)
        es.append(v)
    cols = []
    for ex in exps:
        v = np.ones(bary.shape[0])
        for e_k, p in zip(es, ex):
            v = v * e_k ** p
        cols.append(v)
    return np.stack(cols, 1)


def _invariant_means(d: int, exps):
    d1 = d + 1
    es = [_elem_sym(d1, k) for k in range(2, d1 + 1)]
    out = []
    for ex in exps:
        poly = {tuple([0] * d1): Fraction(1)}
        for e_k, p in zip(es, ex):
            for _ in range(p):
                poly = _poly_mul(poly, e_k)
        out.append(_exact_mean(poly, d))
    return np.array(out)


# ------------------------------------------------------------------ orbits
def _orbit_points(kind, params, d):
    if d == 2:
        if kind == "S3":
            base = (1 / 3, 1 / 3, 1 / 3)
        elif kind == "S21":
            a, = params
            base = (a, a, 1 - 2 * a)
        elif kind == "S111":
            a, b = params
            base = (a, b, 1 - a - b)
        else:
            raise ValueError(kind)
    else:
        if kind == "S4":
            base = (0.25, 0.25, 0.25, 0.25)
        elif kind == "S31":
            a, = params
            base = (a, a, a, 1 - 3 * a)
        elif kind == "S22":
            b, = params
            base = (b, b, 0.5 - b, 0.5 - b)
        else:
            raise ValueError(kind)
    pts = []
    for perm in permutations(range(d + 1)):
        q = tuple(base[i] for i in perm)
        if q not in pts:
            pts.append(q)
    return np.array(pts)


_NPARAM = {"S3": 0, "S4": 0, "S21": 1, "S31": 1, "S22": 1, "S111": 2}


def _assemble(structure, x, d):
    pts, ws = [], []
    i = 0
    for kind in structure:
        w = x[i]
        i += 1
        par = x[i:i + _NPARAM[kind]]
        i += _NPARAM[kind]
        p = _orbit_points(kind, par, d)
        pts.append(p)
        ws.append(np.full(p.shape[0], w))
    return np.concatenate(pts), np.concatenate(ws)


def _solve_symmetric(structure, guess, d, degree):
    exps = _invariant_exponents(d, degree)
    target = _invariant_means(d, exps)
    x = np.array(guess, dtype=np.float64)
    if len(exps) != len(x):
        raise ValueError("moment system is not square")

    def resid(v):
        p, w = _assemble(structure, v, d)
        return _invariants_numeric(p, exps).T @ w - target

    for _ in range(60):
        r = resid(x)
        if np.max(np.abs(r)) < 4e-17:
            break
        J = np.empty((len(r), len(x)))
        for k in range(len(x)):
            h = 1e-7 * max(1.0, abs(x[k]))
            xp, xm = x.copy(), x.copy()
            xp[k] += h
            xm[k] -= h
            J[:, k] = (resid(xp) - resid(xm)) / (2 * h)
        x = x - np.linalg.solve(J, r)
    x = _polish_symmetric(structure, x, d, exps)
    pts, w = _assemble(structure, x, d)
    return pts, w


def _polish_symmetric(structure, x, d, exps, dps=50):
    """Newton on the same invariant equations in dps-digit arithmetic (mpmath),
    with the exact means as targets; the parameters are then rounded once to
    double, so the rule is the double rule nearest the exact one rather than
    one limited by the rounding of a double-precision Newton iteration."""
    import mpmath as mp
    d1 = d + 1
    with mp.workdps(dps):
        es_poly = [_elem_sym(d1, k) for k in range(2, d1 + 1)]
        target = []
        for ex in exps:
            poly = {tuple([0] * d1): Fraction(1)}
            for e_k, p in zip(es_poly, ex):
                for _ in range(p):
                    poly = _poly_mul(poly, e_k)
            s = Fraction(0)
            for e, c in poly.items():
                num = factorial(d)
                for a in e:
                    num *= factorial(a)
                s += c * Fraction(num, factorial(sum(e) + d))
            target.append(mp.mpf(s.numerator) / s.denominator)

        def points(v):
            pts, ws, i = [], [], 0
            for kind in structure:
                w = v[i]
                i += 1
                par = v[i:i + _NPARAM[kind]]
                i += _NPARAM[kind]
                half = mp.mpf(1) / 2
                base = {"S3": lambda: [mp.mpf(1) / 3] * 3, "S4": lambda: [mp.mpf(1) / 4] * 4,
                        "S21": lambda: [par[0], par[0], 1 - 2 * par[0]],
                        "S31": lambda: [par[0]] * 3 + [1 - 3 * par[0]],
                        "S22": lambda: [par[0], par[0], half - par[0], half - par[0]],
                        "S111": lambda: [par[0], par[1], 1 - par[0] - par[1]]}[kind]()
                # invariants are symmetric: one representative per orbit, times its size
                size = len(_orbit_points(kind, [float(t) for t in par], d))
                pts.append(base)
                ws.append(w * size)
            return pts, ws

        def resid(v):
            pts, ws = points(v)
            out = []
            for ex, t in zip(exps, target):
                acc = mp.mpf(0)
                for q, w in zip(pts, ws):
                    val = w
                    for k, p in zip(range(2, d1 + 1), ex):
                        ek = mp.mpf(0)
                        for idx in combinations(range(d1), k):
                            prod = mp.mpf(1)
                            for j in idx:
                                prod *= q[j]
                            ek += prod
                        val *= ek ** p
                    acc += val
                out.append(acc - t)
            return mp.matrix(out)

        v = [mp.mpf(float(t)) for t in x]
        for _ in range(6):
            r = resid(v)
            h = mp.mpf(10) ** (-dps // 2)
            J = mp.matrix(len(r), len(v))
            for k in range(len(v)):
                vp, vm = list(v), list(v)
                vp[k] += h
                vm[k] -= h
                col = (resid(vp) - resid(vm)) / (2 * h)
                for j in range(len(r)):
                    J[j, k] = col[j]
            step = mp.lu_solve(J, r)
            v = [v[k] - step[k] for k in range(len(v))]
        if max(abs(t) for t in resid(v)) > mp.mpf(10) ** (-35):
            raise RuntimeError("high-precision Newton did not converge")
        return np.array([float(t) for t in v])


# Starting guesses: the published Dunavant (triangle) and Keast (tetrahedron)
# values, to about 15 digits.  Newton then converges to the exact rule.
_TRI_SPECS = {
    4: (("S21", "S21"),
        (0.223381589678011, 0.445948490915965, 0.109951743655322, 0.091576213509771)),
    6: (("S21", "S21", "S111"),
        (0.116786275726379, 0.249286745170910, 0.050844906370207, 0.063089014491502,
         0.082851075618374, 0.053145049844817, 0.310352451033784)),
    8: (("S3", "S21", "S21", "S21", "S111"),
        (0.144315607677787, 0.095091634267285, 0.459292588292723, 0.103217370534718, 0.170569307751760,
         0.032458497623198, 0.050547228317031, 0.027230314174435, 0.008394777409958, 0.263112829634638)),
}

_TET_SPECS = {
    4: (("S4", "S31", "S22"),
        (-0.0789333333333333, 0.0457333333333333, 0.0714285714285714, 0.1493333333333333, 0.399403576166799)),
}


@lru_cache(maxsize=None)
def triangle_rule(degree: int):
    """Symmetric triangle rule exact for polynomials of total ``degree`` (4, 6 or 8)."""
    structure, guess = _TRI_SPECS[degree]
    return _solve_symmetric(structure, guess, 2, degree)


@lru_cache(maxsize=None)
def tet_rule(degree: int = 4):
    """11-point tetrahedron rule exact for total degree 4."""
    structure, guess = _TET_SPECS[degree]
    return _solve_symmetric(structure, guess, 3, degree)


def triangle_degree_for(p: int) -> int:
    """Degree of the triangle rule used on the fan sub-triangles of a degree-p cell."""
    return max(4, 2 * p)


def edge_points_for(p_face: int) -> int:
    """Gauss points on an edge whose two sides have maximum degree p_face."""
    return max(3, p_face + 1)
