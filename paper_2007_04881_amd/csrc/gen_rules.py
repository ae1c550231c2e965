#!/usr/bin/env python3
"""Generate rules_data.h: the quadrature rules compiled into the HIP kernels.

The method applies standard rules on each simplex of a subdivision and on each
simplicial sub-face (Section 3).  The rules are derived here in double precision
and emitted as hex-float constants:

* Gauss-Legendre on [0, 1] with n = 1..16 points: Golub-Welsch (eigen-
  decomposition of the symmetric Jacobi matrix of the Legendre recurrence),
  then two Newton polishing steps on P_n.
* Fully symmetric triangle rules of degree 4 (6 points), 6 (12) and 8 (16)
  and the 11-point degree-4 tetrahedron rule: orbit parameters fitted by
  Gauss-Newton to *all* Cartesian monomial moments x^a y^b (z^c) of the
  reference simplex up to the degree (exact values a! b! c! / (a+b+c+d)!),
  started from rounded published values (Dunavant for triangles, Keast for
  the tetrahedron), then polished by the same Gauss-Newton iteration in
  60-digit arithmetic (mpmath) and rounded once to double precision, so that
  each emitted rule is the nearest double rule to the exact one (moment
  residuals at the rounding level of the data, not of the double-precision
  fit).  The Gauss-Legendre nodes and weights are polished the same way.

Run:  python gen_rules.py > rules_data.h
"""

import sys
from math import factorial

import numpy as np


def gauss_legendre(n):
    k = np.arange(1, n)
    beta = k / np.sqrt(4.0 * k * k - 1.0)
    J = np.diag(beta, 1) + np.diag(beta, -1)
    x, V = np.linalg.eigh(J)
    for _ in range(2):
        p0, p1 = np.ones_like(x), x.copy()
        for m in range(2, n + 1):
            p0, p1 = p1, ((2 * m - 1) * x * p1 - (m - 1) * p0) / m
        if n == 1:
            p0, p1 = np.ones_like(x), x.copy()
        dp = n * (x * p1 - p0) / (x * x - 1.0)
        x = x - p1 / dp
    p0, p1 = np.ones_like(x), x.copy()
    for m in range(2, n + 1):
        p0, p1 = p1, ((2 * m - 1) * x * p1 - (m - 1) * p0) / m
    if n == 1:
        p0, p1 = np.ones_like(x), x.copy()
    dp = n * (x * p1 - p0) / (x * x - 1.0)
    w = 2.0 / ((1.0 - x * x) * dp * dp)
    o = np.argsort(x)
    return 0.5 * (x[o] + 1.0), 0.5 * w[o]


def gauss_legendre_mp(n, dps=60):
    """The n-point rule on [0, 1] polished by Newton on P_n in dps-digit arithmetic."""
    import mpmath as mp
    t0, _ = gauss_legendre(n)
    with mp.workdps(dps):
        xs, ws = [], []
        for t in t0:
            x = mp.mpf(2) * mp.mpf(float(t)) - 1
            for _ in range(8):
                x = x - mp.legendre(n, x) / mp.diff(lambda z: mp.legendre(n, z), x)
            dp = mp.diff(lambda z: mp.legendre(n, z), x)
            xs.append((x + 1) / 2)
            ws.append(1 / ((1 - x * x) * dp * dp))
        return np.array([float(v) for v in xs]), np.array([float(v) for v in ws])


def _orbit(kind, par, d):
    if kind == "c":
        base = [1.0 / (d + 1)] * (d + 1)
    elif kind == "a":          # d points equal to a, one 1 - d a
        base = [par[0]] * d + [1 - d * par[0]]
    elif kind == "ab":         # triangle (a, b, 1-a-b)
        base = [par[0], par[1], 1 - par[0] - par[1]]
    elif kind == "bb":         # tetrahedron (b, b, 1/2-b, 1/2-b)
        base = [par[0], par[0], 0.5 - par[0], 0.5 - par[0]]
    pts = set()
    import itertools
    for perm in itertools.permutations(range(d + 1)):
        pts.add(tuple(base[i] for i in perm))
    return sorted(pts)


_NP = {"c": 0, "a": 1, "ab": 2, "bb": 1}


def _build(struct, x, d):
    P, W = [], []
    i = 0
    for kind in struct:
        w = x[i]
        par = x[i + 1:i + 1 + _NP[kind]]
        i += 1 + _NP[kind]
        for q in _orbit(kind, par, d):
            P.append(q)
            W.append(w)
    return np.array(P), np.array(W)


def _moments(d, deg):
    ex = []
    if d == 2:
        for a in range(deg + 1):
            for b in range(deg + 1 - a):
                ex.append((a, b))
    else:
        for a in range(deg + 1):
            for b in range(deg + 1 - a):
                for c in range(deg + 1 - a - b):
                    ex.append((a, b, c))
    vol = 1.0 / factorial(d)
    ref = []
    for e in ex:
        num = 1
        for k in e:
            num *= factorial(k)
        ref.append(num / factorial(sum(e) + d) / vol)  # mean over the simplex
    return ex, np.array(ref)


def fit_rule(struct, guess, d, deg):
    ex, ref = _moments(d, deg)

    def resid(x):
        P, W = _build(struct, x, d)
        cart = P[:, 1:]  # Cartesian coordinates on the reference simplex
        return np.array([np.dot(W, np.prod(cart ** np.array(e), axis=1)) for e in ex]) - ref

    x = np.array(guess, float)
    for _ in range(100):
        r = resid(x)
        if np.abs(r).max() < 3e-17:
            break
        J = np.empty((r.size, x.size))
        for k in range(x.size):
            h = 1e-7
            xp, xm = x.copy(), x.copy()
            xp[k] += h
            xm[k] -= h
            J[:, k] = (resid(xp) - resid(xm)) / (2 * h)
        x = x - np.linalg.lstsq(J, r, rcond=None)[0]
    if np.abs(resid(x)).max() > 1e-15:
        raise RuntimeError("rule fit did not converge")
    x = _polish_mp(struct, x, d, ex)
    return _build(struct, x, d)


def _orbit_mp(kind, par, d, mp):
    if kind == "c":
        base = [mp.mpf(1) / (d + 1)] * (d + 1)
    elif kind == "a":
        base = [par[0]] * d + [1 - d * par[0]]
    elif kind == "ab":
        base = [par[0], par[1], 1 - par[0] - par[1]]
    elif kind == "bb":
        base = [par[0], par[0], mp.mpf(1) / 2 - par[0], mp.mpf(1) / 2 - par[0]]
    import itertools
    # the same permutations, in the same order, as the double-precision orbits
    out, seen = [], []
    ref = _orbit(kind, [float(v) for v in par], d)
    for q in ref:
        for perm in itertools.permutations(range(d + 1)):
            cand = [base[i] for i in perm]
            if all(abs(float(c) - v) < 1e-9 for c, v in zip(cand, q)):
                out.append(cand)
                break
    return out


def _polish_mp(struct, x, d, ex, dps=60):
    """Gauss-Newton on the same moment equations in dps-digit arithmetic."""
    import mpmath as mp
    from fractions import Fraction
    with mp.workdps(dps):
        ref = []
        for e in ex:
            num = 1
            for k in e:
                num *= factorial(k)
            fr = Fraction(num * factorial(d), factorial(sum(e) + d))
            ref.append(mp.mpf(fr.numerator) / fr.denominator)

        def resid(xv):
            rows, i = [], 0
            pts, wts = [], []
            for kind in struct:
                w = xv[i]
                par = xv[i + 1:i + 1 + _NP[kind]]
                i += 1 + _NP[kind]
                for q in _orbit_mp(kind, par, d, mp):
                    pts.append(q)
                    wts.append(w)
            for e, rv in zip(ex, ref):
                s = mp.mpf(0)
                for q, w in zip(pts, wts):
                    t = w
                    for k, a in enumerate(e):
                        t *= q[k + 1] ** a
                    s += t
                rows.append(s - rv)
            return mp.matrix(rows)

        xv = [mp.mpf(float(v)) for v in x]
        for _ in range(6):
            r = resid(xv)
            h = mp.mpf(10) ** (-dps // 2)
            J = mp.matrix(len(r), len(xv))
            for k in range(len(xv)):
                xp = list(xv)
                xm = list(xv)
                xp[k] += h
                xm[k] -= h
                col = (resid(xp) - resid(xm)) / (2 * h)
                for j in range(len(r)):
                    J[j, k] = col[j]
            step = mp.lu_solve(J.T * J, J.T * r)
            xv = [xv[k] - step[k] for k in range(len(xv))]
        if max(abs(v) for v in resid(xv)) > mp.mpf(10) ** (-40):
            raise RuntimeError("high-precision polish did not converge")
        return np.array([float(v) for v in xv])


TRI = {
    4: (("a", "a"), (0.2233815897, 0.4459484909, 0.1099517437, 0.0915762135)),
    6: (("a", "a", "ab"), (0.1167862757, 0.2492867452, 0.0508449064, 0.0630890145,
                           0.0828510756, 0.0531450498, 0.3103524510)),
    8: (("c", "a", "a", "a", "ab"), (0.1443156077, 0.0950916343, 0.4592925883, 0.1032173705, 0.1705693078,
                                     0.0324584976, 0.0505472283, 0.0272303142, 0.0083947774, 0.2631128296)),
}
TET4 = (("c", "a", "bb"), (-0.0789333333, 0.0457333333, 0.0714285714, 0.1493333333, 0.3994035762))


def hexf(v):
    return float(v).hex()


def emit(out):
    w = out.write
    w("// Generated by gen_rules.py -- quadrature rules for the assembly kernels.\n")
    w("// Weights sum to 1 (multiply by the simplex measure).\n#pragma once\n\n")
    w("#define DGP_GL_MAX 16\n")
    ts, ws, offs = [], [], [0]
    for n in range(1, 17):
        t, wt = gauss_legendre_mp(n)
        ts.extend(t)
        ws.extend(wt)
        offs.append(len(ts))
    w("static __constant__ int c_gl_off[%d] = {%s};\n" % (len(offs), ", ".join(map(str, offs))))
    w("static __constant__ double c_gl_t[%d] = {%s};\n" % (len(ts), ", ".join(map(hexf, ts))))
    w("static __constant__ double c_gl_w[%d] = {%s};\n\n" % (len(ws), ", ".join(map(hexf, ws))))
    for deg, (st, g) in TRI.items():
        P, W = fit_rule(st, g, 2, deg)
        w("#define DGP_TRI%d_N %d\n" % (deg, len(W)))
        w("static __constant__ double c_tri%d_l[%d] = {%s};\n" % (deg, P.size, ", ".join(map(hexf, P.ravel()))))
        w("static __constant__ double c_tri%d_w[%d] = {%s};\n\n" % (deg, W.size, ", ".join(map(hexf, W))))
    P, W = fit_rule(*TET4, 3, 4)
    w("#define DGP_TET4_N %d\n" % len(W))
    w("static __constant__ double c_tet4_l[%d] = {%s};\n" % (P.size, ", ".join(map(hexf, P.ravel()))))
    w("static __constant__ double c_tet4_w[%d] = {%s};\n" % (W.size, ", ".join(map(hexf, W))))


if __name__ == "__main__":
    emit(sys.stdout)
