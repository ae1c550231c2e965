"""Pin for the whole SIPG operator: on a Cartesian grid every cell is its own
bounding box, so every integral in (dg-bilinear) has a closed form from 1D
Legendre identities.  The reference matrix below is built straight from the
paper's definitions -- average {w}, vector jump [v] = v_1 n_1 + v_2 n_2, upwind
jump on the inflow part of each element boundary, penalty on interior and
Dirichlet faces -- with no quadrature, no polygon machinery and no row-owner
rewriting.  A sign, index or orientation slip in the oracle fails it.

1D identities on an interval of length h (P_n of the mapped coordinate):
  int P_m P_n      = h/(2m+1) delta_mn
  int P_m' P_n'    = (2/h) min(m,n)(min(m,n)+1)   if m+n even, else 0
  int P_m' P_n     = 2                            if n < m and m-n odd, else 0
  P_n(+-1) = (+-1)^n,   dP_n/dxi(+-1) = (+-1)^(n+1) n(n+1)/2
"""

import numpy as np
import pytest

import oracle
from meshgen import cartesian_mesh
from tests.polyexact import basis_exponents


def K1(m, n):
    k = min(m, n)
    return k * (k + 1) if (m + n) % 2 == 0 else 0.0


def G1(m, n):
    return 2.0 if (n < m and (m - n) % 2 == 1) else 0.0


def trace(n, side):
    """(P_n(side), dP_n/dxi(side)) for side = +1 or -1."""
    return side ** n, side ** (n + 1) * n * (n + 1) / 2.0


def closed_form_matrix(nx, ny, x0, x1, y0, y1, p, a, b, c, csig=10.0):
    hx, hy = (x1 - x0) / nx, (y1 - y0) / ny
    ex = basis_exponents(2, p)
    nb = len(ex)
    N = nx * ny
    A = np.zeros((N * nb, N * nb))
    s = lambda e: np.sqrt((2 * e[0] + 1) / hx) * np.sqrt((2 * e[1] + 1) / hy)
    cid = lambda i, j: j * nx + i
    h = np.hypot(hx, hy)
    sigma = csig * a * p * p / h

    # element terms
    for j in range(ny):
        for i in range(nx):
            K = cid(i, j)
            for ti, (ai, bi) in enumerate(ex):
                for tj, (aj, bj) in enumerate(ex):
                    ss = s((ai, bi)) * s((aj, bj))
                    mx = hx / (2 * ai + 1) if ai == aj else 0.0
                    my = hy / (2 * bi + 1) if bi == bj else 0.0
                    kx = 2.0 / hx * K1(aj, ai)
                    ky = 2.0 / hy * K1(bj, bi)
                    val = a * (kx * my + mx * ky)
                    val += b[0] * G1(aj, ai) * my + b[1] * mx * G1(bj, bi)
                    val += c * mx * my
                    A[K * nb + ti, K * nb + tj] += ss * val

    def face_terms(sides, along_h, normal_axis):
        """sides: list of (cell, side_of_that_cell (+1/-1), outward normal sign along normal_axis).
        Face is perpendicular to normal_axis; tangential 1D integrals give along_h/(2k+1) delta."""
        hn = hx if normal_axis == 0 else hy
        bnorm = b[normal_axis]
        # per side: value trace and normal-derivative trace (w.r.t. the global +axis direction)
        for (Kv, sv, nv) in sides:          # test function side
            for ti, ev in enumerate(ex):
                for (Kw, sw, nw) in sides:  # trial function side
                    for tj, ew in enumerate(ex):
                        tv = ev[1 - normal_axis]
                        tw = ew[1 - normal_axis]
                        if tv != tw:
                            continue
                        tang = along_h / (2 * tv + 1)
                        ss = s(ev) * s(ew)
                        vv, dv = trace(ev[normal_axis], sv)
                        ww, dw = trace(ew[normal_axis], sw)
                        dv *= 2.0 / hn  # d/d(axis) of v on its side
                        dw *= 2.0 / hn
                        nsides = len(sides)
                        # jumps as scalars along the first side's outward normal n_1:
                        # [v] . n_1 = v_1 - v_2 (interior) or v_1 (boundary)
                        n1 = sides[0][2]
                        jv = vv * (1.0 if Kv == sides[0][0] else -1.0)
                        jw = ww * (1.0 if Kw == sides[0][0] else -1.0)
                        # average of A grad . n_1 ; on a boundary face the average is the trace
                        avg = 0.5 if nsides == 2 else 1.0
                        fw = avg * a * dw * n1
                        fv = avg * a * dv * n1
                        val = -(fw * jv + fv * jw - sigma * jw * jv)
                        # upwind terms, written for the test function's element K = Kv
                        bn = bnorm * nv  # b . n_Kv
                        if bn < 0:
                            if Kw == Kv:
                                val += -bn * ww * vv
                            elif nsides == 2:
                                val += bn * ww * vv
                        A[Kv * nb + ti, Kw * nb + tj] += ss * tang * val

    # vertical faces
    for j in range(ny):
        for i in range(nx + 1):
            if 0 < i < nx:
                face_terms([(cid(i - 1, j), +1, +1), (cid(i, j), -1, -1)], hy, 0)
            elif i == 0:
                face_terms([(cid(0, j), -1, -1)], hy, 0)
            else:
                face_terms([(cid(nx - 1, j), +1, +1)], hy, 0)
    # horizontal faces
    for j in range(ny + 1):
        for i in range(nx):
            if 0 < j < ny:
                face_terms([(cid(i, j - 1), +1, +1), (cid(i, j), -1, -1)], hx, 1)
            elif j == 0:
                face_terms([(cid(i, 0), -1, -1)], hx, 1)
            else:
                face_terms([(cid(i, ny - 1), +1, +1)], hx, 1)
    return A


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("coef", [(1.0, (0.0, 0.0), 0.0), (0.7, (0.8, -0.6), 1.3), (1.2, (-0.5, 0.9), 0.0)])
def test_cartesian_closed_form(p, coef):
    a, b, c = coef
    nx, ny, x0, x1, y0, y1 = 3, 2, 0.2, 1.1, -0.3, 0.5
    m = cartesian_mesh(nx, ny, p=p, x0=x0, x1=x1, y0=y0, y1=y1)
    prob = oracle.Problem(a0=a, a1=0.0, b=(b[0], b[1], 0.0), c=c)
    pat = oracle.pattern(m)
    vals, _ = oracle.assemble(m, prob, pat=pat)
    A = oracle.dense(m, pat, vals)
    R = closed_form_matrix(nx, ny, x0, x1, y0, y1, p, a, b, c)
    assert np.abs(A - R).max() <= 1e-13 * np.abs(R).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_cartesian_closed_form_small_cells_far_from_the_origin(p):
    """Cells of 2^-13 x 2^-14 at (0.75, 0.875) (every vertex exact in binary):
    the same closed forms to 1e-13.  A double near 0.8 is known only to ~1e-16,
    i.e. 1e-12 of such a cell, so this pins that quadrature points enter the
    basis through their offsets from a mesh vertex, not through their absolute
    coordinates (which lose about three digits here)."""
    a, b, c = 0.7, (0.8, -0.6), 1.3
    nx, ny = 3, 2
    hx, hy = 2.0 ** -13, 2.0 ** -14
    x0, y0 = 0.75, 0.875
    x1, y1 = x0 + nx * hx, y0 + ny * hy
    m = cartesian_mesh(nx, ny, p=p, x0=x0, x1=x1, y0=y0, y1=y1)
    assert np.array_equal(np.unique(m.x), x0 + hx * np.arange(nx + 1))
    prob = oracle.Problem(a0=a, a1=0.0, b=(b[0], b[1], 0.0), c=c)
    pat = oracle.pattern(m)
    vals, _ = oracle.assemble(m, prob, pat=pat)
    A = oracle.dense(m, pat, vals)
    R = closed_form_matrix(nx, ny, x0, x1, y0, y1, p, a, b, c)
    assert np.abs(A - R).max() <= 1e-13 * np.abs(R).max()
