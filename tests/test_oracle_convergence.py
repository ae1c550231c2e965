"""End-to-end pin: solving the oracle's system on refined Lloyd-Voronoi meshes
converges in L2 at the optimal rate h^(p+1) for the smooth manufactured
solution u = sin(pi x) sin(pi y) of the diffusion-advection-reaction problem
with variable diffusion (the problem of the headline workload).  This checks the
matrix and the right-hand side (including the non-polynomial f and the boundary
data) together.  The L2 error uses its own collapsed Gauss rule on each fan
triangle and numpy's Legendre evaluation, independent of the oracle's rules and
basis code.
"""

import numpy as np
import pytest
from numpy.polynomial import legendre as L

import oracle
from meshgen import voronoi_mesh
from tests.polyexact import basis_exponents


def _collapsed_rule(n=7):
    t, w = np.polynomial.legendre.leggauss(n)
    t, w = 0.5 * (t + 1), 0.5 * w
    U, V = np.meshgrid(t, t, indexing="ij")
    W = np.outer(w, w) * (1 - U)
    l1, l2 = U.ravel(), (V * (1 - U)).ravel()
    return np.stack([1 - l1 - l2, l1, l2], 1), 2.0 * W.ravel()  # weights sum to 1


def l2_error(m, coef, pat, geo, uex):
    bary, w = _collapsed_rule()
    err2 = 0.0
    for c in range(m.n_cells):
        p = int(m.cell_p[c])
        ex = basis_exponents(2, p)
        lo, hi = geo["lo"][c, :2], geo["hi"][c, :2]
        box = np.prod(hi - lo)
        cc = coef[pat.dof_ptr[c]:pat.dof_ptr[c + 1]]
        ids = m.cell_vtx[m.cell_ptr[c]:m.cell_ptr[c + 1]]
        xy = np.stack([m.x[ids], m.y[ids]], 1)
        for k in range(1, xy.shape[0] - 1):
            T = np.stack([xy[0], xy[k], xy[k + 1]])
            e1, e2 = T[1] - T[0], T[2] - T[0]
            area = 0.5 * abs(e1[0] * e2[1] - e1[1] * e2[0])
            X = bary @ T
            xi = (2 * X - lo - hi) / (hi - lo)
            uh = np.zeros(X.shape[0])
            for i, (a, b) in enumerate(ex):
                s = np.sqrt((2 * a + 1) * (2 * b + 1) / box)
                uh += cc[i] * s * L.legval(xi[:, 0], [0] * a + [1]) * L.legval(xi[:, 1], [0] * b + [1])
            err2 += area * np.dot(w, (uh - uex(X)) ** 2)
    return np.sqrt(err2)


@pytest.mark.parametrize("p", [1, 2])
def test_l2_convergence_rate(p):
    prob = oracle.Problem(a0=1.0, a1=0.5, b=(1.0, 0.5, 0.0), c=1.0)
    uex = lambda X: np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1])
    errs, hs = [], []
    for n in (16, 64, 256, 1024):
        m = voronoi_mesh(n, 2024 + n, lloyd=10, p=p)
        pat = oracle.pattern(m)
        vals, rhs = oracle.assemble(m, prob, pat=pat)
        A = oracle.dense(m, pat, vals)
        coef = np.linalg.solve(A, rhs)
        geo = oracle.geometry(m, prob)
        errs.append(l2_error(m, coef, pat, geo, uex))
        hs.append(geo["diam"].mean())
    rates = np.log(np.array(errs[:-1]) / np.array(errs[1:])) / np.log(np.array(hs[:-1]) / np.array(hs[1:]))
    assert rates[-1] >= p + 1 - 0.25, (errs, rates)
    assert errs[-1] < errs[0] / 10
