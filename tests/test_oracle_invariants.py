"""Invariant pins for the oracle on Voronoi meshes (Section 2.2 and the
penalty reading of Appendix A):

* symmetry of the SIPG operator when b = 0, also with variable a;
* constants: for rows with no boundary face, A u_1 = int c phi_i (the interior
  operator annihilates constants);
* polynomial reproduction: with constant coefficients and u in P_2, A Pi(u) = F
  (consistency of SIPG + exact quadrature), uniform and mixed degrees;
* first-order upwind finite volumes as the p = 0, a = 0 special case;
* the penalty formula on every face.
"""

import numpy as np
import pytest

import oracle
from meshgen import cartesian_mesh, split_cartesian_mesh, voronoi_mesh
from tests import polyexact as PE


def _cell_xy(m, c):
    ids = m.cell_vtx[m.cell_ptr[c]:m.cell_ptr[c + 1]]
    return np.stack([m.x[ids], m.y[ids]], 1)


def _box_projection(m, geo, func, p_of):
    """Coefficients of func in each cell's orthonormal box basis (tensor Gauss on the box)."""
    out = []
    for c in range(m.n_cells):
        p = int(p_of[c])
        lo, hi = geo["lo"][c, :2], geo["hi"][c, :2]
        t, w = np.polynomial.legendre.leggauss(p + 3)
        coef = np.zeros(oracle.nb(2, p))
        for i, ti in enumerate(t):
            for j, tj in enumerate(t):
                x = lo + 0.5 * (np.array([ti, tj]) + 1) * (hi - lo)
                phi, _ = oracle.basis(2, p, lo, hi, x)
                coef += w[i] * w[j] * np.prod(0.5 * (hi - lo)) * func(x) * phi
        out.append(coef)
    return np.concatenate(out)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_symmetric_without_advection(p):
    m = voronoi_mesh(60, 11, lloyd=3, p=p)
    pat = oracle.pattern(m)
    vals, _ = oracle.assemble(m, oracle.Problem(a0=1.0, a1=0.5, c=1.0), pat=pat)
    A = oracle.dense(m, pat, vals)
    assert np.linalg.norm(A - A.T) <= 1e-14 * np.linalg.norm(A)
    # with advection the operator is not symmetric
    vals, _ = oracle.assemble(m, oracle.Problem(a0=1.0, a1=0.5, b=(1.0, 0.5, 0.0), c=1.0), pat=pat)
    A = oracle.dense(m, pat, vals)
    assert np.linalg.norm(A - A.T) > 1e-6 * np.linalg.norm(A)


@pytest.mark.parametrize("p", [1, 2])
def test_constants_annihilated_in_interior_rows(p):
    m = voronoi_mesh(80, 12, lloyd=3, p=p)
    pat = oracle.pattern(m)
    prob = oracle.Problem(a0=1.0, a1=0.5, b=(1.0, 0.5, 0.0), c=1.0)
    vals, _ = oracle.assemble(m, prob, pat=pat)
    A = oracle.dense(m, pat, vals)
    geo = oracle.geometry(m, prob)
    nb = oracle.nb(2, p)
    u1 = np.zeros(A.shape[0])
    box = np.prod(geo["hi"][:, :2] - geo["lo"][:, :2], axis=1)
    u1[0::nb] = np.sqrt(box)
    r = A @ u1
    interior = [c for c in range(m.n_cells)
                if all(m.face_bc[f] == 0 for f in m.cell_face[m.cell_face_ptr[c]:m.cell_face_ptr[c + 1]])]
    assert len(interior) > 10
    for c in interior:
        lo, hi = geo["lo"][c, :2], geo["hi"][c, :2]
        xy, J = PE.to_box(_cell_xy(m, c), lo, hi)
        ref = np.array([J * PE.polygon_integral(xy, poly) for poly in PE.basis_polys_2d(p, lo, hi)])
        got = r[c * nb:(c + 1) * nb]
        assert np.abs(got - prob.c * ref).max() <= 1e-12 * np.abs(A).max() * np.abs(u1).max()


U_POLY = (1.0, 2.0, -1.0, 0.0, 1.0, -0.5, 0.0, 1.0, 0.0, 0.0)  # 1 + 2x - y + x^2 - y^2/2 + xy


def _u_poly(x):
    c = U_POLY
    return c[0] + c[1] * x[0] + c[2] * x[1] + c[4] * x[0] ** 2 + c[5] * x[1] ** 2 + c[7] * x[0] * x[1]


@pytest.mark.parametrize("p", [2, 3, 4, "mixed"])
def test_polynomial_reproduction(p):
    m = voronoi_mesh(50, 13, lloyd=2, p=2)
    if p == "mixed":
        m = m.with_degrees(np.random.default_rng(3).integers(2, 5, m.n_cells))
    else:
        m = m.with_degrees(p)
    prob = oracle.Problem(a0=1.3, a1=0.0, b=(0.4, -0.7, 0.0), c=0.9, u_kind=oracle.U_POLY, u_poly=U_POLY)
    pat = oracle.pattern(m)
    vals, rhs = oracle.assemble(m, prob, pat=pat)
    A = oracle.dense(m, pat, vals)
    geo = oracle.geometry(m, prob)
    pu = _box_projection(m, geo, _u_poly, m.cell_p)
    res = A @ pu - rhs
    assert np.abs(res).max() <= 1e-12 * np.abs(A).max() * np.abs(pu).max()
    # the manufactured f is what the pin relies on: check it against the PDE by hand
    u, f = oracle.exact(prob, 2, np.array([0.3, 0.6]))
    x, y = 0.3, 0.6
    ux, uy, lap = 2 + 2 * x + y, -1 - y + x, 2 - 1
    assert abs(f - (-1.3 * lap + 0.4 * ux - 0.7 * uy + 0.9 * u)) < 1e-14
    assert abs(u - _u_poly((x, y))) < 1e-15


def test_upwind_finite_volume_limit():
    """p = 0 and a = 0: the dG matrix is the textbook first-order upwind FV matrix
    for div(b u) + c u (b constant), scaled by the constant basis 1/sqrt|B|."""
    m = voronoi_mesh(70, 14, lloyd=2, p=0)
    b = np.array([0.8, 0.3])
    prob = oracle.Problem(a0=0.0, a1=0.0, b=(b[0], b[1], 0.0), c=0.5)
    pat = oracle.pattern(m)
    vals, _ = oracle.assemble(m, prob, pat=pat)
    A = oracle.dense(m, pat, vals)
    n = m.n_cells
    area = np.array([PE.polygon_monomial(_cell_xy(m, c), 0, 0) for c in range(n)])
    FV = np.diag(prob.c * area)
    for c in range(n):
        xy = _cell_xy(m, c)
        k = xy.shape[0]
        for e in range(k):
            p0, p1 = xy[e], xy[(e + 1) % k]
            t = p1 - p0
            nrm = np.array([t[1], -t[0]])  # outward for a CCW loop, length |F|
            flux = b @ nrm
            f = m.cell_face[m.cell_face_ptr[c] + e]
            other = m.face_cell[2 * f] if m.face_cell[2 * f] != c else m.face_cell[2 * f + 1]
            if flux >= 0:
                FV[c, c] += flux
            elif other >= 0:
                FV[c, other] += flux
            # inflow through the boundary: data goes to the right-hand side
    geo = oracle.geometry(m, prob)
    box = np.prod(geo["hi"][:, :2] - geo["lo"][:, :2], axis=1)
    scaled = A * np.sqrt(np.outer(box, box))
    assert np.abs(scaled - FV).max() <= 1e-13 * np.abs(FV).max()


def test_penalty_is_max_over_sides():
    """Doubling the penalty constant only changes the penalty part: the change of
    each interior cross block equals -C_sigma * max(abar p^2 / h) * int phi'_j phi_i."""
    m = voronoi_mesh(30, 15, lloyd=2, p=1)
    m = m.with_degrees(np.random.default_rng(1).integers(1, 3, m.n_cells))
    pat = oracle.pattern(m)
    p1 = oracle.Problem(a0=1.0, a1=0.5, c_sigma=10.0)
    p2 = oracle.Problem(a0=1.0, a1=0.5, c_sigma=20.0)
    v1, _ = oracle.assemble(m, p1, pat=pat)
    v2, _ = oracle.assemble(m, p2, pat=pat)
    # with sigma fixed to 1 and only interior terms, the cross block is
    #   (consistency part) - int phi'_j phi_i; the consistency part cancels in a difference
    q1 = oracle.Problem(a0=1.0, a1=0.5, sigma_override=1.0, term_mask=oracle.T_INTERIOR)
    q0 = oracle.Problem(a0=1.0, a1=0.5, sigma_override=0.0, term_mask=oracle.T_INTERIOR)
    w1, _ = oracle.assemble(m, q1, pat=pat)
    w0, _ = oracle.assemble(m, q0, pat=pat)
    geo = oracle.geometry(m, p1)
    for r in range(m.n_cells):
        for k in range(pat.row_ptr[r], pat.row_ptr[r + 1]):
            c = pat.col_idx[k]
            if c == r:
                continue
            sl = slice(pat.val_ptr[k], pat.val_ptr[k + 1])
            sig = 10.0 * max(geo["abar"][r] * m.cell_p[r] ** 2 / geo["diam"][r],
                             geo["abar"][c] * m.cell_p[c] ** 2 / geo["diam"][c])
            mass = w1[sl] - w0[sl]  # = - int phi'_j phi_i over the shared face
            assert np.allclose(v2[sl] - v1[sl], sig * mass, rtol=1e-9, atol=1e-9 * np.abs(v1[sl]).max())


def test_manufactured_load_matches_the_pde():
    """f = -div(a grad u) + b.grad u + c u (equation CDR) against central
    differences of u and a computed here with numpy; u vanishes exactly on the
    boundary of the unit square (the Dirichlet data)."""
    prob = oracle.Problem(a0=1.0, a1=0.5, b=(1.0, 0.5, 0.0), c=1.0)
    u = lambda x, y: np.sin(np.pi * x) * np.sin(np.pi * y)
    a = lambda x, y: 1.0 + 0.5 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
    h = 1e-4
    rng = np.random.default_rng(4)
    for x, y in rng.random((20, 2)):
        flux_x = lambda s, t: a(s, t) * (u(s + h, t) - u(s - h, t)) / (2 * h)
        flux_y = lambda s, t: a(s, t) * (u(s, t + h) - u(s, t - h)) / (2 * h)
        div = (flux_x(x + h, y) - flux_x(x - h, y)) / (2 * h) + (flux_y(x, y + h) - flux_y(x, y - h)) / (2 * h)
        ux = (u(x + h, y) - u(x - h, y)) / (2 * h)
        uy = (u(x, y + h) - u(x, y - h)) / (2 * h)
        f_fd = -div + 1.0 * ux + 0.5 * uy + 1.0 * u(x, y)
        uu, f = oracle.exact(prob, 2, np.array([x, y]))
        assert abs(uu - u(x, y)) < 1e-15
        assert abs(f - f_fd) < 1e-5 * max(1.0, abs(f))
    for x, y in ((0.0, 0.37), (1.0, 0.81), (0.42, 0.0), (0.77, 1.0), (1.0, 1.0)):
        assert oracle.exact(prob, 2, np.array([x, y]))[0] == 0.0


@pytest.mark.parametrize("p", [1, 2])
def test_split_edges_change_nothing(p):
    """Splitting every side of a rectangular grid at its midpoint (octagons with
    collinear vertices; neighbours share two edges, some fan triangles are
    degenerate) describes the same cells and faces: with polynomial data every
    integral is exact on each half, so the pattern and the matrix are those of
    the plain grid."""
    prob = oracle.Problem(a0=1.3, a1=0.0, b=(0.4, -0.7, 0.0), c=0.9, u_kind=oracle.U_POLY, u_poly=U_POLY)
    plain = cartesian_mesh(4, 3, p=p, x0=0.1, x1=1.3, y0=-0.2, y1=0.9)
    split = split_cartesian_mesh(4, 3, p=p, x0=0.1, x1=1.3, y0=-0.2, y1=0.9)
    pa, ps = oracle.pattern(plain), oracle.pattern(split)
    for k in ("row_ptr", "col_idx", "val_ptr", "dof_ptr"):
        assert np.array_equal(getattr(pa, k), getattr(ps, k))
    va, fa = oracle.assemble(plain, prob, pat=pa)
    vs, fs = oracle.assemble(split, prob, pat=ps)
    assert np.abs(va - vs).max() <= 1e-12 * np.abs(va).max()
    assert np.abs(fa - fs).max() <= 1e-12 * np.abs(fa).max()


def test_openmp_build_is_the_same_oracle():
    """The OpenMP build (rows over threads, for the all-core CPU baseline) gives
    bit-identical values: every row is the same arithmetic in the same order."""
    m = voronoi_mesh(400, 31, lloyd=1, p=1)
    m = m.with_degrees(np.random.default_rng(2).integers(1, 5, m.n_cells))
    prob = oracle.Problem(a0=1.0, a1=0.5, b=(1.0, 0.5, 0.0), c=1.0)
    pat = oracle.pattern(m)
    v1, r1 = oracle.assemble(m, prob, pat=pat)
    v2, r2 = oracle.assemble(m, prob, pat=pat, parallel=True)
    assert np.array_equal(v1, v2) and np.array_equal(r1, r2)
    assert oracle.threads() == 1
