"""Pins for the oracle in three dimensions, on polyhedra agglomerated from Kuhn
tetrahedra (Section 3: quadrature on the tetrahedra of each polyhedron and on
its boundary triangles; Section 3.1: bounding-box Legendre basis).

* The mesh generator: a partition of the tetrahedra into connected clusters,
  closed cell surfaces, total volume 1.
* Mass, stiffness and advection element blocks against exact integrals by the
  divergence theorem over the cell's boundary triangles (tests/polyexact.py).
* Cubic cells (each its own bounding box): the mass block is the identity and
  the stiffness block has the closed form of the Legendre derivative integrals.
* Symmetry when b = 0, constants annihilated in interior rows, and polynomial
  reproduction with constant coefficients (which checks every face normal,
  the upwind side and the Dirichlet terms).
"""

import numpy as np
import pytest

import oracle
from meshgen.kuhn import agglomerated_cube, cube_cells
from tests import polyexact as PE


def _diag_blocks(m, pat, vals):
    out = []
    for r in range(m.n_cells):
        nb = oracle.nb(3, int(m.cell_p[r]))
        k = [k for k in range(pat.row_ptr[r], pat.row_ptr[r + 1]) if pat.col_idx[k] == r][0]
        out.append(vals[pat.val_ptr[k]:pat.val_ptr[k + 1]].reshape(nb, nb))
    return out


def _tris_box(m, c, lo, hi):
    tris = PE.cell_triangles_outward(m, c)
    return (2 * tris - lo - hi) / (hi - lo)


def test_kuhn_agglomeration_structure():
    m = agglomerated_cube(6, 9, 123, p=1)
    T = m.cell_vtx.shape[0] // 4
    assert T == 6 * 6 ** 3
    xyz = np.stack([m.x, m.y, m.z], 1)
    v = xyz[m.cell_vtx.reshape(-1, 4)]
    vol = np.abs(np.einsum("ij,ij->i", v[:, 1] - v[:, 0], np.cross(v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]))) / 6
    assert abs(vol.sum() - 1.0) < 1e-13
    assert np.allclose(vol, 1.0 / (6 * 6 ** 3), rtol=1e-12)
    fc = m.face_cell.reshape(-1, 2)
    assert (fc[:, 0] < np.where(fc[:, 1] < 0, np.iinfo(np.int32).max, fc[:, 1])).all()
    for c in range(m.n_cells):
        tris = PE.cell_triangles_outward(m, c)
        S = 0.5 * np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0]).sum(0)
        assert np.abs(S).max() < 1e-14  # closed surface
        # divergence theorem for x: the cell volume
        xs = tris.mean(1)[:, 0]
        flux = (0.5 * np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0])[:, 0] * xs).sum()
        n_t = (m.cell_ptr[c + 1] - m.cell_ptr[c]) // 4
        assert abs(flux - n_t / (6 * 6 ** 3)) < 1e-14
        # connected through interior tetrahedron faces
        tets = m.cell_vtx[m.cell_ptr[c]:m.cell_ptr[c + 1]].reshape(-1, 4)
        keys = {}
        for t, tv in enumerate(tets):
            for q in range(4):
                keys.setdefault(tuple(sorted(np.delete(tv, q))), []).append(t)
        adj = {t: set() for t in range(len(tets))}
        for ts in keys.values():
            if len(ts) == 2:
                adj[ts[0]].add(ts[1])
                adj[ts[1]].add(ts[0])
        seen, stack = {0}, [0]
        while stack:
            for u in adj[stack.pop()]:
                if u not in seen:
                    seen.add(u)
                    stack.append(u)
        assert len(seen) == len(tets)
    # each interior face is listed by both of its cells, each boundary face once
    listed = np.bincount(m.cell_face, minlength=m.n_faces)
    assert (listed == np.where(fc[:, 1] >= 0, 2, 1)).all()
    assert (m.face_bc == np.where(fc[:, 1] < 0, 1, 0)).all()
    # deterministic in the seed
    m2 = agglomerated_cube(6, 9, 123, p=1)
    assert all(np.array_equal(a, b) for a, b in zip(m.arrays().values(), m2.arrays().values()))


@pytest.mark.parametrize("mesh", ["agglo", "cubes"])
@pytest.mark.parametrize("p", [1, 2])
def test_element_blocks_against_divergence_theorem(mesh, p):
    m = agglomerated_cube(4, 5, 321, p=p) if mesh == "agglo" else cube_cells(2, p=p)
    pat = oracle.pattern(m)
    b = np.array([0.3, -0.7, 0.5])
    cases = {
        "mass": oracle.Problem(a0=0.0, c=1.0, term_mask=oracle.T_VOLUME),
        "stiff": oracle.Problem(a0=1.0, c=0.0, term_mask=oracle.T_VOLUME),
        "adv": oracle.Problem(a0=0.0, c=0.0, b=tuple(b), term_mask=oracle.T_VOLUME),
    }
    blocks = {k: _diag_blocks(m, pat, oracle.assemble(m, pr, pat=pat)[0]) for k, pr in cases.items()}
    geo = oracle.geometry(m)
    for c in range(m.n_cells):
        lo, hi = geo["lo"][c], geo["hi"][c]
        J = np.prod(hi - lo) / 8.0
        sc = 2.0 / (hi - lo)
        tris = _tris_box(m, c, lo, hi)
        polys = PE.basis_polys_3d(p, lo, hi)
        n = len(polys)
        ref = {k: np.zeros((n, n)) for k in cases}
        for i in range(n):
            for j in range(n):
                ref["mass"][i, j] = J * PE.polyhedron_integral_box(tris, PE.mul3(polys[i], polys[j]))
                st, ad = 0.0, 0.0
                for d in range(3):
                    gi, gj = PE.d3(polys[i], d) * sc[d], PE.d3(polys[j], d) * sc[d]
                    st += PE.polyhedron_integral_box(tris, PE.mul3(gi, gj))
                    ad += b[d] * PE.polyhedron_integral_box(tris, PE.mul3(gj, polys[i]))
                ref["stiff"][i, j] = J * st
                ref["adv"][i, j] = J * ad
        for k in cases:
            assert np.abs(blocks[k][c] - ref[k]).max() <= 1e-13 * np.abs(ref[k]).max(), (k, c)
        assert abs(geo["meas"][c] - J * PE.polyhedron_integral_box(tris, np.ones((1, 1, 1)))) < 1e-14


@pytest.mark.parametrize("p", [1, 2])
def test_cubic_cells_closed_form(p):
    """A cubic cell is its own bounding box: orthonormality gives the identity
    mass block (the degree-4 tetrahedron rule integrates it exactly for p <= 2), and int_{-1}^{1} P_m' P_n' = min(m,n)(min(m,n)+1) for m+n even
    (0 otherwise) gives the stiffness block."""
    m = cube_cells(2, p=p)
    pat = oracle.pattern(m)
    mass = _diag_blocks(m, pat, oracle.assemble(m, oracle.Problem(a0=0.0, c=1.0, term_mask=oracle.T_VOLUME),
                                                pat=pat)[0])
    stiff = _diag_blocks(m, pat, oracle.assemble(m, oracle.Problem(a0=1.0, c=0.0, term_mask=oracle.T_VOLUME),
                                                 pat=pat)[0])
    e = PE.basis_exponents(3, p)
    n = len(e)
    h = 0.5
    S = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            for d in range(3):
                if any(e[i][k] != e[j][k] for k in range(3) if k != d):
                    continue
                a, b = e[i][d], e[j][d]
                if (a + b) % 2:
                    continue
                mn = min(a, b)
                # s_i s_j (2/h)^2 J prod_{k != d} 2/(2e+1) * mn(mn+1), with s = sqrt(prod(2e+1)/h^3), J = h^3/8
                S[i, j] += np.sqrt((2 * a + 1) * (2 * b + 1)) / 2.0 * mn * (mn + 1) * (2.0 / h) ** 2
    for c in range(m.n_cells):
        assert np.abs(mass[c] - np.eye(n)).max() < 1e-14
        assert np.abs(stiff[c] - S).max() < 1e-13 * np.abs(S).max()


@pytest.mark.parametrize("p", [1, 2])
def test_symmetric_without_advection_3d(p):
    m = agglomerated_cube(4, 6, 55, p=p)
    pat = oracle.pattern(m)
    A = oracle.dense(m, pat, oracle.assemble(m, oracle.Problem(a0=1.0, c=1.0), pat=pat)[0])
    assert np.linalg.norm(A - A.T) <= 1e-14 * np.linalg.norm(A)
    A = oracle.dense(m, pat, oracle.assemble(m, oracle.Problem(a0=1.0, b=(0.5, -0.3, 0.8), c=1.0), pat=pat)[0])
    assert np.linalg.norm(A - A.T) > 1e-6 * np.linalg.norm(A)


def test_constants_annihilated_in_interior_rows_3d():
    m = agglomerated_cube(8, 96, 77, p=1)
    pat = oracle.pattern(m)
    prob = oracle.Problem(a0=1.0, b=(0.5, -0.3, 0.8), c=0.7)
    A = oracle.dense(m, pat, oracle.assemble(m, prob, pat=pat)[0])
    geo = oracle.geometry(m, prob)
    nb = oracle.nb(3, 1)
    box = np.prod(geo["hi"] - geo["lo"], axis=1)
    u1 = np.zeros(A.shape[0])
    u1[0::nb] = np.sqrt(box)
    r = A @ u1
    interior = [c for c in range(m.n_cells)
                if all(m.face_bc[f] == 0 for f in m.cell_face[m.cell_face_ptr[c]:m.cell_face_ptr[c + 1]])]
    assert len(interior) >= 2
    for c in interior:
        lo, hi = geo["lo"][c], geo["hi"][c]
        J = np.prod(hi - lo) / 8.0
        tris = _tris_box(m, c, lo, hi)
        ref = np.array([J * PE.polyhedron_integral_box(tris, poly) for poly in PE.basis_polys_3d(1, lo, hi)])
        assert np.abs(r[c * nb:(c + 1) * nb] - prob.c * ref).max() <= 1e-12 * np.abs(A).max() * np.abs(u1).max()


U_POLY3 = (1.0, 2.0, -1.0, 0.5, 1.0, -0.5, 0.75, 1.0, -0.25, 0.6)


def _u3(x):
    c = U_POLY3
    return (c[0] + c[1] * x[0] + c[2] * x[1] + c[3] * x[2] + c[4] * x[0] ** 2 + c[5] * x[1] ** 2
            + c[6] * x[2] ** 2 + c[7] * x[0] * x[1] + c[8] * x[0] * x[2] + c[9] * x[1] * x[2])


def test_polynomial_reproduction_3d():
    m = agglomerated_cube(4, 7, 99, p=2)
    prob = oracle.Problem(a0=1.3, b=(0.4, -0.7, 0.5), c=0.9, u_kind=oracle.U_POLY, u_poly=U_POLY3)
    pat = oracle.pattern(m)
    vals, rhs = oracle.assemble(m, prob, pat=pat)
    A = oracle.dense(m, pat, vals)
    geo = oracle.geometry(m, prob)
    t, w = np.polynomial.legendre.leggauss(4)
    pu = []
    for c in range(m.n_cells):
        lo, hi = geo["lo"][c], geo["hi"][c]
        coef = np.zeros(oracle.nb(3, 2))
        for idx in np.ndindex(4, 4, 4):
            xi = t[list(idx)]
            x = lo + 0.5 * (xi + 1) * (hi - lo)
            phi, _ = oracle.basis(3, 2, lo, hi, x)
            coef += np.prod(w[list(idx)]) * np.prod(0.5 * (hi - lo)) * _u3(x) * phi
        pu.append(coef)
    pu = np.concatenate(pu)
    res = A @ pu - rhs
    assert np.abs(res).max() <= 1e-12 * np.abs(A).max() * np.abs(pu).max()
    # f from the PDE by hand at one point
    x = np.array([0.3, 0.6, 0.2])
    c = U_POLY3
    grad = np.array([c[1] + 2 * c[4] * x[0] + c[7] * x[1] + c[8] * x[2],
                     c[2] + 2 * c[5] * x[1] + c[7] * x[0] + c[9] * x[2],
                     c[3] + 2 * c[6] * x[2] + c[8] * x[0] + c[9] * x[1]])
    lap = 2 * (c[4] + c[5] + c[6])
    u, f = oracle.exact(prob, 3, x)
    assert abs(u - _u3(x)) < 1e-15
    assert abs(f - (-1.3 * lap + np.dot(prob.b, grad) + 0.9 * u)) < 1e-13


def test_sin_data_vanishes_on_the_cube_boundary():
    prob = oracle.Problem(a0=1.0)
    for x in ((0.0, 0.3, 0.7), (1.0, 0.5, 0.5), (0.2, 0.0, 0.9), (0.4, 1.0, 0.1), (0.6, 0.8, 1.0)):
        assert oracle.exact(prob, 3, np.array(x))[0] == 0.0
    x = np.array([0.3, 0.45, 0.8])
    u, f = oracle.exact(prob, 3, x)
    assert abs(f - 3 * np.pi ** 2 * u) < 1e-13 * abs(f)
