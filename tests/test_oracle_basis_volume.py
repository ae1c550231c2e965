"""Pins for the oracle's basis (Section 3.1: orthonormal bounding-box Legendre
basis of total degree p) and its element (volume) quadrature on polygons.

* Basis values against numpy's Legendre evaluation, orthonormality on the box
  with a tensor Gauss rule, Legendre trace values P_n(+-1), P_n'(+-1), and the
  hierarchy of the ordering.
* Mass, stiffness and advection element blocks on Voronoi polygons against
  exact integrals from the divergence theorem (tests/polyexact.py).
"""

import numpy as np
import pytest
from numpy.polynomial import legendre as L

import oracle
from meshgen import voronoi_mesh
from tests import polyexact as PE


def _exps(dim, p):
    return PE.basis_exponents(dim, p)


@pytest.mark.parametrize("dim,p", [(2, 0), (2, 1), (2, 2), (2, 3), (2, 4), (3, 1), (3, 2), (3, 3)])
def test_basis_values_against_numpy(dim, p):
    rng = np.random.default_rng(7)
    lo = rng.random(dim) - 1.0
    hi = lo + 0.2 + rng.random(dim)
    box = np.prod(hi - lo)
    for _ in range(5):
        x = lo + (hi - lo) * rng.random(dim)
        phi, grad = oracle.basis(dim, p, lo, hi, x)
        xi = (2 * x - lo - hi) / (hi - lo)
        for i, e in enumerate(_exps(dim, p)):
            s = np.sqrt(np.prod([2 * k + 1 for k in e]) / box)
            vals = [L.legval(xi[d], [0] * e[d] + [1]) for d in range(dim)]
            ders = [L.legval(xi[d], L.legder([0] * e[d] + [1])) * 2 / (hi[d] - lo[d]) if e[d] > 0 else 0.0
                    for d in range(dim)]
            assert abs(phi[i] - s * np.prod(vals)) < 1e-12 * max(1.0, abs(phi[i]))
            for d in range(dim):
                g = s * ders[d] * np.prod([vals[k] for k in range(dim) if k != d])
                assert abs(grad[i, d] - g) < 1e-11 * max(1.0, abs(g))


@pytest.mark.parametrize("dim,p", [(2, 4), (3, 3)])
def test_basis_orthonormal_on_box(dim, p):
    lo = np.array([0.3, -0.2, 1.0])[:dim]
    hi = np.array([0.7, 0.9, 1.25])[:dim]
    t, w = np.polynomial.legendre.leggauss(p + 2)
    nb = oracle.nb(dim, p)
    G = np.zeros((nb, nb))
    grids = np.meshgrid(*[t] * dim, indexing="ij")
    wgrid = np.prod(np.meshgrid(*[w] * dim, indexing="ij"), axis=0)
    for idx in np.ndindex(*[len(t)] * dim):
        xi = np.array([g[idx] for g in grids])
        x = lo + 0.5 * (xi + 1) * (hi - lo)
        phi, _ = oracle.basis(dim, p, lo, hi, x)
        G += wgrid[idx] * np.prod(0.5 * (hi - lo)) * np.outer(phi, phi)
    assert np.abs(G - np.eye(nb)).max() < 1e-13


def test_basis_traces_and_hierarchy():
    lo, hi = np.array([-1.0, -1.0]), np.array([1.0, 1.0])
    for p in range(5):
        for corner in ([1.0, 1.0], [-1.0, 1.0], [-1.0, -1.0]):
            phi, grad = oracle.basis(2, p, lo, hi, np.array(corner))
            for i, (a, b) in enumerate(_exps(2, p)):
                s = np.sqrt((2 * a + 1) * (2 * b + 1) / 4.0)
                ta, tb = corner[0] ** a, corner[1] ** b
                assert abs(phi[i] - s * ta * tb) < 1e-14
                dta = corner[0] ** (a + 1) * a * (a + 1) / 2.0
                assert abs(grad[i, 0] - s * dta * tb) < 1e-13
    # hierarchical: the first nb(p') functions of degree p are the degree-p' basis
    x = np.array([0.31, -0.44])
    phi4, g4 = oracle.basis(2, 4, lo, hi, x)
    for q in range(4):
        phiq, gq = oracle.basis(2, q, lo, hi, x)
        assert np.array_equal(phiq, phi4[:len(phiq)]) and np.array_equal(gq, g4[:len(phiq)])


def _volume_points(m, c):
    """Fan sub-triangles from the first vertex times the degree-4 rule (p <= 2)."""
    xy = _cell_xy(m, c)
    bary, _ = oracle.rules.triangle_rule(4)
    return np.concatenate([bary @ np.stack([xy[0], xy[k], xy[k + 1]]) for k in range(1, len(xy) - 1)])


def _cell_xy(m, c):
    ids = m.cell_vtx[m.cell_ptr[c]:m.cell_ptr[c + 1]]
    return np.stack([m.x[ids], m.y[ids]], 1)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_element_blocks_exact_on_polygons(p):
    """Element term of (dg-bilinear) on Voronoi polygons vs the divergence theorem."""
    m = voronoi_mesh(24, 99, lloyd=2, p=p)
    pat = oracle.pattern(m)
    b = (0.7, -1.3, 0.0)
    prob_m = oracle.Problem(a0=0.0, c=1.0, term_mask=oracle.T_VOLUME)
    prob_k = oracle.Problem(a0=1.0, c=0.0, term_mask=oracle.T_VOLUME)
    prob_b = oracle.Problem(a0=0.0, b=b, c=0.0, term_mask=oracle.T_VOLUME)
    vm, _ = oracle.assemble(m, prob_m, pat=pat)
    vk, _ = oracle.assemble(m, prob_k, pat=pat)
    vb, _ = oracle.assemble(m, prob_b, pat=pat)
    geo = oracle.geometry(m)
    nb = oracle.nb(2, p)
    for c in range(m.n_cells):
        lo, hi = geo["lo"][c, :2], geo["hi"][c, :2]
        xy, J = PE.to_box(_cell_xy(m, c), lo, hi)
        cx, cy = 2 / (hi[0] - lo[0]), 2 / (hi[1] - lo[1])  # d/dx = cx d/dxi
        polys = PE.basis_polys_2d(p, lo, hi)
        I = lambda poly: J * PE.polygon_integral(xy, poly)
        M = np.array([[I(PE.mul(pi, pj)) for pj in polys] for pi in polys])
        K = np.array([[cx * cx * I(PE.mul(PE.dx(pi), PE.dx(pj))) + cy * cy * I(PE.mul(PE.dy(pi), PE.dy(pj)))
                       for pj in polys] for pi in polys])
        Bv = np.array([[b[0] * cx * I(PE.mul(PE.dx(pj), pi)) + b[1] * cy * I(PE.mul(PE.dy(pj), pi))
                        for pj in polys] for pi in polys])
        k = [kk for kk in range(pat.row_ptr[c], pat.row_ptr[c + 1]) if pat.col_idx[kk] == c][0]
        sl = slice(pat.val_ptr[k], pat.val_ptr[k + 1])
        for got, ref in ((vm[sl], M), (vk[sl], K), (vb[sl], Bv)):
            ref = ref.reshape(-1)
            assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_geometry_against_closed_forms():
    m = voronoi_mesh(40, 5, lloyd=1, p=1)
    geo = oracle.geometry(m, oracle.Problem(a0=2.0, a1=0.5))
    for c in range(m.n_cells):
        xy = _cell_xy(m, c)
        assert abs(geo["meas"][c] - PE.polygon_monomial(xy, 0, 0)) < 1e-15
        d = np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1)).max()
        assert geo["diam"][c] == d
        assert np.array_equal(geo["lo"][c, :2], xy.min(0)) and np.array_equal(geo["hi"][c, :2], xy.max(0))
        # abar: a = 2 + 0.5 sin(2 pi x) cos(2 pi y) at the cell's volume points, maximised
        pts = _volume_points(m, c)
        ref = 2.0 + 0.5 * (np.sin(2 * np.pi * pts[:, 0]) * np.cos(2 * np.pi * pts[:, 1])).max()
        assert abs(geo["abar"][c] - ref) <= 1e-14
