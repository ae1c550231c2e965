"""Pins of the penalty inputs (Appendix A): abar_kappa, the L-infinity norm of
the diffusion coefficient over the element taken at its volume quadrature
points, and sigma_F = C_sigma max over the face's elements of abar p^2 / h with
h the element diameter.  Everything the oracle is compared with here is
rebuilt with numpy from the mesh alone: the fan sub-triangles, the reference
triangle rule of the element's degree, a(x) = a0 + a1 sin(2 pi x) cos(2 pi y)
and the largest vertex distance.  The penalty itself is read back from
assembled matrices (the difference of two assemblies with the penalty fixed to
0 and 1 isolates the penalty's face mass term), so a wrong point set for abar,
a wrong h, a missing p^2 or a maximum over the wrong elements all fail."""

import numpy as np
import pytest

import oracle
from meshgen import voronoi_mesh
from oracle import rules

A0, A1 = 1.0, 0.5


def _a(x, y):
    return A0 + A1 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)


def _xy(m, c):
    ids = m.cell_vtx[m.cell_ptr[c]:m.cell_ptr[c + 1]]
    return np.stack([m.x[ids], m.y[ids]], 1)


def _volume_points(m, c):
    """Fan triangles (v0, v_k, v_k+1) times the reference rule of degree max(4, 2p)."""
    xy = _xy(m, c)
    bary, _ = rules.triangle_rule(max(4, 2 * int(m.cell_p[c])))
    pts = []
    for k in range(1, len(xy) - 1):
        tri = np.stack([xy[0], xy[k], xy[k + 1]])
        pts.append(bary @ tri)
    return np.concatenate(pts)


def _mesh():
    m = voronoi_mesh(80, 21, lloyd=1, p=1)
    return m.with_degrees(np.random.default_rng(3).integers(1, 5, m.n_cells))


def test_abar_is_the_max_of_a_at_the_volume_points():
    m = _mesh()
    geo = oracle.geometry(m, oracle.Problem(a0=A0, a1=A1))
    far_v = far_c = 0
    for c in range(m.n_cells):
        pts = _volume_points(m, c)
        ref = _a(pts[:, 0], pts[:, 1]).max()
        # the same maximum up to the rounding of sin/cos and of the point coordinates
        assert abs(geo["abar"][c] - ref) <= 1e-14, (c, geo["abar"][c], ref)
        xy = _xy(m, c)
        far_v += abs(_a(xy[:, 0], xy[:, 1]).max() - ref) > 1e-6
        cen = xy.mean(0)
        far_c += abs(_a(cen[0], cen[1]) - ref) > 1e-6
    # the check tells the volume points apart from the vertices and the centroid
    assert far_v > m.n_cells // 2 and far_c > m.n_cells // 2, (far_v, far_c)


def test_abar_uses_the_rule_of_the_element_degree():
    """A degree-4 element takes its points from the degree-8 rule: abar differs
    from the degree-4 rule's maximum on most elements."""
    m = voronoi_mesh(40, 22, lloyd=1, p=4)
    geo = oracle.geometry(m, oracle.Problem(a0=A0, a1=A1))
    differ = 0
    for c in range(m.n_cells):
        xy = _xy(m, c)
        bary, _ = rules.triangle_rule(4)
        low = np.concatenate([bary @ np.stack([xy[0], xy[k], xy[k + 1]]) for k in range(1, len(xy) - 1)])
        ref = _a(*_volume_points(m, c).T).max()
        assert abs(geo["abar"][c] - ref) <= 1e-14
        differ += abs(_a(*low.T).max() - ref) > 1e-9
    assert differ > m.n_cells // 2


def _diam(m, c):
    xy = _xy(m, c)
    return np.sqrt(((xy[:, None, :] - xy[None, :, :]) ** 2).sum(-1)).max()


@pytest.mark.parametrize("c_sigma", [10.0, 3.5])
def test_penalty_read_back_from_the_matrix(c_sigma):
    """sigma_F on every interior face pair and every boundary element, from
    assembled blocks, against C_sigma max(abar p^2 / h) computed here."""
    m = _mesh()
    pat = oracle.pattern(m)

    def asm(mask, override):
        pr = oracle.Problem(a0=A0, a1=A1, c_sigma=c_sigma, term_mask=mask, sigma_override=override)
        return oracle.assemble(m, pr, pat=pat)[0]

    abar = np.array([_a(*_volume_points(m, c).T).max() for c in range(m.n_cells)])
    h = np.array([_diam(m, c) for c in range(m.n_cells)])
    p = m.cell_p.astype(float)
    s = abar * p * p / h
    nb_checked = 0
    for mask in (oracle.T_INTERIOR, oracle.T_BOUNDARY):
        v, v0, v1 = asm(mask, -1.0), asm(mask, 0.0), asm(mask, 1.0)
        for r in range(m.n_cells):
            for k in range(pat.row_ptr[r], pat.row_ptr[r + 1]):
                c = pat.col_idx[k]
                if (mask == oracle.T_INTERIOR) == (c == r):
                    continue  # interior: cross blocks; boundary: diagonal blocks
                sl = slice(pat.val_ptr[k], pat.val_ptr[k + 1])
                mass = v1[sl] - v0[sl]  # the penalty's face mass term for sigma = 1
                if np.abs(mass).max() == 0.0:
                    continue  # an element without boundary faces
                j = np.argmax(np.abs(mass))
                sigma = (v[sl][j] - v0[sl][j]) / mass[j]
                ref = c_sigma * (max(s[r], s[c]) if c != r else s[r])
                assert abs(sigma - ref) <= 1e-9 * ref, (mask, r, c, sigma, ref)
                # and the whole block is that multiple of the mass term
                assert np.abs(v[sl] - v0[sl] - ref * mass).max() <= 1e-9 * ref * np.abs(mass).max()
                nb_checked += 1
    assert nb_checked > 2 * m.n_cells
