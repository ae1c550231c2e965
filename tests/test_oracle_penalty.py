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


# ------------------------------------------------------------ covering penalty
def _sigma_read_back(m, c_sigma, a0, a1, penalty, check):
    """sigma_F per (row, block) read back from assembled interior / boundary terms;
    check(r, c, sigma) is called for every cross block and every boundary diagonal block."""
    pat = oracle.pattern(m)

    def asm(mask, override):
        pr = oracle.Problem(a0=a0, a1=a1, c_sigma=c_sigma, term_mask=mask, sigma_override=override,
                            penalty=penalty)
        return oracle.assemble(m, pr, pat=pat)[0]

    faces = lambda r: set(m.cell_face[m.cell_face_ptr[r]:m.cell_face_ptr[r + 1]].tolist())
    n = 0
    for mask in (oracle.T_INTERIOR, oracle.T_BOUNDARY):
        v, v0, v1 = asm(mask, -1.0), asm(mask, 0.0), asm(mask, 1.0)
        for r in range(m.n_cells):
            for k in range(pat.row_ptr[r], pat.row_ptr[r + 1]):
                c = pat.col_idx[k]
                if (mask == oracle.T_INTERIOR) == (c == r):
                    continue
                # blocks that one face alone contributes to (the penalty is per face)
                if c == r:
                    if sum(m.face_cell[2 * f + 1] < 0 for f in faces(r)) != 1:
                        continue
                elif len(faces(r) & faces(c)) != 1:
                    continue
                sl = slice(pat.val_ptr[k], pat.val_ptr[k + 1])
                mass = v1[sl] - v0[sl]
                if np.abs(mass).max() == 0.0:
                    continue
                j = np.argmax(np.abs(mass))
                sigma = (v[sl][j] - v0[sl][j]) / mass[j]
                # one sigma for the whole block (one face per block here)
                assert np.abs(v[sl] - v0[sl] - sigma * mass).max() <= 1e-9 * abs(sigma) * np.abs(mass).max()
                check(r, c, sigma)
                n += 1
    return n


def test_covering_penalty_on_a_rectangular_grid():
    """Cells hx x hy split into two fan triangles of area hx hy / 2, one of them
    having each side as an edge: min(1 / |K^F|, p^2 / |kappa|) = min(2, p^2) / (hx hy),
    so sigma_F = C_sigma a max_kappa p^2 min(2, p^2) |F| / (hx hy)."""
    from meshgen import cartesian_mesh
    nx, ny, x0, x1, y0, y1 = 3, 2, 0.1, 1.3, -0.2, 0.9
    m = cartesian_mesh(nx, ny, p=1, x0=x0, x1=x1, y0=y0, y1=y1)
    m = m.with_degrees(np.array([1, 2, 3, 3, 1, 2], np.int8))
    hx, hy = (x1 - x0) / nx, (y1 - y0) / ny
    a0 = 1.3
    ix = lambda c: c % nx
    factor = lambda p: p * p * min(2, p * p) / (hx * hy)

    def check(r, c, sigma):
        pr, pc = int(m.cell_p[r]), int(m.cell_p[c])
        # a vertical face between columns, else a horizontal one (the middle
        # column's single boundary face is horizontal too: c == r there)
        flen = hy if ix(r) != ix(c) else hx
        ref = 10.0 * a0 * max(factor(pr), factor(pc)) * flen
        assert abs(sigma - ref) <= 1e-12 * ref, (r, c, sigma, ref)

    n = _sigma_read_back(m, 10.0, a0, 0.0, oracle.PEN_COVERING, check)
    # seven interior faces seen from both sides, and the middle column's two
    # elements with one boundary face each (the corners have two)
    assert n == 2 * 7 + 2


def test_covering_penalty_on_voronoi_cells():
    """Mixed degrees, variable a: sigma_F from the fan triangles computed here."""
    m = _mesh()
    abar = np.array([_a(*_volume_points(m, c).T).max() for c in range(m.n_cells)])
    area = np.array([0.5 * np.sum(_xy(m, c)[:, 0] * np.roll(_xy(m, c)[:, 1], -1)
                                  - np.roll(_xy(m, c)[:, 0], -1) * _xy(m, c)[:, 1]) for c in range(m.n_cells)])

    def side(c, f):
        s, e = m.cell_ptr[c], m.cell_ptr[c + 1]
        n = e - s
        k = int(np.where(m.cell_face[s:e] == f)[0][0])
        t = 1 if k == 0 else (n - 2 if k == n - 1 else k)
        xy = _xy(m, c)
        v0, v1, v2 = xy[0], xy[t], xy[t + 1]
        kf = 0.5 * abs((v1[0] - v0[0]) * (v2[1] - v0[1]) - (v2[0] - v0[0]) * (v1[1] - v0[1]))
        a, b = m.face_vtx[2 * f], m.face_vtx[2 * f + 1]
        flen = np.hypot(m.x[a] - m.x[b], m.y[a] - m.y[b])
        p = int(m.cell_p[c])
        return abar[c] * p * p * flen * min(1.0 / kf, p * p / area[c])

    # faces between r and c (Voronoi neighbours share one edge)
    def shared(r, c):
        fr = set(m.cell_face[m.cell_face_ptr[r]:m.cell_face_ptr[r + 1]].tolist())
        fc = set(m.cell_face[m.cell_face_ptr[c]:m.cell_face_ptr[c + 1]].tolist())
        return sorted(fr & fc)

    def check(r, c, sigma):
        if c == r:
            bf = [f for f in m.cell_face[m.cell_face_ptr[r]:m.cell_face_ptr[r + 1]] if m.face_cell[2 * f + 1] < 0]
            ref = 3.5 * side(r, bf[0])
        else:
            fs = shared(r, c)
            assert len(fs) == 1
            ref = 3.5 * max(side(r, fs[0]), side(c, fs[0]))
        assert abs(sigma - ref) <= 1e-12 * ref, (r, c, sigma, ref)

    n = _sigma_read_back(m, 3.5, A0, A1, oracle.PEN_COVERING, check)
    assert n > 2 * m.n_cells
