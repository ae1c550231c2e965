"""Seeded 2D polygonal meshes of the unit square.

* ``voronoi_mesh``: Voronoi tessellation of uniform random seeds, clipped exactly
  to the unit square by mirroring the seeds near each side, with optional Lloyd
  iterations.  Cells are numbered along a Morton curve of their seeds so that
  neighbouring cells have nearby ids.
* ``cartesian_mesh``: an nx x ny grid of rectangles (every cell equals its own
  bounding box), used by closed-form tests.
"""

import numpy as np
from scipy.spatial import Voronoi, cKDTree

from .mesh import Mesh

_MERGE_TOL = 1e-12


def _morton_key(p: np.ndarray, bits: int = 20) -> np.ndarray:
    q = np.clip((p * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)
    key = np.zeros(q.shape[0], dtype=np.int64)
    for b in range(bits):
        key |= ((q[:, 0] >> b) & 1) << (2 * b)
        key |= ((q[:, 1] >> b) & 1) << (2 * b + 1)
    return key


def _clipped_regions(pts: np.ndarray):
    """Voronoi vertex array and, per seed, its cyclic vertex list clipped to [0,1]^2."""
    n = pts.shape[0]
    # mirror the seeds near each side; small meshes mirror every seed
    margin = max(0.05, 24.0 / np.sqrt(n))
    if margin > 0.5:
        margin = 1.0
    mir = [pts]
    for axis, side in ((0, 0.0), (0, 1.0), (1, 0.0), (1, 1.0)):
        sel = np.abs(pts[:, axis] - side) < margin
        m = pts[sel].copy()
        m[:, axis] = 2.0 * side - m[:, axis]
        mir.append(m)
    vor = Voronoi(np.concatenate(mir))
    verts = vor.vertices.copy()
    for axis in (0, 1):
        c = verts[:, axis]
        c[np.abs(c) < 1e-12] = 0.0
        c[np.abs(c - 1.0) < 1e-12] = 1.0
    regions = []
    for i in range(n):
        reg = vor.regions[vor.point_region[i]]
        if len(reg) == 0 or min(reg) < 0:
            raise RuntimeError("unbounded Voronoi region for an interior seed")
        regions.append(list(reg))
    return verts, regions


def _polygon_area_centroid(xy: np.ndarray):
    x, y = xy[:, 0], xy[:, 1]
    xs, ys = np.roll(x, -1), np.roll(y, -1)
    cr = x * ys - xs * y
    a = 0.5 * cr.sum()
    cx = ((x + xs) * cr).sum() / (6.0 * a)
    cy = ((y + ys) * cr).sum() / (6.0 * a)
    return a, np.array([cx, cy])


def _lloyd_step(pts: np.ndarray) -> np.ndarray:
    verts, regions = _clipped_regions(pts)
    out = np.empty_like(pts)
    for i, reg in enumerate(regions):
        _, c = _polygon_area_centroid(verts[reg])
        out[i] = c
    return out


def _build_mesh(verts: np.ndarray, regions, name: str) -> Mesh:
    # merge vertices closer than the tolerance (degenerate Voronoi vertices)
    used = sorted({v for r in regions for v in r})
    used_arr = np.array(used, dtype=np.int64)
    tree = cKDTree(verts[used_arr])
    parent = {int(v): int(v) for v in used}

    def find(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for i, j in tree.query_pairs(_MERGE_TOL):
        a, b = find(int(used_arr[i])), find(int(used_arr[j]))
        if a != b:
            parent[max(a, b)] = min(a, b)

    loops = []
    for reg in regions:
        loop = [find(v) for v in reg]
        clean = []
        for v in loop:
            if not clean or clean[-1] != v:
                clean.append(v)
        while len(clean) > 1 and clean[0] == clean[-1]:
            clean.pop()
        if len(clean) < 3:
            raise RuntimeError("degenerate Voronoi cell")
        xy = verts[clean]
        a, _ = _polygon_area_centroid(xy)
        if a < 0:
            clean = clean[::-1]
        loops.append(clean)

    # renumber vertices by first appearance along the cell order
    new_id = {}
    for loop in loops:
        for v in loop:
            if v not in new_id:
                new_id[v] = len(new_id)
    old_of_new = np.empty(len(new_id), dtype=np.int64)
    for o, nw in new_id.items():
        old_of_new[nw] = o
    xy = verts[old_of_new]

    n_cells = len(loops)
    cell_ptr = np.zeros(n_cells + 1, dtype=np.int64)
    cell_ptr[1:] = np.cumsum([len(l) for l in loops])
    cell_vtx = np.array([new_id[v] for l in loops for v in l], dtype=np.int32)

    face_id = {}
    face_vtx = []
    face_cell = []
    cell_face = np.empty(cell_vtx.shape[0], dtype=np.int32)
    for c in range(n_cells):
        s, e = cell_ptr[c], cell_ptr[c + 1]
        m = e - s
        for k in range(m):
            va, vb = int(cell_vtx[s + k]), int(cell_vtx[s + (k + 1) % m])
            key = (va, vb) if va < vb else (vb, va)
            f = face_id.get(key)
            if f is None:
                f = len(face_vtx)
                face_id[key] = f
                face_vtx.append(key)
                face_cell.append([c, -1])
            else:
                if face_cell[f][1] != -1:
                    raise RuntimeError("edge shared by more than two cells")
                face_cell[f][1] = c
            cell_face[s + k] = f
    face_cell = np.array(face_cell, dtype=np.int32)
    face_bc = np.where(face_cell[:, 1] < 0, 1, 0).astype(np.int8)
    # boundary edges must lie on the sides of the (rectangular) domain
    fv = np.array(face_vtx, dtype=np.int32)
    bnd = fv[face_bc == 1]
    lo, hi = xy.min(axis=0), xy.max(axis=0)
    for a, b in bnd:
        pa, pb = xy[a], xy[b]
        on = ((pa[0] == pb[0]) and pa[0] in (lo[0], hi[0])) or ((pa[1] == pb[1]) and pa[1] in (lo[1], hi[1]))
        if not on:
            raise RuntimeError("non-conforming boundary edge in Voronoi mesh")
    mesh = Mesh(
        dim=2,
        x=np.ascontiguousarray(xy[:, 0]),
        y=np.ascontiguousarray(xy[:, 1]),
        z=np.zeros(0),
        cell_ptr=cell_ptr,
        cell_vtx=cell_vtx,
        cell_p=np.ones(n_cells, dtype=np.int8),
        cell_face_ptr=cell_ptr.copy(),
        cell_face=cell_face,
        face_vtx=fv.reshape(-1),
        face_cell=face_cell.reshape(-1),
        face_bc=face_bc,
        name=name,
    )
    mesh.check()
    return mesh


def voronoi_mesh(n: int, seed: int, lloyd: int = 0, p=1) -> Mesh:
    """Clipped Voronoi mesh of ``n`` uniform seeds drawn with ``numpy.random.default_rng(seed)``."""
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 2))
    for _ in range(lloyd):
        pts = _lloyd_step(pts)
    pts = pts[np.argsort(_morton_key(pts), kind="stable")]
    verts, regions = _clipped_regions(pts)
    mesh = _build_mesh(verts, regions, f"voronoi(n={n},seed={seed},lloyd={lloyd})")
    total = sum(_polygon_area_centroid(np.stack([mesh.x[mesh.cell_vtx[s:e]], mesh.y[mesh.cell_vtx[s:e]]], 1))[0]
                for s, e in zip(mesh.cell_ptr[:-1], mesh.cell_ptr[1:]))
    if abs(total - 1.0) > 1e-9:
        raise RuntimeError(f"Voronoi cells do not tile the unit square (area {total})")
    return mesh.with_degrees(p)


def cartesian_mesh(nx: int, ny: int, p=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0) -> Mesh:
    """Rectangular nx x ny grid; cells counter-clockwise from their lower-left corner."""
    xs = np.linspace(x0, x1, nx + 1)
    ys = np.linspace(y0, y1, ny + 1)
    verts = np.array([[xs[i], ys[j]] for j in range(ny + 1) for i in range(nx + 1)])
    vid = lambda i, j: j * (nx + 1) + i
    regions = [[vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)]
               for j in range(ny) for i in range(nx)]
    mesh = _build_mesh(verts, regions, f"cartesian({nx}x{ny})")
    return mesh.with_degrees(p)


def split_cartesian_mesh(nx: int, ny: int, p=1, x0=0.0, x1=1.0, y0=0.0, y1=1.0) -> Mesh:
    """Rectangular nx x ny grid whose cell sides are all split at their midpoints:
    every cell is an octagon with collinear vertices, and two neighbouring cells
    share two edges (the mesh a refined neighbour leaves behind)."""
    xs = np.linspace(x0, x1, 2 * nx + 1)
    ys = np.linspace(y0, y1, 2 * ny + 1)
    verts = np.array([[xs[i], ys[j]] for j in range(2 * ny + 1) for i in range(2 * nx + 1)])
    vid = lambda i, j: j * (2 * nx + 1) + i
    ring = [(0, 0), (1, 0), (2, 0), (2, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
    regions = [[vid(2 * i + a, 2 * j + b) for a, b in ring] for j in range(ny) for i in range(nx)]
    mesh = _build_mesh(verts, regions, f"split-cartesian({nx}x{ny})")
    return mesh.with_degrees(p)
