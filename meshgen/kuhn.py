"""3D polyhedral meshes of the unit cube built from Kuhn tetrahedra.

The cube is cut into n^3 sub-cubes and every sub-cube into the six Kuhn
(Freudenthal) tetrahedra that share its main diagonal.  Polyhedra are unions
of tetrahedra:

* ``agglomerated_cube``: seeded multi-source breadth-first agglomeration of
  the tetrahedra into ``n_clusters`` connected clusters (uneven sizes, as in
  agglomeration-based polytopic meshes);
* ``cube_cells``: one polyhedron per sub-cube (every cell is its own bounding
  box).

The faces of a polyhedral cell are the triangles of its tetrahedra that lie on
the cell boundary: one face per interface triangle between two cells, one per
triangle on the boundary of the unit cube (Dirichlet).  A face's ``left`` cell
is the smaller cell id, and ``face_opp`` names the vertex of the left cell's
tetrahedron opposite the triangle, which fixes the outward normal.  Each cell's
face list is ordered by neighbour (boundary first), then by face id.
"""

import numpy as np

from .mesh import Mesh

# the six orderings of the axes; tetrahedron s of a sub-cube walks from its
# lowest corner along the axes in the order _PERMS[s]
_PERMS = np.array([(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)], dtype=np.int64)


def kuhn_tets(n: int):
    """Vertex coordinates and the [6 n^3, 4] vertex ids of the Kuhn tetrahedra."""
    m = n + 1
    g = np.arange(m, dtype=np.float64) / n
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = xx.ravel().copy(), yy.ravel().copy(), zz.ravel().copy()
    stride = np.array([1, m, m * m], dtype=np.int64)
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = (i.ravel() + m * (j.ravel() + m * k.ravel())).astype(np.int64)  # cube id = i + n (j + n k)
    tets = np.empty((base.shape[0], 6, 4), dtype=np.int64)
    for s in range(6):
        v = base.copy()
        tets[:, s, 0] = v
        for a in range(3):
            v = v + stride[_PERMS[s, a]]
            tets[:, s, a + 1] = v
    return x, y, z, tets.reshape(-1, 4)


def tet_neighbours(tets: np.ndarray, n_vertices: int) -> np.ndarray:
    """[T, 4] tetrahedron across the face opposite each vertex (-1 on the boundary)."""
    T = tets.shape[0]
    faces = np.empty((T, 4, 3), dtype=np.int64)
    for q in range(4):
        faces[:, q, :] = np.delete(tets, q, axis=1)
    faces.sort(axis=2)
    N = np.uint64(n_vertices)
    f = faces.reshape(-1, 3).astype(np.uint64)
    key = (f[:, 0] * N + f[:, 1]) * N + f[:, 2]
    del f, faces
    order = np.argsort(key, kind="stable")
    ks = key[order]
    same = ks[1:] == ks[:-1]
    nbr = np.full(4 * T, -1, dtype=np.int64)
    a, b = order[:-1][same], order[1:][same]
    nbr[a] = b // 4
    nbr[b] = a // 4
    return nbr.reshape(T, 4)


def bfs_clusters(nbr: np.ndarray, n_clusters: int, seed: int) -> np.ndarray:
    """Owner cluster of every tetrahedron.

    ``n_clusters`` distinct seed tetrahedra are drawn from the seeded generator;
    a first-in first-out breadth-first search starts from all of them, queued in
    seed order, and a tetrahedron joins the first cluster that reaches it
    (neighbours visited in face order).  Processing the queue one level at a
    time in discovery order gives the same assignment."""
    T = nbr.shape[0]
    rng = np.random.default_rng(seed)
    seeds = rng.choice(T, size=n_clusters, replace=False).astype(np.int64)
    owner = np.full(T, -1, dtype=np.int64)
    owner[seeds] = np.arange(n_clusters)
    front = seeds
    while front.size:
        cand = nbr[front].ravel()
        cl = np.repeat(owner[front], 4)
        keep = cand >= 0
        cand, cl = cand[keep], cl[keep]
        keep = owner[cand] < 0
        cand, cl = cand[keep], cl[keep]
        if cand.size == 0:
            break
        _, first = np.unique(cand, return_index=True)
        first.sort()
        front = cand[first]
        owner[front] = cl[first]
    if (owner < 0).any():
        raise RuntimeError("tetrahedra unreachable from every seed")
    return owner


def polyhedral_mesh(x, y, z, tets, nbr, owner, p: int, name: str = "") -> Mesh:
    """Mesh whose cell k is the union of the tetrahedra with owner k."""
    n_cells = int(owner.max()) + 1
    T = tets.shape[0]
    order = np.argsort(owner, kind="stable")
    counts = np.bincount(owner, minlength=n_cells)
    cell_ptr = np.zeros(n_cells + 1, dtype=np.int64)
    cell_ptr[1:] = 4 * np.cumsum(counts)
    cell_vtx = tets[order].ravel().astype(np.int32)

    t = np.repeat(np.arange(T, dtype=np.int64), 4)
    q = np.tile(np.arange(4, dtype=np.int64), T)
    o = nbr.ravel()
    own = owner[t]
    oth = np.where(o >= 0, owner[np.maximum(o, 0)], -1)
    # boundary triangles, and each interface triangle once, from the side of the smaller cell id
    keep = (o < 0) | ((oth >= 0) & (own < oth))
    t, q, own, oth = t[keep], q[keep], own[keep], oth[keep]
    fv = np.empty((t.shape[0], 3), dtype=np.int64)
    rows = tets[t]
    col = np.arange(4)[None, :] != q[:, None]
    fv[:] = rows[col].reshape(-1, 3)
    fv.sort(axis=1)
    opp = rows[np.arange(t.shape[0]), q]
    N = np.int64(x.shape[0])
    key = (fv[:, 0] * N + fv[:, 1]) * N + fv[:, 2]
    forder = np.lexsort((key, oth, own))
    fv, opp, own, oth = fv[forder], opp[forder], own[forder], oth[forder]
    n_faces = fv.shape[0]
    face_cell = np.stack([own, oth], axis=1).ravel().astype(np.int32)
    face_bc = np.where(oth < 0, 1, 0).astype(np.int8)

    fid = np.arange(n_faces, dtype=np.int64)
    inner = oth >= 0
    ent_cell = np.concatenate([own, oth[inner]])
    ent_other = np.concatenate([oth, own[inner]])
    ent_face = np.concatenate([fid, fid[inner]])
    eorder = np.lexsort((ent_face, ent_other, ent_cell))
    cell_face = ent_face[eorder].astype(np.int32)
    cell_face_ptr = np.zeros(n_cells + 1, dtype=np.int64)
    cell_face_ptr[1:] = np.cumsum(np.bincount(ent_cell, minlength=n_cells))

    mesh = Mesh(dim=3, x=x, y=y, z=z, cell_ptr=cell_ptr, cell_vtx=cell_vtx,
                cell_p=np.full(n_cells, p, dtype=np.int8), cell_face_ptr=cell_face_ptr,
                cell_face=cell_face, face_vtx=fv.ravel().astype(np.int32), face_cell=face_cell,
                face_bc=face_bc, face_opp=opp.astype(np.int32), name=name)
    mesh.check()
    return mesh


def agglomerated_cube(n: int, n_clusters: int, seed: int, p: int = 2) -> Mesh:
    """n^3 sub-cubes, 6 n^3 Kuhn tetrahedra, agglomerated into ``n_clusters`` polyhedra."""
    x, y, z, tets = kuhn_tets(n)
    nbr = tet_neighbours(tets, x.shape[0])
    owner = bfs_clusters(nbr, n_clusters, seed)
    return polyhedral_mesh(x, y, z, tets, nbr, owner, p, name=f"kuhn{n}_agglo{n_clusters}_s{seed}")


def cube_cells(n: int, p: int = 2) -> Mesh:
    """n^3 cubic cells, each the union of its six Kuhn tetrahedra."""
    x, y, z, tets = kuhn_tets(n)
    nbr = tet_neighbours(tets, x.shape[0])
    owner = np.arange(tets.shape[0], dtype=np.int64) // 6
    return polyhedral_mesh(x, y, z, tets, nbr, owner, p, name=f"cubes{n}")
