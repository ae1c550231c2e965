"""Pin of the oracle's block pattern (Section 3.4, Approach 2: a block for
every element and for every pair of elements sharing at least one face) by
brute force from the cells' vertex lists alone, not from the mesh's face
arrays: two polygons are neighbours when they share an edge of their loops,
two polyhedra when they share a triangle of their tetrahedra that lies on
both cells' boundaries.  Columns ascend; values and dofs follow from the
degrees."""

import itertools

import numpy as np
import pytest

import oracle
from meshgen import voronoi_mesh
from meshgen.kuhn import agglomerated_cube


def _nb(dim, p):
    return (p + 1) * (p + 2) // 2 if dim == 2 else (p + 1) * (p + 2) * (p + 3) // 6


def _neighbours_2d(m):
    edges = []
    for c in range(m.n_cells):
        loop = m.cell_vtx[m.cell_ptr[c]:m.cell_ptr[c + 1]].tolist()
        edges.append({frozenset((loop[k], loop[(k + 1) % len(loop)])) for k in range(len(loop))})
    return [{o for o in range(m.n_cells) if o != c and edges[c] & edges[o]} for c in range(m.n_cells)]


def _neighbours_3d(m):
    surf = []
    for c in range(m.n_cells):
        tets = m.cell_vtx[m.cell_ptr[c]:m.cell_ptr[c + 1]].reshape(-1, 4)
        count = {}
        for t in tets:
            for tri in itertools.combinations(sorted(t.tolist()), 3):
                count[tri] = count.get(tri, 0) + 1
        surf.append({tri for tri, k in count.items() if k == 1})
    return [{o for o in range(m.n_cells) if o != c and surf[c] & surf[o]} for c in range(m.n_cells)]


@pytest.mark.parametrize("dim", [2, 3])
def test_pattern_brute_force(dim):
    if dim == 2:
        m = voronoi_mesh(120, 21, lloyd=2, p=1)
        m = m.with_degrees(np.random.default_rng(2).integers(1, 5, m.n_cells))
        nbrs = _neighbours_2d(m)
    else:
        m = agglomerated_cube(4, 12, 22, p=1)
        m = m.with_degrees(np.random.default_rng(3).integers(1, 3, m.n_cells))
        nbrs = _neighbours_3d(m)
    pat = oracle.pattern(m)
    row_ptr, col_idx, val_ptr, dof_ptr = [0], [], [0], [0]
    for c in range(m.n_cells):
        cols = sorted(nbrs[c] | {c})
        nr = _nb(dim, int(m.cell_p[c]))
        for o in cols:
            col_idx.append(o)
            val_ptr.append(val_ptr[-1] + nr * _nb(dim, int(m.cell_p[o])))
        row_ptr.append(len(col_idx))
        dof_ptr.append(dof_ptr[-1] + nr)
    assert np.array_equal(pat.row_ptr, row_ptr)
    assert np.array_equal(pat.col_idx, col_idx)
    assert np.array_equal(pat.val_ptr, val_ptr)
    assert np.array_equal(pat.dof_ptr, dof_ptr)
