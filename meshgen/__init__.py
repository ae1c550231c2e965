"""Seeded synthetic meshes: the only module shared by the oracle side and the GPU side.

It produces inputs (vertex coordinates, connectivity, per-cell degrees) and
nothing else: no basis, quadrature, penalty or integral of the dG method lives
here.  Every generator is deterministic in its seed.

Mesh layout (all numpy arrays, host memory):

    dim            2 or 3
    x, y, z        float64 [n_vertices] vertex coordinates (z empty in 2D)
    cell_ptr       int64  [n_cells+1]  offsets into cell_vtx
    cell_vtx       int32               2D: counter-clockwise vertex loop of the
                                       polygon, the first vertex is the fan apex;
                                       3D: four vertex ids per sub-tetrahedron
    cell_p         int8   [n_cells]    polynomial degree of each cell
    cell_face_ptr  int64  [n_cells+1]  offsets into cell_face
    cell_face      int32               faces of each cell; in 2D face k of the
                                       cell is the edge (v_k, v_{k+1}) of its loop
    face_vtx       int32  [n_faces*dim] 2D: edge end points, lower id first;
                                       3D: triangle vertex ids
    face_cell      int32  [n_faces*2]  (left, right) cells, right = -1 on the
                                       boundary
    face_bc        int8   [n_faces]    0 interior, 1 Dirichlet, 2 Neumann
    face_opp       int32  [n_faces]    3D only: vertex of the left cell's
                                       sub-tetrahedron opposite the face
"""

from .mesh import Mesh
from .voronoi import voronoi_mesh, cartesian_mesh, split_cartesian_mesh
from .kuhn import agglomerated_cube, cube_cells
from .configs import config_mesh, problem_params, CONFIG_SEED_BASE

__all__ = ["Mesh", "voronoi_mesh", "cartesian_mesh", "split_cartesian_mesh", "agglomerated_cube", "cube_cells", "config_mesh", "problem_params", "CONFIG_SEED_BASE"]
