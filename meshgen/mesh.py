"""Container for a polytopic mesh in the flat array layout described in the package docstring."""

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Mesh:
    dim: int
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    cell_ptr: np.ndarray
    cell_vtx: np.ndarray
    cell_p: np.ndarray
    cell_face_ptr: np.ndarray
    cell_face: np.ndarray
    face_vtx: np.ndarray
    face_cell: np.ndarray
    face_bc: np.ndarray
    face_opp: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))
    name: str = ""

    @property
    def n_vertices(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.cell_ptr.shape[0] - 1)

    @property
    def n_faces(self) -> int:
        return int(self.face_bc.shape[0])

    def with_degrees(self, p) -> "Mesh":
        """Copy of the mesh with every cell degree replaced by ``p`` (scalar or array)."""
        q = np.broadcast_to(np.asarray(p, dtype=np.int8), (self.n_cells,)).copy()
        d = dict(self.__dict__)
        d["cell_p"] = q
        return Mesh(**d)

    def check(self) -> None:
        """Structural checks on the arrays (dtypes, lengths, index ranges)."""
        assert self.dim in (2, 3)
        assert self.x.dtype == np.float64 and self.y.dtype == np.float64
        assert self.cell_ptr.dtype == np.int64 and self.cell_face_ptr.dtype == np.int64
        for a in (self.cell_vtx, self.cell_face, self.face_vtx, self.face_cell):
            assert a.dtype == np.int32
        assert self.cell_p.dtype == np.int8 and self.face_bc.dtype == np.int8
        assert self.cell_ptr[0] == 0 and self.cell_ptr[-1] == self.cell_vtx.shape[0]
        assert self.cell_face_ptr[0] == 0 and self.cell_face_ptr[-1] == self.cell_face.shape[0]
        assert self.face_vtx.shape[0] == self.dim * self.n_faces
        assert self.face_cell.shape[0] == 2 * self.n_faces
        assert self.cell_p.shape[0] == self.n_cells
        if self.cell_vtx.size:
            assert self.cell_vtx.min() >= 0 and self.cell_vtx.max() < self.n_vertices
        assert self.face_cell[0::2].min() >= 0
        assert self.face_cell[1::2].min() >= -1 and self.face_cell.max() < self.n_cells
        if self.dim == 3:
            assert self.face_opp.shape[0] == self.n_faces

    def arrays(self) -> dict:
        return {k: v for k, v in self.__dict__.items() if isinstance(v, np.ndarray)}
