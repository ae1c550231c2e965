"""FP64 CPU oracle for SIPG assembly on polytopic meshes -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` import this package.  It shares no code with the GPU path
(``paper_2007_04881_amd``) and does not import it.  The arithmetic lives in
``oracle.c`` (plain single-threaded C, double precision); this module compiles
it with gcc, derives the quadrature rules (``rules.py``) and marshals arrays.

Parity status: every function is pinned by the ``-m "not gpu"`` tests
(closed-form moments, Cartesian closed forms, symmetry, constants, polynomial
reproduction, convergence rates, the upwind finite-volume special case); the
right-hand side with non-polynomial data and variable coefficients is pinned only
indirectly (through polynomial reproduction and convergence rates).
"""

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

from . import rules as _rules

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

U_SIN, U_POLY = 0, 1
T_VOLUME, T_INTERIOR, T_BOUNDARY, T_RHS, T_ALL = 1, 2, 4, 8, 15
PEN_DIAMETER, PEN_COVERING = 0, 1


_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")


def _compile(target, extra, force):
    if force or not os.path.exists(target) or os.path.getmtime(target) < max(
            os.path.getmtime(_SRC), os.path.getmtime(os.path.join(_HERE, "oracle.h"))):
        tmp = target + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra",
                               "-Wno-unused-parameter", *extra, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, target)
    return target


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so (plain -O2, no fast-math, one thread:
    the canonical oracle) and liboracle_omp.so (the same source with OpenMP:
    rows assembled in parallel, for the CPU baseline on all host cores)."""
    _compile(_LIB_OMP, ["-fopenmp"], force)
    return _compile(_LIB, [], force)


class _Mesh(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_vertices", C.c_int64),
                ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("n_cells", C.c_int64), ("cell_ptr", C.c_void_p), ("cell_vtx", C.c_void_p),
                ("cell_p", C.c_void_p), ("cell_face_ptr", C.c_void_p), ("cell_face", C.c_void_p),
                ("n_faces", C.c_int64), ("face_vtx", C.c_void_p), ("face_cell", C.c_void_p),
                ("face_bc", C.c_void_p), ("face_opp", C.c_void_p)]


class _Problem(C.Structure):
    _fields_ = [("a0", C.c_double), ("a1", C.c_double), ("b", C.c_double * 3), ("c", C.c_double),
                ("c_sigma", C.c_double), ("u_kind", C.c_int32), ("u_poly", C.c_double * 10),
                ("term_mask", C.c_int32), ("sigma_override", C.c_double), ("penalty", C.c_int32)]


class _Rule(C.Structure):
    _fields_ = [("n", C.c_int32), ("pts", C.c_void_p), ("w", C.c_void_p)]


class _Rules(C.Structure):
    _fields_ = [("tri", _Rule * 3), ("seg", _Rule * 16), ("tet", _Rule)]


@dataclass
class Problem:
    """Coefficients and manufactured data of -div(a grad u) + b.grad u + c u = f."""
    a0: float = 1.0
    a1: float = 0.0
    b: tuple = (0.0, 0.0, 0.0)
    c: float = 0.0
    c_sigma: float = 10.0
    u_kind: int = U_SIN
    u_poly: tuple = field(default_factory=lambda: (0.0,) * 10)
    term_mask: int = T_ALL
    sigma_override: float = -1.0
    penalty: int = PEN_DIAMETER

    def _struct(self) -> _Problem:
        s = _Problem()
        s.a0, s.a1, s.c, s.c_sigma = self.a0, self.a1, self.c, self.c_sigma
        for i in range(3):
            s.b[i] = self.b[i] if i < len(self.b) else 0.0
        s.u_kind = self.u_kind
        up = list(self.u_poly) + [0.0] * (10 - len(self.u_poly))
        for i in range(10):
            s.u_poly[i] = up[i]
        s.term_mask = self.term_mask
        s.sigma_override = self.sigma_override
        s.penalty = self.penalty
        return s

    @staticmethod
    def from_params(d: dict) -> "Problem":
        return Problem(a0=d["a0"], a1=d["a1"], b=tuple(d["b"]), c=d["c"], c_sigma=d.get("c_sigma", 10.0),
                       u_kind=U_SIN if d.get("u", "sin") == "sin" else U_POLY,
                       u_poly=tuple(d.get("u_poly", (0.0,) * 10)),
                       penalty=PEN_COVERING if d.get("penalty", "diameter") == "covering" else PEN_DIAMETER)


_lib = None
_lib_omp = None
_keep = []


def _load(path):
    L = C.CDLL(path)
    L.orc_nb.restype = C.c_int
    L.orc_basis.restype = C.c_int
    for fn in ("orc_geometry", "orc_pattern_sizes", "orc_pattern", "orc_assemble", "orc_threads",
               "orc_assemble_st"):
        getattr(L, fn).restype = C.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        _lib = _load(build())
    return _lib


def lib_omp():
    """The OpenMP build (rows in parallel over OMP_NUM_THREADS threads)."""
    global _lib_omp
    if _lib_omp is None:
        build()
        _lib_omp = _load(_LIB_OMP)
    return _lib_omp


def threads(parallel: bool = False) -> int:
    return (lib_omp() if parallel else lib()).orc_threads()


def _ptr(a):
    return None if a is None or a.size == 0 else a.ctypes.data


def _mesh_struct(m):
    arrs = [np.ascontiguousarray(a) for a in (m.x, m.y, m.z, m.cell_ptr, m.cell_vtx, m.cell_p, m.cell_face_ptr,
                                              m.cell_face, m.face_vtx, m.face_cell, m.face_bc, m.face_opp)]
    s = _Mesh()
    s.dim = m.dim
    s.n_vertices = m.n_vertices
    s.x, s.y, s.z = _ptr(arrs[0]), _ptr(arrs[1]), _ptr(arrs[2])
    s.n_cells = m.n_cells
    s.cell_ptr, s.cell_vtx, s.cell_p = _ptr(arrs[3]), _ptr(arrs[4]), _ptr(arrs[5])
    s.cell_face_ptr, s.cell_face = _ptr(arrs[6]), _ptr(arrs[7])
    s.n_faces = m.n_faces
    s.face_vtx, s.face_cell, s.face_bc, s.face_opp = _ptr(arrs[8]), _ptr(arrs[9]), _ptr(arrs[10]), _ptr(arrs[11])
    return s, arrs


_rules_cache = None


def _rules_struct():
    global _rules_cache
    if _rules_cache is None:
        keep = []
        s = _Rules()

        def put(r, pts, w):
            pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1)
            w = np.ascontiguousarray(w, dtype=np.float64)
            keep.extend([pts, w])
            r.n, r.pts, r.w = w.shape[0], pts.ctypes.data, w.ctypes.data

        for i, deg in enumerate((4, 6, 8)):
            put(s.tri[i], *_rules.triangle_rule(deg))
        for n in range(1, 16):
            put(s.seg[n], *_rules.gauss_legendre01(n))
        put(s.tet, *_rules.tet_rule(4))
        _rules_cache = (s, keep)
    return _rules_cache[0]


def nb(dim: int, p: int) -> int:
    return lib().orc_nb(dim, p)


def basis(dim, p, lo, hi, x):
    n = nb(dim, p)
    phi = np.zeros(n)
    grad = np.zeros(n * dim)
    lo = np.ascontiguousarray(lo, dtype=np.float64)
    hi = np.ascontiguousarray(hi, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    rc = lib().orc_basis(dim, p, C.c_void_p(lo.ctypes.data), C.c_void_p(hi.ctypes.data),
                         C.c_void_p(x.ctypes.data), C.c_void_p(phi.ctypes.data), C.c_void_p(grad.ctypes.data))
    if rc < 0:
        raise ValueError(f"orc_basis failed ({rc})")
    return phi, grad.reshape(n, dim)


def exact(problem: Problem, dim: int, x):
    u, f = C.c_double(), C.c_double()
    x = np.ascontiguousarray(x, dtype=np.float64)
    ps = problem._struct()
    lib().orc_exact(C.byref(ps), dim, C.c_void_p(x.ctypes.data), C.byref(u), C.byref(f))
    return u.value, f.value


def geometry(mesh, problem: Problem = None):
    problem = problem or Problem()
    ms, keep = _mesh_struct(mesh)
    n = mesh.n_cells
    lo, hi = np.zeros((n, 3)), np.zeros((n, 3))
    meas, diam, abar = np.zeros(n), np.zeros(n), np.zeros(n)
    ps = problem._struct()
    rc = lib().orc_geometry(C.byref(ms), C.byref(ps), C.byref(_rules_struct()), *[C.c_void_p(a.ctypes.data) for a in (lo, hi, meas, diam, abar)])
    if rc:
        raise ValueError(f"orc_geometry failed ({rc})")
    return dict(lo=lo, hi=hi, meas=meas, diam=diam, abar=abar)


@dataclass
class Pattern:
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val_ptr: np.ndarray
    dof_ptr: np.ndarray

    @property
    def nnzb(self):
        return int(self.col_idx.shape[0])

    @property
    def n_vals(self):
        return int(self.val_ptr[-1])

    @property
    def n_dofs(self):
        return int(self.dof_ptr[-1])


def pattern(mesh) -> Pattern:
    ms, keep = _mesh_struct(mesh)
    nnzb, nv, nd = C.c_int64(), C.c_int64(), C.c_int64()
    lib().orc_pattern_sizes(C.byref(ms), C.byref(nnzb), C.byref(nv), C.byref(nd))
    row_ptr = np.zeros(mesh.n_cells + 1, np.int64)
    col_idx = np.zeros(nnzb.value, np.int32)
    val_ptr = np.zeros(nnzb.value + 1, np.int64)
    dof_ptr = np.zeros(mesh.n_cells + 1, np.int64)
    rc = lib().orc_pattern(C.byref(ms), *[C.c_void_p(a.ctypes.data) for a in (row_ptr, col_idx, val_ptr, dof_ptr)])
    if rc:
        raise ValueError(f"orc_pattern failed ({rc})")
    return Pattern(row_ptr, col_idx, val_ptr, dof_ptr)


def assemble(mesh, problem: Problem, rows=None, pat: Pattern = None, parallel: bool = False):
    """FP64 block-CSR values and right-hand side.  With ``rows`` only those block
    rows are computed (the other entries stay NaN).  ``parallel`` runs the
    OpenMP build (the same arithmetic per row, rows spread over threads)."""
    pat = pat or pattern(mesh)
    ms, keep = _mesh_struct(mesh)
    vals = np.full(pat.n_vals, np.nan)
    rhs = np.full(pat.n_dofs, np.nan)
    if rows is None:
        rptr, nr = None, 0
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        rptr, nr = rows.ctypes.data, rows.shape[0]
    ps = problem._struct()
    L = lib_omp() if parallel else lib()
    rc = L.orc_assemble(C.byref(ms), C.byref(ps), C.byref(_rules_struct()),
                            *[C.c_void_p(a.ctypes.data) for a in (pat.row_ptr, pat.col_idx, pat.val_ptr, pat.dof_ptr)],
                            C.c_void_p(rptr), C.c_int64(nr),
                            C.c_void_p(vals.ctypes.data), C.c_void_p(rhs.ctypes.data))
    if rc:
        raise ValueError(f"orc_assemble failed ({rc})")
    return vals, rhs


def dense(mesh, pat: Pattern, vals):
    """Dense matrix from block-CSR (small meshes only)."""
    n = pat.n_dofs
    A = np.zeros((n, n))
    dim = mesh.dim
    for r in range(mesh.n_cells):
        nr = nb(dim, int(mesh.cell_p[r]))
        r0 = pat.dof_ptr[r]
        for k in range(pat.row_ptr[r], pat.row_ptr[r + 1]):
            c = pat.col_idx[k]
            ncol = nb(dim, int(mesh.cell_p[c]))
            c0 = pat.dof_ptr[c]
            A[r0:r0 + nr, c0:c0 + ncol] = vals[pat.val_ptr[k]:pat.val_ptr[k + 1]].reshape(nr, ncol)
    return A


# ------------------------------------------------------------ space-time slabs
class _Slab(C.Structure):
    _fields_ = [("t0", C.c_double), ("t1", C.c_double), ("tp0", C.c_double), ("tau1", C.c_double),
                ("tau2", C.c_double), ("prev", C.c_void_p)]


def pattern_st(mesh) -> Pattern:
    """Block pattern of a space-time slab over a 2D mesh: the spatial blocks,
    each n_b(p) x n_b(p') with the space-time count n_b = (p+1)(p+2)(p+3)/6."""
    sp = pattern(mesh)
    nb3 = lambda p: (p + 1) * (p + 2) * (p + 3) // 6
    nbc = np.array([nb3(int(p)) for p in mesh.cell_p], dtype=np.int64)
    rows = np.repeat(np.arange(mesh.n_cells), np.diff(sp.row_ptr))
    sizes = nbc[rows] * nbc[sp.col_idx]
    val_ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    dof_ptr = np.concatenate([[0], np.cumsum(nbc)]).astype(np.int64)
    return Pattern(sp.row_ptr, sp.col_idx, val_ptr, dof_ptr)


def assemble_st(mesh, problem: Problem, t0, t1, tau=(0.0, 0.0), prev=None, tp0=None, rows=None,
                pat: Pattern = None, parallel: bool = False):
    """FP64 matrix and load of the space-time slab (t0, t1] over a 2D mesh
    (orc_assemble_st): u = u_s(x, y) (1 + tau[0] t + tau[1] t^2); prev = the
    previous slab's coefficients (its time box [tp0, t0]) or None for the exact u(., t0)."""
    pat = pat or pattern_st(mesh)
    ms, keep = _mesh_struct(mesh)
    vals = np.full(pat.n_vals, np.nan)
    rhs = np.full(pat.n_dofs, np.nan)
    sl = _Slab()
    sl.t0, sl.t1, sl.tau1, sl.tau2 = t0, t1, tau[0], tau[1]
    sl.tp0 = tp0 if tp0 is not None else t0 - (t1 - t0)
    prev_arr = None
    if prev is not None:
        prev_arr = np.ascontiguousarray(prev, dtype=np.float64)
        sl.prev = prev_arr.ctypes.data
    if rows is None:
        rptr, nr = None, 0
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        rptr, nr = rows.ctypes.data, rows.shape[0]
    ps = problem._struct()
    L = lib_omp() if parallel else lib()
    rc = L.orc_assemble_st(C.byref(ms), C.byref(ps), C.byref(_rules_struct()), C.byref(sl),
                           *[C.c_void_p(a.ctypes.data) for a in (pat.row_ptr, pat.col_idx, pat.val_ptr, pat.dof_ptr)],
                           C.c_void_p(rptr), C.c_int64(nr), C.c_void_p(vals.ctypes.data), C.c_void_p(rhs.ctypes.data))
    if rc:
        raise ValueError(f"orc_assemble_st failed ({rc})")
    return vals, rhs
