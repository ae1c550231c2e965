"""dgpoly: SIPG matrix assembly on polytopic meshes for AMD MI355X.

Thin ctypes binding of ``libdgpoly.so`` (C ABI in ``include/dgpoly.h``).  It only
marshals arguments: every step of the assembly runs in the library's HIP
kernels.  PyTorch provides device memory (output tensors) and the HIP stream.
If the library is not built the import fails loudly; there is no fallback.
"""

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdgpoly.so")

F64, F32 = 0, 1
U_SIN, U_POLY = 0, 1

_STATUS = {0: "DGP_OK", -1: "DGP_EINVAL", -2: "DGP_EMESH", -3: "DGP_EUNSUPPORTED", -4: "DGP_ENOMEM",
           -5: "DGP_EDEVICE", -6: "DGP_ESTATE"}


class DgpError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class MeshDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("n_vertices", C.c_int64),
                ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("n_cells", C.c_int64), ("cell_ptr", C.c_void_p), ("cell_vtx", C.c_void_p),
                ("cell_p", C.c_void_p), ("cell_face_ptr", C.c_void_p), ("cell_face", C.c_void_p),
                ("n_faces", C.c_int64), ("face_vtx", C.c_void_p), ("face_cell", C.c_void_p),
                ("face_bc", C.c_void_p), ("face_opp", C.c_void_p)]


class ProblemDesc(C.Structure):
    _fields_ = [("a0", C.c_double), ("a1", C.c_double), ("b", C.c_double * 3), ("c", C.c_double),
                ("c_sigma", C.c_double), ("u_kind", C.c_int32), ("u_poly", C.c_double * 10)]


class PatternInfo(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("nnzb", C.c_int64), ("n_vals", C.c_int64), ("n_dofs", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val_ptr", C.c_void_p),
                ("dof_ptr", C.c_void_p)]


EXPORTS = ["dgp_create", "dgp_destroy", "dgp_set_stream", "dgp_last_error", "dgp_mesh_upload", "dgp_pattern",
           "dgp_pattern_copy", "dgp_assemble", "dgp_run", "dgp_graph_capture", "dgp_graph_launch",
           "dgp_set_timing", "dgp_kernel_ms"]

_lib = None


def lib():
    """Load libdgpoly.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2007_04881_amd.build` "
                              "(there is no CPU fallback)")
        L = C.CDLL(LIB_PATH)
        for name in EXPORTS:
            getattr(L, name).restype = C.c_int32
        L.dgp_last_error.restype = C.c_char_p
        L.dgp_create.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.c_void_p]
        for name in ("dgp_destroy", "dgp_graph_launch"):
            getattr(L, name).argtypes = [C.c_void_p]
        L.dgp_last_error.argtypes = [C.c_void_p]
        L.dgp_set_stream.argtypes = [C.c_void_p, C.c_void_p]
        L.dgp_mesh_upload.argtypes = [C.c_void_p, C.POINTER(MeshDesc)]
        L.dgp_pattern.argtypes = [C.c_void_p, C.POINTER(PatternInfo)]
        L.dgp_pattern_copy.argtypes = [C.c_void_p] + [C.c_void_p] * 4
        for name in ("dgp_assemble", "dgp_run"):
            getattr(L, name).argtypes = [C.c_void_p, C.POINTER(ProblemDesc), C.c_int, C.c_void_p, C.c_void_p]
        L.dgp_graph_capture.argtypes = [C.c_void_p, C.c_int, C.POINTER(ProblemDesc), C.c_int, C.c_void_p,
                                        C.c_void_p]
        L.dgp_set_timing.argtypes = [C.c_void_p, C.c_int]
        L.dgp_kernel_ms.argtypes = [C.c_void_p, C.c_char_p, C.POINTER(C.c_float)]
        _lib = L
    return _lib


def problem_desc(params: dict) -> ProblemDesc:
    """ProblemDesc from a plain dict (a0, a1, b, c, c_sigma, u, u_poly)."""
    p = ProblemDesc()
    p.a0, p.a1, p.c = params["a0"], params["a1"], params["c"]
    p.c_sigma = params.get("c_sigma", 10.0)
    b = list(params.get("b", (0.0, 0.0, 0.0))) + [0.0] * 3
    for i in range(3):
        p.b[i] = b[i]
    p.u_kind = U_SIN if params.get("u", "sin") == "sin" else U_POLY
    up = list(params.get("u_poly", ())) + [0.0] * 10
    for i in range(10):
        p.u_poly[i] = up[i]
    return p


def _ptr(a):
    return None if a is None or a.size == 0 else a.ctypes.data


def _torch_stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


class Context:
    """One device, one HIP stream; owns the device mesh, geometry and pattern."""

    def __init__(self, device: int = 0, stream=None):
        import torch
        self.device = device
        torch.cuda.set_device(device)
        self._h = C.c_void_p()
        self._check(lib().dgp_create(C.byref(self._h), device, C.c_void_p(_torch_stream(stream))), "dgp_create")
        self.info = None
        self._keep = None

    def _check(self, st, what):
        if st != 0:
            msg = lib().dgp_last_error(self._h).decode() if self._h else ""
            raise DgpError(st, f"{what}: {msg}")

    def close(self):
        if self._h:
            lib().dgp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self._check(lib().dgp_set_stream(self._h, C.c_void_p(_torch_stream(stream))), "dgp_set_stream")

    def upload(self, mesh):
        arrs = {k: np.ascontiguousarray(v) for k, v in mesh.arrays().items()}
        d = MeshDesc()
        d.dim = mesh.dim
        d.n_vertices = mesh.n_vertices
        d.x, d.y, d.z = _ptr(arrs["x"]), _ptr(arrs["y"]), _ptr(arrs["z"])
        d.n_cells = mesh.n_cells
        d.cell_ptr, d.cell_vtx, d.cell_p = _ptr(arrs["cell_ptr"]), _ptr(arrs["cell_vtx"]), _ptr(arrs["cell_p"])
        d.cell_face_ptr, d.cell_face = _ptr(arrs["cell_face_ptr"]), _ptr(arrs["cell_face"])
        d.n_faces = mesh.n_faces
        d.face_vtx, d.face_cell, d.face_bc = _ptr(arrs["face_vtx"]), _ptr(arrs["face_cell"]), _ptr(arrs["face_bc"])
        d.face_opp = _ptr(arrs.get("face_opp"))
        self._check(lib().dgp_mesh_upload(self._h, C.byref(d)), "dgp_mesh_upload")
        self.info = None

    def pattern(self) -> PatternInfo:
        info = PatternInfo()
        self._check(lib().dgp_pattern(self._h, C.byref(info)), "dgp_pattern")
        self.info = info
        return info

    def pattern_tensors(self):
        """Copies of row_ptr, col_idx, val_ptr, dof_ptr as torch tensors on the device."""
        import torch
        i = self.info or self.pattern()
        dev = torch.device("cuda", self.device)
        rp = torch.empty(i.n_rows + 1, dtype=torch.int64, device=dev)
        ci = torch.empty(i.nnzb, dtype=torch.int32, device=dev)
        vp = torch.empty(i.nnzb + 1, dtype=torch.int64, device=dev)
        dp = torch.empty(i.n_rows + 1, dtype=torch.int64, device=dev)
        self._check(lib().dgp_pattern_copy(self._h, rp.data_ptr(), ci.data_ptr(), vp.data_ptr(), dp.data_ptr()),
                    "dgp_pattern_copy")
        return rp, ci, vp, dp

    def outputs(self, precision=F32):
        import torch
        i = self.info or self.pattern()
        dt = torch.float32 if precision == F32 else torch.float64
        dev = torch.device("cuda", self.device)
        return torch.empty(i.n_vals, dtype=dt, device=dev), torch.empty(i.n_dofs, dtype=dt, device=dev)

    @staticmethod
    def _tensors_ok(vals, rhs, precision):
        import torch
        dt = torch.float32 if precision == F32 else torch.float64
        for t in (vals, rhs):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"outputs must be contiguous {dt} device tensors")

    def assemble(self, problem: dict, precision, vals, rhs):
        self._tensors_ok(vals, rhs, precision)
        pd = problem_desc(problem)
        self._check(lib().dgp_assemble(self._h, C.byref(pd), precision, vals.data_ptr(), rhs.data_ptr()),
                    "dgp_assemble")

    def run(self, problem: dict, precision, vals, rhs):
        self._tensors_ok(vals, rhs, precision)
        pd = problem_desc(problem)
        self._check(lib().dgp_run(self._h, C.byref(pd), precision, vals.data_ptr(), rhs.data_ptr()), "dgp_run")

    def graph_capture(self, what, problem: dict, precision, vals, rhs):
        self._tensors_ok(vals, rhs, precision)
        pd = problem_desc(problem)
        self._check(lib().dgp_graph_capture(self._h, what, C.byref(pd), precision, vals.data_ptr(), rhs.data_ptr()),
                    "dgp_graph_capture")

    def graph_launch(self):
        self._check(lib().dgp_graph_launch(self._h), "dgp_graph_launch")

    def set_timing(self, on: bool):
        self._check(lib().dgp_set_timing(self._h, 1 if on else 0), "dgp_set_timing")

    def kernel_ms(self, name: str) -> float:
        ms = C.c_float()
        self._check(lib().dgp_kernel_ms(self._h, name.encode(), C.byref(ms)), "dgp_kernel_ms")
        return ms.value
