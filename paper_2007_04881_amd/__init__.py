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
RULE_PLAIN, RULE_REDUCED = 0, 1
INIT_NETWORK, INIT_TEMPLATE = 0, 1
PEN_DIAMETER, PEN_COVERING = 0, 1
MLP_PARAMS = 43952

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
                ("c_sigma", C.c_double), ("u_kind", C.c_int32), ("u_poly", C.c_double * 10),
                ("penalty", C.c_int32)]


class PatternInfo(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("nnzb", C.c_int64), ("n_vals", C.c_int64), ("n_dofs", C.c_int64),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p), ("val_ptr", C.c_void_p),
                ("dof_ptr", C.c_void_p)]


class QruleStats(C.Structure):
    _fields_ = [("n_cells", C.c_int64), ("n_eligible", C.c_int64), ("n_accepted", C.c_int64),
                ("iters_hist", C.c_int64 * 16), ("max_residual_accepted", C.c_double),
                ("ms_features", C.c_float), ("ms_network", C.c_float), ("ms_refine", C.c_float),
                ("n_start_network", C.c_int64), ("n_retried", C.c_int64), ("n_retry_accepted", C.c_int64)]


class SlabDesc(C.Structure):
    _fields_ = [("t0", C.c_double), ("t1", C.c_double), ("tp0", C.c_double), ("tau1", C.c_double),
                ("tau2", C.c_double), ("prev", C.c_void_p)]


class TrainCfg(C.Structure):
    _fields_ = [("n_polygons", C.c_int64), ("data_seed", C.c_uint64), ("init_seed", C.c_uint64),
                ("epochs", C.c_int32), ("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float),
                ("beta2", C.c_float), ("eps", C.c_float)]


class TrainStats(C.Structure):
    _fields_ = [("loss_first", C.c_float), ("loss_last", C.c_float), ("ms", C.c_double), ("steps", C.c_int64)]


EXPORTS = ["dgp_create", "dgp_destroy", "dgp_set_stream", "dgp_last_error", "dgp_mesh_check", "dgp_mesh_upload", "dgp_pattern",
           "dgp_pattern_copy", "dgp_assemble", "dgp_run", "dgp_run_static", "dgp_graph_capture", "dgp_graph_launch",
           "dgp_set_timing", "dgp_kernel_ms", "dgp_time_kernels", "dgp_autotune", "dgp_set_launch", "dgp_mlp_load", "dgp_qrule_build", "dgp_qrule_get",
           "dgp_qrule_cell_data", "dgp_train_polygons", "dgp_mlp_forward", "dgp_mlp_loss_grad", "dgp_adam_step",
           "dgp_mlp_train", "dgp_assemble_coo", "dgp_assemble_st"]

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
        L.dgp_mesh_check.argtypes = [C.POINTER(MeshDesc), C.c_char_p, C.c_size_t]
        L.dgp_mesh_upload.argtypes = [C.c_void_p, C.POINTER(MeshDesc)]
        L.dgp_pattern.argtypes = [C.c_void_p, C.POINTER(PatternInfo)]
        L.dgp_pattern_copy.argtypes = [C.c_void_p] + [C.c_void_p] * 4
        for name in ("dgp_assemble", "dgp_run", "dgp_run_static"):
            getattr(L, name).argtypes = [C.c_void_p, C.POINTER(ProblemDesc), C.c_int, C.c_int, C.c_void_p,
                                         C.c_void_p]
        L.dgp_graph_capture.argtypes = [C.c_void_p, C.c_int, C.POINTER(ProblemDesc), C.c_int, C.c_int,
                                        C.c_void_p, C.c_void_p]
        L.dgp_mlp_load.argtypes = [C.c_void_p, C.c_void_p, C.c_int64]
        L.dgp_qrule_build.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.POINTER(QruleStats)]
        L.dgp_qrule_get.argtypes = [C.c_void_p] + [C.c_void_p] * 5
        L.dgp_qrule_cell_data.argtypes = [C.c_void_p] + [C.c_void_p] * 3
        L.dgp_train_polygons.argtypes = [C.c_void_p, C.c_uint64, C.c_int64, C.c_int64] + [C.c_void_p] * 4
        L.dgp_mlp_forward.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p]
        L.dgp_mlp_loss_grad.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                        C.c_void_p, C.c_void_p]
        L.dgp_adam_step.argtypes = [C.c_void_p] + [C.c_void_p] * 4 + [C.c_int64, C.c_int32] + [C.c_float] * 4
        L.dgp_mlp_train.argtypes = [C.c_void_p, C.POINTER(TrainCfg), C.c_void_p, C.c_void_p,
                                    C.POINTER(TrainStats)]
        L.dgp_set_timing.argtypes = [C.c_void_p, C.c_int]
        L.dgp_kernel_ms.argtypes = [C.c_void_p, C.c_char_p, C.POINTER(C.c_float)]
        L.dgp_time_kernels.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_float), C.POINTER(C.c_float)]
        L.dgp_autotune.argtypes = [C.c_void_p, C.c_int, C.c_void_p]
        L.dgp_set_launch.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_int]
        L.dgp_assemble_coo.argtypes = [C.c_void_p, C.POINTER(ProblemDesc), C.c_int] + [C.c_void_p] * 6
        L.dgp_assemble_st.argtypes = [C.c_void_p, C.POINTER(ProblemDesc), C.c_int, C.POINTER(SlabDesc),
                                      C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def problem_desc(params: dict) -> ProblemDesc:
    """ProblemDesc from a plain dict (a0, a1, b, c, c_sigma, u, u_poly, penalty)."""
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
    p.penalty = PEN_COVERING if params.get("penalty", "diameter") == "covering" else PEN_DIAMETER
    return p


def _ptr(a):
    return None if a is None or a.size == 0 else a.ctypes.data


def _torch_stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def mesh_desc(mesh):
    """dgp_mesh_desc of a mesh (host arrays), and the arrays it points into (keep them alive)."""
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
    return d, arrs


def mesh_check(mesh):
    """The library's host checks of a mesh (dgp_mesh_check, no device): (status, message)."""
    d, arrs = mesh_desc(mesh)
    buf = C.create_string_buffer(512)
    st = lib().dgp_mesh_check(C.byref(d), buf, len(buf))
    return st, buf.value.decode()


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
        self._p = -1

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
        d, arrs = mesh_desc(mesh)
        self._check(lib().dgp_mesh_upload(self._h, C.byref(d)), "dgp_mesh_upload")
        self.info = None
        ps = np.unique(np.asarray(mesh.cell_p))
        self._p = int(ps[0]) if ps.size == 1 else -1

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

    def _tensors_ok(self, vals, rhs, precision):
        """Output tensors of the right type, device and size.  The library keeps
        their addresses for graph replays and re-timed launches, so the context
        holds a reference to the last pair until the next call replaces it."""
        import torch
        dt = torch.float32 if precision == F32 else torch.float64
        for t in (vals, rhs):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"outputs must be contiguous {dt} device tensors")
            if t.device.index != self.device:
                raise ValueError(f"outputs on {t.device}, context on cuda:{self.device}")
        i = self.info or self.pattern()
        if vals.numel() < i.n_vals or rhs.numel() < i.n_dofs:
            raise ValueError(f"outputs too small: vals {vals.numel()} < {i.n_vals} or rhs {rhs.numel()} < {i.n_dofs}")
        self._keep = (vals, rhs)

    def assemble(self, problem: dict, precision, vals, rhs, rule_mode=RULE_PLAIN):
        self._tensors_ok(vals, rhs, precision)
        pd = problem_desc(problem)
        self._check(lib().dgp_assemble(self._h, C.byref(pd), precision, rule_mode, vals.data_ptr(), rhs.data_ptr()),
                    "dgp_assemble")

    def run(self, problem: dict, precision, vals, rhs, rule_mode=RULE_PLAIN):
        self._tensors_ok(vals, rhs, precision)
        pd = problem_desc(problem)
        self._check(lib().dgp_run(self._h, C.byref(pd), precision, rule_mode, vals.data_ptr(), rhs.data_ptr()),
                    "dgp_run")

    def run_static(self, problem: dict, precision, vals, rhs, rule_mode=RULE_PLAIN):
        """dgp_run with the step's scratch in the library's static device array (allocates nothing)."""
        self._tensors_ok(vals, rhs, precision)
        pd = problem_desc(problem)
        self._check(lib().dgp_run_static(self._h, C.byref(pd), precision, rule_mode, vals.data_ptr(),
                                         rhs.data_ptr()), "dgp_run_static")

    def graph_capture(self, what, problem: dict, precision, vals, rhs, rule_mode=RULE_PLAIN):
        self._tensors_ok(vals, rhs, precision)
        pd = problem_desc(problem)
        self._check(lib().dgp_graph_capture(self._h, what, C.byref(pd), precision, rule_mode, vals.data_ptr(),
                                            rhs.data_ptr()), "dgp_graph_capture")

    def assemble_coo(self, problem: dict, precision):
        """The Approach-1 ablation (COO records, radix sort, segmented sums): a dict
        of device tensors row_ptr, col_idx, val_ptr, dof_ptr, vals, rhs."""
        import torch
        i = self.info or self.pattern()
        dev = torch.device("cuda", self.device)
        dt = torch.float32 if precision == F32 else torch.float64
        out = dict(row_ptr=torch.empty(i.n_rows + 1, dtype=torch.int64, device=dev),
                   col_idx=torch.empty(i.nnzb, dtype=torch.int32, device=dev),
                   val_ptr=torch.empty(i.nnzb + 1, dtype=torch.int64, device=dev),
                   dof_ptr=torch.empty(i.n_rows + 1, dtype=torch.int64, device=dev),
                   vals=torch.empty(i.n_vals, dtype=dt, device=dev),
                   rhs=torch.empty(i.n_dofs, dtype=dt, device=dev))
        pd = problem_desc(problem)
        self._keep = (out["vals"], out["rhs"])
        self._check(lib().dgp_assemble_coo(self._h, C.byref(pd), precision, out["vals"].data_ptr(),
                                           out["rhs"].data_ptr(), out["row_ptr"].data_ptr(),
                                           out["col_idx"].data_ptr(), out["val_ptr"].data_ptr(),
                                           out["dof_ptr"].data_ptr()), "dgp_assemble_coo")
        return out

    def assemble_st(self, problem: dict, precision, t0, t1, tau=(0.0, 0.0), prev=None, tp0=None, out=None):
        """One space-time slab (t0, t1] on prisms over the uploaded 2D mesh (uniform
        degree): (vals, rhs) device tensors, blocks of n_b = (p+1)(p+2)(p+3)/6 on
        the spatial pattern; prev = previous slab's FP64 coefficients (device) or None."""
        import torch
        i = self.info or self.pattern()
        p = int(self._p_uniform())
        nb = (p + 1) * (p + 2) * (p + 3) // 6
        dev = torch.device("cuda", self.device)
        dt = torch.float32 if precision == F32 else torch.float64
        if out is None:
            out = (torch.empty(i.nnzb * nb * nb, dtype=dt, device=dev), torch.empty(i.n_rows * nb, dtype=dt, device=dev))
        vals, rhs = out
        if vals.numel() < i.nnzb * nb * nb or rhs.numel() < i.n_rows * nb or vals.dtype != dt or rhs.dtype != dt:
            raise ValueError("space-time outputs of the wrong size or type")
        sl = SlabDesc(t0, t1, tp0 if tp0 is not None else t0 - (t1 - t0), tau[0], tau[1],
                      prev.data_ptr() if prev is not None else None)
        if prev is not None and (prev.dtype != torch.float64 or prev.numel() < i.n_rows * nb or not prev.is_cuda):
            raise ValueError("prev must be a device FP64 tensor of n_cells * n_b coefficients")
        pd = problem_desc(problem)
        self._keep = (vals, rhs, prev)
        self._check(lib().dgp_assemble_st(self._h, C.byref(pd), precision, C.byref(sl), vals.data_ptr(),
                                          rhs.data_ptr()), "dgp_assemble_st")
        return vals, rhs

    def _p_uniform(self):
        return self._p

    def graph_launch(self):
        self._check(lib().dgp_graph_launch(self._h), "dgp_graph_launch")

    def set_timing(self, on: bool):
        self._check(lib().dgp_set_timing(self._h, 1 if on else 0), "dgp_set_timing")

    def time_kernels(self, reps=50):
        """(prep, assembly) device ms per launch, averaged over reps back-to-back re-launches."""
        a, b = C.c_float(), C.c_float()
        self._check(lib().dgp_time_kernels(self._h, reps, C.byref(a), C.byref(b)), "dgp_time_kernels")
        return a.value, b.value

    def autotune(self, budget_ms=200):
        """Pick each degree bin's 2D launch configuration (cfg = register budget
        + 2 * row order) for the last assembly's precision; returns the
        [FP64, FP32][degree] table of configurations in use."""
        out = (C.c_int32 * 10)()
        self._check(lib().dgp_autotune(self._h, int(budget_ms), C.cast(out, C.c_void_p)), "dgp_autotune")
        return [[out[q * 5 + p] for p in range(5)] for q in range(2)]

    def set_launch(self, precision, p, cfg):
        """Set the 2D launch configuration of one precision and degree."""
        self._check(lib().dgp_set_launch(self._h, precision, int(p), int(cfg)), "dgp_set_launch")

    def kernel_ms(self, name: str) -> float:
        ms = C.c_float()
        self._check(lib().dgp_kernel_ms(self._h, name.encode(), C.byref(ms)), "dgp_kernel_ms")
        return ms.value

    # ------------------------------------------------------ reduced volume rules
    def mlp_load(self, params):
        a = np.ascontiguousarray(params, dtype=np.float32)
        self._check(lib().dgp_mlp_load(self._h, a.ctypes.data, a.size), "dgp_mlp_load")

    def qrule_build(self, init=INIT_NETWORK, max_iters=8, tol=1e-10) -> QruleStats:
        st = QruleStats()
        self._check(lib().dgp_qrule_build(self._h, init, max_iters, tol, C.byref(st)), "dgp_qrule_build")
        return st

    def qrule_get(self):
        """nodes [N,16,2], weights [N,16], accepted [N] (uint8), residual [N], iters [N] as device tensors."""
        import torch
        n = self.info.n_rows
        dev = torch.device("cuda", self.device)
        nodes = torch.empty((n, 16, 2), dtype=torch.float64, device=dev)
        w = torch.empty((n, 16), dtype=torch.float64, device=dev)
        ok = torch.empty(n, dtype=torch.uint8, device=dev)
        res = torch.empty(n, dtype=torch.float64, device=dev)
        it = torch.empty(n, dtype=torch.int32, device=dev)
        self._check(lib().dgp_qrule_get(self._h, nodes.data_ptr(), w.data_ptr(), ok.data_ptr(), res.data_ptr(),
                                        it.data_ptr()), "dgp_qrule_get")
        return nodes, w, ok, res, it

    def qrule_cell_data(self):
        import torch
        n = self.info.n_rows
        dev = torch.device("cuda", self.device)
        feat = torch.empty((n, 36), dtype=torch.float32, device=dev)
        mom = torch.empty((n, 28), dtype=torch.float64, device=dev)
        area = torch.empty(n, dtype=torch.float64, device=dev)
        self._check(lib().dgp_qrule_cell_data(self._h, feat.data_ptr(), mom.data_ptr(), area.data_ptr()),
                    "dgp_qrule_cell_data")
        return feat, mom, area

    def train_polygons(self, seed, first, n, with_f64=False):
        import torch
        dev = torch.device("cuda", self.device)
        feat = torch.empty((n, 36), dtype=torch.float32, device=dev)
        f64 = torch.empty((n, 36), dtype=torch.float64, device=dev) if with_f64 else None
        mom = torch.empty((n, 28), dtype=torch.float64, device=dev)
        area = torch.empty(n, dtype=torch.float64, device=dev)
        self._check(lib().dgp_train_polygons(self._h, seed, first, n, feat.data_ptr(),
                                             f64.data_ptr() if f64 is not None else None, mom.data_ptr(),
                                             area.data_ptr()), "dgp_train_polygons")
        return feat, f64, mom, area

    def mlp_forward(self, params, x):
        import torch
        out = torch.empty((x.shape[0], 48), dtype=torch.float32, device=x.device)
        self._check(lib().dgp_mlp_forward(self._h, params.data_ptr(), x.data_ptr(), x.shape[0], out.data_ptr()),
                    "dgp_mlp_forward")
        return out

    def mlp_loss_grad(self, params, x, moments, area):
        import torch
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
        loss = torch.empty(1, dtype=torch.float32, device=x.device)
        self._check(lib().dgp_mlp_loss_grad(self._h, params.data_ptr(), x.data_ptr(), moments.data_ptr(),
                                            area.data_ptr(), x.shape[0], g.data_ptr(), loss.data_ptr()),
                    "dgp_mlp_loss_grad")
        return g, loss

    def adam_step(self, params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self._check(lib().dgp_adam_step(self._h, params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(),
                                        params.numel(), t, lr, beta1, beta2, eps), "dgp_adam_step")

    def mlp_train(self, n_polygons, data_seed, init_seed=1, epochs=10, batch=4096, lr=2e-3, beta1=0.9,
                  beta2=0.999, eps=1e-8):
        cfg = TrainCfg(n_polygons, data_seed, init_seed, epochs, batch, lr, beta1, beta2, eps)
        params = np.empty(MLP_PARAMS, dtype=np.float32)
        losses = np.empty(epochs, dtype=np.float32)
        st = TrainStats()
        self._check(lib().dgp_mlp_train(self._h, C.byref(cfg), params.ctypes.data, losses.ctypes.data,
                                        C.byref(st)), "dgp_mlp_train")
        return params, losses, st
