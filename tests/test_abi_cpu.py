"""CPU checks of the C-ABI library: it loads, exports every function the header
declares, and the binding mirrors the header's structs.  No device calls."""

import copy
import ctypes as C
import os
import re
import subprocess

import numpy as np

import paper_2007_04881_amd as D

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "dgpoly.h")).read()
    return sorted(set(re.findall(r"^\S.*?\b(dgp_[a-z_0-9]+)\s*\(", src, re.M)))


def test_every_declared_symbol_is_exported():
    lib = C.CDLL(D.LIB_PATH)
    names = _declared()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(D.EXPORTS) == names


def test_struct_layouts_match_header(tmp_path):
    """Compile a C program against the header and compare every field offset."""
    structs = {"dgp_mesh_desc": D.MeshDesc, "dgp_problem": D.ProblemDesc, "dgp_pattern_info": D.PatternInfo,
               "dgp_qrule_stats": D.QruleStats, "dgp_train_cfg": D.TrainCfg, "dgp_train_stats": D.TrainStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dgpoly.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_library_is_built_for_gfx950():
    data = open(D.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def _reverse_loop(m, c):
    """Copy of a 2D mesh with cell c's vertex loop reversed (clockwise), faces kept consistent."""
    m2 = copy.deepcopy(m)
    s, e = int(m.cell_ptr[c]), int(m.cell_ptr[c + 1])
    n = e - s
    loop = m.cell_vtx[s:e].copy()
    faces = m.cell_face[s:e].copy()
    # reversed loop [v0, v_{n-1}, ..., v1]: its edge k joins old vertices n-k and n-k-1
    m2.cell_vtx[s:e] = np.concatenate([loop[:1], loop[1:][::-1]])
    m2.cell_face[s:e] = [faces[(n - 1 - k) % n] for k in range(n)]
    return m2


def test_mesh_check_rejects_clockwise_and_degenerate_cells():
    """dgp_mesh_check (host only): a valid mesh passes; a clockwise loop, a
    zero-area polygon and a zero-volume tetrahedron fail with DGP_EMESH before
    anything reaches a device."""
    from meshgen import cube_cells, voronoi_mesh
    from meshgen.mesh import Mesh

    m = voronoi_mesh(40, 5, lloyd=1, p=2)
    assert D.mesh_check(m) == (0, "")
    st, msg = D.mesh_check(_reverse_loop(m, 7))
    assert st == -2 and "clockwise" in msg and "cell 7" in msg, msg
    # a triangle whose three vertices lie on one line
    tri = Mesh(dim=2, x=np.array([0.0, 1.0, 2.0]), y=np.array([0.0, 0.0, 0.0]), z=np.zeros(0),
               cell_ptr=np.array([0, 3], np.int64), cell_vtx=np.array([0, 1, 2], np.int32),
               cell_p=np.array([1], np.int8), cell_face_ptr=np.array([0, 3], np.int64),
               cell_face=np.array([0, 1, 2], np.int32), face_vtx=np.array([0, 1, 1, 2, 0, 2], np.int32),
               face_cell=np.array([0, -1, 0, -1, 0, -1], np.int32), face_bc=np.array([1, 1, 1], np.int8))
    st, msg = D.mesh_check(tri)
    assert st == -2 and "zero-area" in msg, msg
    good = cube_cells(2, p=2)
    assert D.mesh_check(good)[0] == 0
    flat = copy.deepcopy(good)
    flat.z = np.zeros_like(good.z)
    st, msg = D.mesh_check(flat)
    assert st == -2 and "zero volume" in msg, msg
    # degrees the kernels are not built for
    assert D.mesh_check(m.with_degrees(5))[0] == -3
