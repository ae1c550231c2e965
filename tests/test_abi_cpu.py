"""CPU checks of the C-ABI library: it loads, exports every function the header
declares, and the binding mirrors the header's structs.  No device calls."""

import ctypes as C
import os
import re
import subprocess

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
