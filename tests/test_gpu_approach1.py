"""The Approach-1 ablation (Section 3.3: every element and face emits its local
blocks as COO records with duplicates; a radix sort by (row, column) and a
segmented reduction form the matrix) against the oracle: its own pattern must
be bit-identical to the oracle's, its values within the usual tolerances."""

import numpy as np
import pytest

import oracle
from meshgen import config_mesh, problem_params, voronoi_mesh, split_cartesian_mesh
from tests.parity import TOL, block_errors, check_pattern

pytestmark = pytest.mark.gpu

DAR = dict(a0=1.0, a1=0.5, b=(1.0, 0.5, 0.0), c=1.0, c_sigma=10.0, u="sin")


def _a1_case(mesh, params, precision):
    import torch
    import paper_2007_04881_amd as D
    print(f"[case] approach1 {mesh.name} cells={mesh.n_cells} p={int(mesh.cell_p[0])} prec={precision}", flush=True)
    pat = oracle.pattern(mesh)
    ctx = D.Context(0)
    ctx.upload(mesh)
    info = ctx.pattern()
    out = ctx.assemble_coo(params, precision)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items()}
    g["vals"] = out["vals"].double().cpu().numpy()
    g["rhs"] = out["rhs"].double().cpu().numpy()
    g["info"] = (info.n_rows, info.nnzb, info.n_vals, info.n_dofs)
    ctx.close()
    check_pattern(g, pat)
    ov, orhs = oracle.assemble(mesh, oracle.Problem.from_params(params), pat=pat)
    eb, er = block_errors(g, ov, orhs, pat)
    print(f"       worst block {eb:.3e}  worst rhs row {er:.3e}", flush=True)
    assert eb <= TOL[precision], eb
    assert er <= TOL[precision], er


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("precision", [0, 1])
def test_approach1_degrees(p, precision):
    _a1_case(voronoi_mesh(1000, 98, lloyd=0, p=p), DAR, precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_approach1_headline_mesh_and_octagons(precision):
    _a1_case(config_mesh(2), problem_params(2), precision)
    _a1_case(split_cartesian_mesh(12, 10, p=2, x0=0.1, x1=1.3, y0=-0.2, y1=0.9), dict(DAR, penalty="covering"),
             precision)


def test_approach1_refuses_mixed_degrees():
    import paper_2007_04881_amd as D
    m = voronoi_mesh(100, 99, p=1)
    m = m.with_degrees(np.random.default_rng(1).integers(1, 3, m.n_cells))
    ctx = D.Context(0)
    ctx.upload(m)
    ctx.pattern()
    with pytest.raises(D.DgpError) as e:
        ctx.assemble_coo(DAR, 1)
    assert e.value.status == -3
    ctx.close()
