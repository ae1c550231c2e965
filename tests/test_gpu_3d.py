"""GPU parity in 3D: polyhedra agglomerated from Kuhn tetrahedra, the HIP path
(through the C ABI) against the FP64 oracle.

Pattern arrays bit-exact; values per block within 1e-12 (FP64) or 1e-5 (FP32)
relative Frobenius error, the right-hand side per row the same.  The
128^3-cube workload (32,768 polyhedra, p = 2) is checked in full for the
pattern and on sampled rows for the values, in the launch configuration the
benchmark times.
"""

import numpy as np
import pytest

import oracle
from meshgen import config_mesh, problem_params
from meshgen.kuhn import agglomerated_cube, cube_cells
from tests.parity import TOL, block_errors, check_pattern, gpu_assemble, oracle_problem

pytestmark = pytest.mark.gpu

POISSON3 = dict(a0=1.0, a1=0.0, b=(0.0, 0.0, 0.0), c=0.0, c_sigma=10.0, u="sin")
DAR3 = dict(a0=1.3, a1=0.0, b=(0.4, -0.7, 0.5), c=0.9, c_sigma=10.0, u="sin")
ADV3 = dict(a0=0.8, a1=0.0, b=(-0.6, 0.3, 0.9), c=0.0, c_sigma=10.0, u="sin")
POLY3 = dict(a0=1.3, a1=0.0, b=(0.4, -0.7, 0.5), c=0.9, c_sigma=10.0, u="poly",
             u_poly=(1.0, 2.0, -1.0, 0.5, 1.0, -0.5, 0.75, 1.0, -0.25, 0.6))


def _case(mesh, params, precision, rows=None):
    print(f"[case] {mesh.name} p={sorted(set(mesh.cell_p.tolist()))} prec={precision} "
          f"b={params['b']} c={params['c']} u={params['u']}", flush=True)
    pat = oracle.pattern(mesh)
    g = gpu_assemble(mesh, params, precision)
    check_pattern(g, pat)
    vals, rhs = oracle.assemble(mesh, oracle_problem(params), rows=rows, pat=pat)
    where = {}
    eb, er = block_errors(g, vals, rhs, pat, rows=rows, where=where)
    print(f"       worst block {eb:.3e} (row {where['row']})  worst rhs row {er:.3e} (row {where['rhs_row']})", flush=True)
    assert eb <= TOL[precision], eb
    assert er <= TOL[precision], er
    return g


@pytest.mark.parametrize("params", [POISSON3, DAR3, ADV3, POLY3], ids=["poisson", "dar", "adv", "poly"])
@pytest.mark.parametrize("precision", [0, 1])
def test_agglomerated_p2(params, precision):
    # 3,072 tetrahedra in 70 polyhedra: 18 work-groups of 4 rows, the last one ragged
    _case(agglomerated_cube(8, 70, 2024, p=2), params, precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_agglomerated_p1(precision):
    _case(agglomerated_cube(8, 70, 2025, p=1), DAR3, precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_mixed_degrees_3d(precision):
    m = agglomerated_cube(8, 70, 2026, p=1)
    m = m.with_degrees(np.random.default_rng(5).integers(1, 3, m.n_cells))
    _case(m, DAR3, precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_pure_advection_3d(precision):
    """a = 0: advection, reaction and upwind faces only (sigma = 0)."""
    _case(agglomerated_cube(8, 70, 2032, p=2), dict(ADV3, a0=0.0, c=0.7), precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_cubic_cells(precision):
    _case(cube_cells(4, p=2), DAR3, precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_neumann_faces(precision):
    """Boundary triangles on the x = 0 side carry Neumann data instead of Dirichlet."""
    m = agglomerated_cube(6, 30, 2027, p=2)
    fv = m.face_vtx.reshape(-1, 3)
    on_x0 = (m.face_bc == 1) & (np.abs(m.x[fv]).max(axis=1) == 0.0)
    assert on_x0.any()
    m.face_bc = np.where(on_x0, 2, m.face_bc).astype(np.int8)
    _case(m, DAR3, precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_large_cells_and_groups(precision):
    """Three polyhedra of about 1,000 tetrahedra each: several hundred faces per
    cell and interfaces of more than 64 triangles (staged in several chunks)."""
    m = agglomerated_cube(8, 3, 2029, p=2)
    fc = m.face_cell.reshape(-1, 2)
    inner = fc[fc[:, 1] >= 0]
    _, counts = np.unique(inner, axis=0, return_counts=True)
    assert counts.max() > 64
    _case(m, DAR3, precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_unordered_face_lists(precision):
    """Each cell's face list in a random order: the preparation kernel groups the
    faces by neighbour itself (the pattern is unchanged, the sums are reordered)."""
    m = agglomerated_cube(8, 70, 2030, p=2)
    rng = np.random.default_rng(3)
    cf = m.cell_face.copy()
    for c in range(m.n_cells):
        s, e = m.cell_face_ptr[c], m.cell_face_ptr[c + 1]
        cf[s:e] = rng.permutation(cf[s:e])
    m.cell_face = cf
    _case(m, DAR3, precision)


def test_3d_graph_replay_deterministic():
    """The captured whole path replayed: every replay bit-identical to the eager result."""
    import torch
    import paper_2007_04881_amd as D

    m = agglomerated_cube(8, 70, 2031, p=2)
    ctx = D.Context(0)
    ctx.upload(m)
    ctx.pattern()
    vals, rhs = ctx.outputs(1)
    ctx.run(DAR3, 1, vals, rhs)
    torch.cuda.synchronize()
    v0, r0 = vals.clone(), rhs.clone()
    ctx.graph_capture(0, DAR3, 1, vals, rhs)
    for _ in range(4):
        vals.fill_(float("nan"))
        rhs.fill_(float("nan"))
        ctx.graph_launch()
        torch.cuda.synchronize()
        assert torch.equal(vals, v0) and torch.equal(rhs, r0)
        ctx.run(DAR3, 1, vals, rhs)  # eager work between replays
        torch.cuda.synchronize()
    ctx.close()


@pytest.mark.parametrize("precision", [1, 0])
def test_workload4_full_size_sampled(precision):
    """128^3 cubes, 12.6M Kuhn tetrahedra in 32,768 polyhedra, p = 2: full
    pattern, values of 2,049 rows (every 16th row, and the last)."""
    m = config_mesh(4)
    rows = np.unique(np.concatenate([np.arange(0, m.n_cells, 16), [m.n_cells - 1]]))
    _case(m, problem_params(4), precision, rows=rows)


@pytest.mark.parametrize("params", [DAR3, ADV3], ids=["dar", "adv"])
@pytest.mark.parametrize("precision", [0, 1])
def test_cells_near_their_centre(params, precision):
    """16^3 cubes of 6 tetrahedra each: every cell fits within the radius where
    the kernels take sin/cos of the manufactured data by angle addition from
    the box centre (pi times half the box diagonal <= 0.2), so the short series
    of the load, with and without advection, are compared in full."""
    m = cube_cells(16, p=2)
    _case(m, params, precision)


def test_3d_error_paths():
    import torch
    import paper_2007_04881_amd as D

    m = agglomerated_cube(4, 5, 2028, p=2)
    ctx = D.Context(0)
    ctx.upload(m)
    ctx.pattern()
    vals, rhs = ctx.outputs(1)
    with pytest.raises(D.DgpError) as e:
        ctx.assemble(dict(POISSON3, a1=0.5), 1, vals, rhs)
    assert e.value.status == -3
    with pytest.raises(D.DgpError) as e:
        ctx.assemble(POISSON3, 1, vals, rhs, rule_mode=D.RULE_REDUCED)
    assert e.value.status in (-3, -6)
    with pytest.raises(D.DgpError) as e:
        ctx.assemble(dict(POISSON3, penalty="covering"), 1, vals, rhs)
    assert e.value.status == -3
    ctx.close()
    # degree 3 is outside the 3D kernels
    ctx = D.Context(0)
    with pytest.raises(D.DgpError) as e:
        ctx.upload(m.with_degrees(3))
    assert e.value.status == -3
    ctx.close()
    torch.cuda.synchronize()
