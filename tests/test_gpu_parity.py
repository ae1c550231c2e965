"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Pattern arrays bit-exact; values per block within 1e-12 (FP64 path) or 1e-5
(FP32 path) relative Frobenius error, the right-hand side per element row the
same.  Sizes span many work-groups and a ragged last one; the headline
workload (16,384 cells, p = 2, variable diffusion, advection, reaction) is
checked in full, in the launch configuration the benchmark times.
"""

import numpy as np
import pytest

import oracle
from meshgen import cartesian_mesh, config_mesh, problem_params, split_cartesian_mesh, voronoi_mesh
from tests.parity import TOL, block_errors, check_pattern, gpu_assemble, oracle_problem

pytestmark = pytest.mark.gpu

DAR = dict(a0=1.0, a1=0.5, b=(1.0, 0.5, 0.0), c=1.0, c_sigma=10.0, u="sin")
POISSON = dict(a0=1.0, a1=0.0, b=(0.0, 0.0, 0.0), c=0.0, c_sigma=10.0, u="sin")
POLY = dict(a0=1.3, a1=0.0, b=(0.4, -0.7, 0.0), c=0.9, c_sigma=10.0, u="poly",
            u_poly=(1.0, 2.0, -1.0, 0.0, 1.0, -0.5, 0.0, 1.0, 0.0, 0.0))


def _case(mesh, params, precision, full_path=False):
    print(f"[case] {mesh.name} p={sorted(set(mesh.cell_p.tolist()))} prec={precision} full={full_path}", flush=True)
    pat = oracle.pattern(mesh)
    g = gpu_assemble(mesh, params, precision, full_path)
    check_pattern(g, pat)
    vals, rhs = oracle.assemble(mesh, oracle_problem(params), pat=pat)
    where = {}
    eb, er = block_errors(g, vals, rhs, pat, where=where)
    print(f"       worst block {eb:.3e} (row {where['row']})  worst rhs row {er:.3e} (row {where['rhs_row']})", flush=True)
    assert eb <= TOL[precision], eb
    assert er <= TOL[precision], er
    return g


@pytest.mark.parametrize("precision", [0, 1])
def test_workload1_64_cells(precision):
    _case(config_mesh(1), problem_params(1), precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_workload2_full_size(precision):
    _case(config_mesh(2), problem_params(2), precision)


@pytest.mark.parametrize("p", [1, 2, 3, 4])
@pytest.mark.parametrize("precision", [0, 1])
def test_voronoi_degrees(p, precision):
    # 1000 cells: 32 rows per FP32 work-group -> a ragged last work-group
    m = voronoi_mesh(1000, 77, lloyd=1, p=p)
    _case(m, DAR, precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_mixed_degrees(precision):
    # degrees drawn from {1, 2, 3, 4}: one launch per degree, cross blocks n_b(p) x n_b(p')
    m = voronoi_mesh(1000, 79, lloyd=1, p=1)
    m = m.with_degrees(np.random.default_rng(7).integers(1, 5, m.n_cells))
    _case(m, DAR, precision)
    _case(m, POLY, precision, full_path=True)


def _full_size_case(mesh, params, precision):
    """Full-size run in the benchmark's launch configuration (whole path), every
    row compared with the oracle; the worst block's row is printed."""
    print(f"[case] {mesh.name} cells={mesh.n_cells} prec={precision} full size", flush=True)
    pat = oracle.pattern(mesh)
    g = gpu_assemble(mesh, params, precision, full_path=True)
    check_pattern(g, pat)
    vals, rhs = oracle.assemble(mesh, oracle_problem(params), pat=pat)
    where = {}
    eb, er = block_errors(g, vals, rhs, pat, where=where)
    r = where["row"]
    print(f"       worst block {eb:.3e} (row {r}, p={mesh.cell_p[r]}, "
          f"{mesh.cell_ptr[r + 1] - mesh.cell_ptr[r]} vertices, block {where['block']})  "
          f"worst rhs row {er:.3e} (row {where['rhs_row']}) over {mesh.n_cells} rows", flush=True)
    assert eb <= TOL[precision], eb
    assert er <= TOL[precision], er


@pytest.mark.parametrize("precision", [0, 1])
def test_workload3_mixed_degrees_full_size(precision):
    _full_size_case(config_mesh(3), problem_params(3), precision)


@pytest.mark.parametrize("precision", [1, 0])
def test_workload5_p3_full_size(precision):
    _full_size_case(config_mesh(5), problem_params(5), precision)


@pytest.mark.parametrize("n_cells", [32768, 32800])
def test_tile_sums_at_the_inline_limit(n_cells):
    # 1,024 tiles of 32 cells: the assembly adds up the tile sums before its
    # tile itself (up to 16 loads per lane); 1,025 tiles: the scan kernel runs
    _full_size_case(voronoi_mesh(n_cells, 85, lloyd=0, p=2), DAR, 1)


@pytest.mark.parametrize("precision", [0, 1])
def test_polynomial_data_and_full_path(precision):
    m = voronoi_mesh(333, 78, lloyd=2, p=2)
    _case(m, POLY, precision, full_path=True)


@pytest.mark.parametrize("precision", [0, 1])
def test_pure_advection(precision):
    """a = 0 (the hyperbolic case): no diffusion terms and sigma = 0, so only the
    element advection-reaction terms and the upwind face terms remain; on the
    boundary only the inflow part (b . n < 0) carries the Dirichlet data."""
    m = voronoi_mesh(700, 88, lloyd=1, p=1)
    m = m.with_degrees(np.random.default_rng(10).integers(1, 5, m.n_cells))
    _case(m, dict(a0=0.0, a1=0.0, b=(1.0, -0.4, 0.0), c=0.5, c_sigma=10.0, u="sin"), precision)
    _case(m, dict(POLY, a0=0.0), precision)
    # one degree (the FP32 one-degree row kernel for p <= 2)
    for p in (1, 2):
        u = voronoi_mesh(500, 89, lloyd=1, p=p)
        _case(u, dict(a0=0.0, a1=0.0, b=(1.0, -0.4, 0.0), c=0.5, c_sigma=10.0, u="sin"), precision)


@pytest.mark.parametrize("precision", [0, 1])
def test_covering_penalty(precision):
    """sigma_F of Appendix A with the fan sub-triangles as the covering (per face:
    |F|, the sub-triangle having F as a side, |kappa|, C_cov = p^2), on mixed
    degrees with variable a, and on octagons whose degenerate fan triangles
    leave the C_cov bound and whose neighbours share two edges."""
    m = voronoi_mesh(1000, 94, lloyd=1, p=1)
    m = m.with_degrees(np.random.default_rng(13).integers(1, 5, m.n_cells))
    _case(m, dict(DAR, penalty="covering"), precision)
    _case(m, dict(POLY, penalty="covering"), precision, full_path=True)
    s = split_cartesian_mesh(12, 10, p=2, x0=0.1, x1=1.3, y0=-0.2, y1=0.9)
    _case(s, dict(DAR, penalty="covering"), precision)
    g = voronoi_mesh(16384, 2007048812, lloyd=0, p=2)  # the benchmark's mesh size
    _case(g, dict(DAR, penalty="covering"), precision, full_path=True)


@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("precision", [0, 1])
def test_cartesian_and_neumann(p, precision):
    m = cartesian_mesh(7, 5, p=p, x0=0.1, x1=1.3, y0=-0.2, y1=0.9)
    _case(m, DAR, precision)
    # turn the faces on the left side into Neumann faces
    m2 = cartesian_mesh(7, 5, p=p)
    xl = np.where(m2.x == 0.0)[0]
    fv = m2.face_vtx.reshape(-1, 2)
    left = np.isin(fv[:, 0], xl) & np.isin(fv[:, 1], xl)
    m2.face_bc[left] = 2
    _case(m2, DAR, precision)
    _case(m2, POLY, precision)


@pytest.mark.parametrize("p", [1, 2, "mixed"])
@pytest.mark.parametrize("precision", [0, 1])
def test_neighbours_sharing_two_edges(p, precision):
    # octagons whose neighbours share two collinear edges each: the second edge
    # of every neighbour group is a second point set added to the same block;
    # 24 x 20 cells span several work-groups and a ragged last one
    m = split_cartesian_mesh(24, 20, p=1 if p == "mixed" else p, x0=0.1, x1=1.3, y0=-0.2, y1=0.9)
    if p == "mixed":
        m = m.with_degrees(np.random.default_rng(5).integers(1, 4, m.n_cells))
    _case(m, DAR, precision)
    _case(m, POLY, precision)


def test_single_cell_and_tiny():
    m = cartesian_mesh(1, 1, p=2)
    _case(m, DAR, 0)
    _case(voronoi_mesh(5, 3, p=1), POISSON, 1)


def test_deterministic_and_graph_replay():
    import torch
    import paper_2007_04881_amd as D
    m = config_mesh(2)
    params = problem_params(2)
    ctx = D.Context(0)
    ctx.upload(m)
    ctx.pattern()
    v1, r1 = ctx.outputs(D.F32)
    ctx.run(params, D.F32, v1, r1)
    torch.cuda.synchronize()
    v2, r2 = ctx.outputs(D.F32)
    ctx.assemble(params, D.F32, v2, r2)
    torch.cuda.synchronize()
    assert torch.equal(v1, v2) and torch.equal(r1, r2)
    # re-launching the step's kernels for timing rewrites the same values
    prep_ms, asm_ms = ctx.time_kernels(3)
    torch.cuda.synchronize()
    assert prep_ms > 0.0 and asm_ms > 0.0
    assert torch.equal(v1, v2) and torch.equal(r1, r2)
    for what in (0, 1):
        v3, r3 = ctx.outputs(D.F32)
        ctx.graph_capture(what, params, D.F32, v3, r3)
        for rep in range(3):
            v3.fill_(-1.0)
            r3.fill_(-1.0)
            torch.cuda.synchronize()
            ctx.graph_launch()
            torch.cuda.synchronize()
            assert torch.equal(v1, v3) and torch.equal(r1, r3), (what, rep)
    ctx.close()


def test_error_paths():
    import paper_2007_04881_amd as D
    ctx = D.Context(0)
    with pytest.raises(D.DgpError) as e:
        ctx.pattern()
    assert e.value.status == -6
    m = voronoi_mesh(50, 5, p=2)
    bad = m.with_degrees(2)
    bad.cell_vtx = bad.cell_vtx.copy()
    bad.cell_vtx[3] = bad.n_vertices + 5
    with pytest.raises(D.DgpError) as e:
        ctx.upload(bad)
    assert e.value.status == -2
    bad = m.with_degrees(2)
    bad.face_cell = bad.face_cell.copy()
    f = int(np.where(bad.face_cell[1::2] >= 0)[0][0])
    bad.face_cell[2 * f + 1] = (bad.face_cell[2 * f] + 7) % bad.n_cells
    with pytest.raises(D.DgpError):
        ctx.upload(bad)
    with pytest.raises(D.DgpError) as e:
        ctx.upload(m.with_degrees(7))
    assert e.value.status == -3
    ctx.upload(m)
    ctx.pattern()
    v, r = ctx.outputs(D.F32)
    with pytest.raises(ValueError):
        ctx.assemble(DAR, D.F64, v, r)
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_autotune_keeps_results(precision):
    """dgp_autotune picks each degree bin's register budget; the arithmetic is
    the same in both, so the values after tuning are bit-identical."""
    import torch
    import paper_2007_04881_amd as D

    m = voronoi_mesh(1000, 83, lloyd=1, p=1)
    m = m.with_degrees(np.random.default_rng(8).integers(1, 5, m.n_cells))
    ctx = D.Context(0)
    ctx.upload(m)
    ctx.pattern()
    vals, rhs = ctx.outputs(precision)
    with pytest.raises(D.DgpError) as e:
        ctx.autotune(50)
    assert e.value.status == -6
    ctx.assemble(DAR, precision, vals, rhs)
    torch.cuda.synchronize()
    v0, r0 = vals.clone(), rhs.clone()
    choice = ctx.autotune(50)
    assert all(c in (0, 1, 2, 3) for row in choice for c in row)
    vals.fill_(float("nan"))
    rhs.fill_(float("nan"))
    ctx.assemble(DAR, precision, vals, rhs)
    torch.cuda.synchronize()
    assert torch.equal(vals, v0) and torch.equal(rhs, r0)
    ctx.close()


@pytest.mark.parametrize("mixed", [False, True])
@pytest.mark.parametrize("precision", [0, 1])
def test_launch_configurations(mixed, precision):
    """Every 2D launch configuration (register budget x row order: id order or
    the (degree, sub-triangle count) bins) gives bit-identical values and the
    full path's pattern; configuration 0 is checked against the oracle."""
    import torch
    import paper_2007_04881_amd as D

    m = voronoi_mesh(1500, 84, lloyd=0, p=2)  # raw seeds: 3 to 12 vertices per cell
    if mixed:
        m = m.with_degrees(np.random.default_rng(9).integers(1, 5, m.n_cells))
    pat = oracle.pattern(m)
    ctx = D.Context(0)
    ctx.upload(m)
    ctx.pattern()
    vals, rhs = ctx.outputs(precision)
    ref = None
    for cfg in range(4):
        print(f"[case] mixed={mixed} prec={precision} cfg={cfg}", flush=True)
        for p in range(1, 5):
            ctx.set_launch(precision, p, cfg)
        vals.fill_(float("nan"))
        rhs.fill_(float("nan"))
        ctx.run(DAR, precision, vals, rhs)
        rp, ci, vp, dp = ctx.pattern_tensors()
        torch.cuda.synchronize()
        assert np.array_equal(rp.cpu().numpy(), pat.row_ptr) and np.array_equal(ci.cpu().numpy(), pat.col_idx)
        assert np.array_equal(vp.cpu().numpy(), pat.val_ptr) and np.array_equal(dp.cpu().numpy(), pat.dof_ptr)
        if ref is None:
            ref = vals.clone(), rhs.clone()
            g = dict(vals=vals.double().cpu().numpy(), rhs=rhs.double().cpu().numpy())
            ov, orhs = oracle.assemble(m, oracle_problem(DAR), pat=pat)
            eb, er = block_errors(g, ov, orhs, pat)
            assert eb <= TOL[precision] and er <= TOL[precision], (eb, er)
        else:
            assert torch.equal(vals, ref[0]) and torch.equal(rhs, ref[1])
    with pytest.raises(D.DgpError):
        ctx.set_launch(precision, 2, 4)
    with pytest.raises(D.DgpError):
        ctx.set_launch(precision, 5, 0)
    ctx.close()


def test_back_to_back_steps():
    """Steps issued back to back without synchronisation, with different data
    and outputs and a graph replay between them, equal the same steps run one
    at a time (the preparation outputs are reused by every step)."""
    import torch
    import paper_2007_04881_amd as D

    m = voronoi_mesh(3000, 86, lloyd=1, p=2)
    probs = [DAR, POISSON, POLY, dict(DAR, a1=0.25, c=2.0), DAR, POLY]
    ref = []
    solo = D.Context(0)
    solo.upload(m)
    solo.pattern()
    for pr in probs:
        v, r = solo.outputs(1)
        solo.run(pr, 1, v, r)
        torch.cuda.synchronize()
        ref.append((v.clone(), r.clone()))
    solo.close()
    ctx = D.Context(0)
    ctx.upload(m)
    ctx.pattern()
    outs = [ctx.outputs(1) for _ in probs]
    for v, r in outs:
        v.fill_(float("nan"))
        r.fill_(float("nan"))
    torch.cuda.synchronize()
    ctx.graph_capture(0, probs[2], 1, *outs[2])
    for k in (0, 1):
        ctx.run(probs[k], 1, *outs[k])
    ctx.graph_launch()
    for k in (3, 4, 5):
        ctx.run(probs[k], 1, *outs[k])
    torch.cuda.synchronize()
    for k, (v, r) in enumerate(outs):
        assert torch.equal(v, ref[k][0]) and torch.equal(r, ref[k][1]), k
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_single_persistent_launch_over_all_bins(precision):
    """Mixed degrees in one persistent launch (rows bin by bin, costliest
    first, static assignment to the resident waves) give bit-identical values
    and pattern to one launch per degree, also captured in a graph; the
    tuner's choice between the two keeps the results."""
    import torch
    import paper_2007_04881_amd as D

    m = voronoi_mesh(5000, 87, lloyd=0, p=1)
    m = m.with_degrees(np.random.default_rng(14).integers(1, 5, m.n_cells))
    pat = oracle.pattern(m)
    ctx = D.Context(0)
    ctx.upload(m)
    ctx.pattern()
    outs = {}
    for fused in (0, 1):
        print(f"[case] mixed degrees prec={precision} single launch={fused}", flush=True)
        ctx.set_launch(precision, 0, fused)
        v, r = ctx.outputs(precision)
        v.fill_(float("nan"))
        r.fill_(float("nan"))
        ctx.run(DAR, precision, v, r)
        torch.cuda.synchronize()
        rp, ci, vp, dp = ctx.pattern_tensors()
        assert np.array_equal(rp.cpu().numpy(), pat.row_ptr) and np.array_equal(ci.cpu().numpy(), pat.col_idx)
        assert np.array_equal(vp.cpu().numpy(), pat.val_ptr) and np.array_equal(dp.cpu().numpy(), pat.dof_ptr)
        outs[fused] = (v.clone(), r.clone())
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])
    g = dict(vals=outs[1][0].double().cpu().numpy(), rhs=outs[1][1].double().cpu().numpy())
    ov, orhs = oracle.assemble(m, oracle_problem(DAR), pat=pat)
    eb, er = block_errors(g, ov, orhs, pat)
    assert eb <= TOL[precision] and er <= TOL[precision], (eb, er)
    # graph replay of the single launch
    v3, r3 = ctx.outputs(precision)
    ctx.graph_capture(0, DAR, precision, v3, r3)
    for _ in range(3):
        v3.fill_(-1.0)
        torch.cuda.synchronize()
        ctx.graph_launch()
        torch.cuda.synchronize()
        assert torch.equal(v3, outs[1][0]) and torch.equal(r3, outs[1][1])
    # the tuner picks one of the two; results unchanged
    ctx.run(DAR, precision, v3, r3)
    choice = ctx.autotune(100)
    assert choice[1 if precision == 1 else 0][0] in (0, 1)
    v3.fill_(float("nan"))
    ctx.run(DAR, precision, v3, r3)
    torch.cuda.synchronize()
    assert torch.equal(v3, outs[1][0]) and torch.equal(r3, outs[1][1])
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_small_cells_far_from_the_origin(precision):
    """Cells of size ~1e-4 near (0.7, 0.8), degrees 1..4, variable a with
    advection: quadrature points enter the basis through their offsets from a
    mesh vertex on both sides, so FP64 agrees to 1e-12 although absolute
    coordinates carry rounding of ~1e-12 of a cell."""
    import copy
    m = voronoi_mesh(400, 89, lloyd=1, p=1)
    m = m.with_degrees(np.random.default_rng(15).integers(1, 5, m.n_cells))
    t = copy.deepcopy(m)
    t.x = 0.7 + 2.0 ** -12 * m.x
    t.y = 0.8 + 2.0 ** -12 * m.y
    t.name = m.name + "_small"
    _case(t, DAR, precision)
    _case(t, dict(DAR, penalty="covering"), precision)
