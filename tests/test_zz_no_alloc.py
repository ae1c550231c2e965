"""dgp_run_static, the entry point that allocates nothing: the step's scratch
lives in the library's static device array.  Its output must equal dgp_run's
(same kernels, so bit for bit) on two calls in a row, the second with a
smaller mesh (the array then still holds the first call's larger contents),
and stay within the oracle's tolerance; a mesh needing more scratch than the
array holds is refused."""

import numpy as np
import pytest

import oracle
from meshgen import cartesian_mesh, voronoi_mesh
from meshgen.kuhn import agglomerated_cube
from tests.parity import TOL, block_errors, oracle_problem

pytestmark = pytest.mark.gpu

DAR = dict(a0=1.0, a1=0.5, b=(1.0, 0.5, 0.0), c=1.0, c_sigma=10.0, u="sin")
DAR3 = dict(a0=1.3, a1=0.0, b=(0.4, -0.7, 0.5), c=0.9, c_sigma=10.0, u="sin")


def _both(ctx, mesh, params, precision):
    """dgp_run and dgp_run_static on the same context and mesh."""
    import torch
    ctx.upload(mesh)
    ctx.pattern()
    v1, r1 = ctx.outputs(precision)
    v2, r2 = ctx.outputs(precision)
    v2.fill_(float("nan"))
    r2.fill_(float("nan"))
    ctx.run(params, precision, v1, r1)
    ctx.run_static(params, precision, v2, r2)
    torch.cuda.synchronize()
    return v1, r1, v2, r2


@pytest.mark.parametrize("precision", [1, 0])
def test_static_scratch_matches_run_twice(precision):
    import torch
    import paper_2007_04881_amd as D

    big = voronoi_mesh(6000, 91, lloyd=0, p=2)
    small = voronoi_mesh(700, 92, lloyd=1, p=1)
    small = small.with_degrees(np.random.default_rng(12).integers(1, 5, small.n_cells))
    ctx = D.Context(0)
    for mesh in (big, small):
        print(f"[case] run_static cells={mesh.n_cells} prec={precision}", flush=True)
        v1, r1, v2, r2 = _both(ctx, mesh, DAR, precision)
        assert torch.equal(v1, v2) and torch.equal(r1, r2)
        pat = oracle.pattern(mesh)
        rp, ci, vp, dp = ctx.pattern_tensors()
        torch.cuda.synchronize()
        assert np.array_equal(rp.cpu().numpy(), pat.row_ptr) and np.array_equal(ci.cpu().numpy(), pat.col_idx)
        assert np.array_equal(vp.cpu().numpy(), pat.val_ptr) and np.array_equal(dp.cpu().numpy(), pat.dof_ptr)
        ov, orhs = oracle.assemble(mesh, oracle_problem(DAR), pat=pat)
        g = dict(vals=v2.double().cpu().numpy(), rhs=r2.double().cpu().numpy())
        eb, er = block_errors(g, ov, orhs, pat)
        print(f"       worst block {eb:.3e}  worst rhs row {er:.3e}", flush=True)
        assert eb <= TOL[precision] and er <= TOL[precision]
    # the step's own timing re-launch needs a regular step first
    with pytest.raises(D.DgpError) as e:
        ctx.time_kernels(1)
    assert e.value.status == -6
    ctx.close()


def test_static_scratch_polyhedra_then_polygons():
    """3D (whose limit flag in the array must be cleared) then a smaller 2D mesh."""
    import torch
    import paper_2007_04881_amd as D

    ctx = D.Context(0)
    print("[case] run_static 3D", flush=True)
    v1, r1, v2, r2 = _both(ctx, agglomerated_cube(8, 70, 2033, p=2), DAR3, 1)
    assert torch.equal(v1, v2) and torch.equal(r1, r2)
    print("[case] run_static 2D after 3D", flush=True)
    v1, r1, v2, r2 = _both(ctx, voronoi_mesh(300, 93, lloyd=1, p=3), DAR, 0)
    assert torch.equal(v1, v2) and torch.equal(r1, r2)
    ctx.close()


def test_static_scratch_limit():
    """360,000 cells need about 80 MB of scratch: refused, nothing written."""
    import torch
    import paper_2007_04881_amd as D

    ctx = D.Context(0)
    ctx.upload(cartesian_mesh(600, 600, p=1))
    ctx.pattern()
    v, r = ctx.outputs(1)
    v.fill_(7.0)
    with pytest.raises(D.DgpError) as e:
        ctx.run_static(DAR, 1, v, r)
    assert e.value.status == -3 and "static" in str(e.value)
    torch.cuda.synchronize()
    assert bool((v == 7.0).all())
    ctx.close()
