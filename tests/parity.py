"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI and
compare block-CSR output with the oracle block by block."""

import numpy as np

import oracle

TOL = {0: 1e-12, 1: 1e-5}  # FP64, FP32: per block ||dB||_F <= tol ||B_oracle||_F


def gpu_assemble(mesh, params, precision, full_path=False):
    import torch
    import paper_2007_04881_amd as D
    ctx = D.Context(0)
    ctx.upload(mesh)
    info = ctx.pattern()
    vals, rhs = ctx.outputs(precision)
    vals.fill_(float("nan"))
    rhs.fill_(float("nan"))
    if full_path:
        ctx.run(params, precision, vals, rhs)
    else:
        ctx.assemble(params, precision, vals, rhs)
    rp, ci, vp, dp = ctx.pattern_tensors()
    torch.cuda.synchronize()
    out = dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val_ptr=vp.cpu().numpy(),
               dof_ptr=dp.cpu().numpy(), vals=vals.double().cpu().numpy(), rhs=rhs.double().cpu().numpy(),
               info=(info.n_rows, info.nnzb, info.n_vals, info.n_dofs))
    ctx.close()
    return out


def check_pattern(g, pat):
    assert np.array_equal(g["row_ptr"], pat.row_ptr)
    assert np.array_equal(g["col_idx"], pat.col_idx)
    assert np.array_equal(g["val_ptr"], pat.val_ptr)
    assert np.array_equal(g["dof_ptr"], pat.dof_ptr)
    assert g["info"][1:] == (pat.nnzb, pat.n_vals, pat.n_dofs)


def block_errors(g, vals_ref, rhs_ref, pat, rows=None):
    """Largest per-block relative Frobenius error of the matrix and per-row of the rhs."""
    rows = range(len(pat.row_ptr) - 1) if rows is None else rows
    worst_b = 0.0
    worst_r = 0.0
    # with sampled rows the oracle leaves the other rows NaN: scale by the sampled ones
    rhs_scale = max(np.abs(rhs_ref[pat.dof_ptr[r]:pat.dof_ptr[r + 1]]).max() for r in rows)
    for r in rows:
        for k in range(pat.row_ptr[r], pat.row_ptr[r + 1]):
            sl = slice(pat.val_ptr[k], pat.val_ptr[k + 1])
            ref = vals_ref[sl]
            nrm = np.linalg.norm(ref)
            err = np.linalg.norm(g["vals"][sl] - ref)
            assert not np.isnan(err), f"block {k} of row {r} is NaN"
            worst_b = max(worst_b, err / nrm if nrm > 0 else err)
        sl = slice(pat.dof_ptr[r], pat.dof_ptr[r + 1])
        ref = rhs_ref[sl]
        assert not np.isnan(ref).any(), f"oracle load of row {r} missing"
        nrm = np.linalg.norm(ref)
        err = np.linalg.norm(g["rhs"][sl] - ref)
        assert not np.isnan(err), f"load of row {r} is NaN"
        # a row whose load vanishes (g_D = 0, f ~ 0) is compared in absolute terms
        worst_r = max(worst_r, err / nrm if nrm > 1e-10 * rhs_scale else err / rhs_scale)
    return worst_b, worst_r


def oracle_problem(params):
    return oracle.Problem.from_params(params)
