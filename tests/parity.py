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


def block_errors(g, vals_ref, rhs_ref, pat, rows=None, where=None):
    """Largest per-block relative Frobenius error of the matrix and per-row of the
    right-hand side (numpy segment sums over val_ptr / dof_ptr).  ``rows``
    restricts the check to those block rows (the oracle leaves the others NaN).
    ``where`` (a dict) receives the row and block of the worst matrix error."""
    n_rows = len(pat.row_ptr) - 1
    rows = np.arange(n_rows) if rows is None else np.unique(np.asarray(rows, dtype=np.int64))
    # blocks of the selected rows
    cnt = pat.row_ptr[rows + 1] - pat.row_ptr[rows]
    blk = np.repeat(pat.row_ptr[rows], cnt) + (np.arange(cnt.sum()) - np.repeat(np.cumsum(cnt) - cnt, cnt))
    brow = np.repeat(rows, cnt)
    b0, b1 = pat.val_ptr[blk], pat.val_ptr[blk + 1]
    worst_b = _segment_worst(g["vals"], vals_ref, b0, b1, what="block", where=where, ids=(brow, blk))
    d0, d1 = pat.dof_ptr[rows], pat.dof_ptr[rows + 1]
    rw = {}
    worst_r = _segment_worst(g["rhs"], rhs_ref, d0, d1, what="load", rows_for_abs=True, where=rw,
                             ids=(rows, rows))
    if where is not None:
        where.update(rhs_row=rw["row"])
    return worst_b, worst_r


def _segment_worst(got, ref, s0, s1, what, where=None, ids=None, rows_for_abs=False):
    lens = s1 - s0
    assert (lens > 0).all()
    idx = np.repeat(s0, lens) + (np.arange(lens.sum()) - np.repeat(np.cumsum(lens) - lens, lens))
    r = ref[idx]
    d = got[idx] - r
    assert not np.isnan(r).any(), f"oracle {what} missing"
    assert not np.isnan(d).any(), f"{what} is NaN"
    starts = np.cumsum(lens) - lens
    nrm = np.sqrt(np.add.reduceat(r * r, starts))
    err = np.sqrt(np.add.reduceat(d * d, starts))
    if rows_for_abs:
        # a row whose load vanishes (g_D = 0, f ~ 0) is compared in absolute terms
        scale = np.abs(r).max()
        rel = np.where(nrm > 1e-10 * scale, err / np.where(nrm > 0, nrm, 1.0), err / scale)
    else:
        rel = np.where(nrm > 0, err / np.where(nrm > 0, nrm, 1.0), err)
    k = int(np.argmax(rel))
    if where is not None and ids is not None:
        where.update(row=int(ids[0][k]), block=int(ids[1][k]), err=float(rel[k]))
    return float(rel[k])


def oracle_problem(params):
    return oracle.Problem.from_params(params)
