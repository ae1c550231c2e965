"""GPU parity of the reduced volume rules against the FP64 oracle (oracle.learned).

* training polygons: Philox stream, normalisation, features and moments;
* element data of a mesh: features (exact), moments;
* the network: forward pass and loss gradient of the FP32 matrix-core kernels
  against the oracle's FP64 forward and hand-written backward pass, and Adam;
* the fitted rules: every accepted rule is re-judged by the oracle's moments;
* assembly with accepted rules against the oracle's plain assembly (constant
  coefficients: every volume integrand has degree <= 6, so the reduced rule
  integrates it to the residual of its moments; variable a: the difference is
  quadrature error and falls like h^7).
Several rules fit the same moments: nodes and weights are never compared.
"""

import numpy as np
import pytest

import oracle
from meshgen import voronoi_mesh
from oracle import learned as L
from tests.parity import block_errors, check_pattern, oracle_problem

pytestmark = pytest.mark.gpu

SEED = 2007048815
POISSON = dict(a0=1.0, a1=0.0, b=(0.0, 0.0, 0.0), c=0.0, c_sigma=10.0, u="sin")
CONST_DAR = dict(a0=1.3, a1=0.0, b=(1.0, 0.5, 0.0), c=1.0, c_sigma=10.0, u="sin")


def _ctx():
    import paper_2007_04881_amd as D
    return D.Context(0)


def _cell_xy(m, c):
    ids = m.cell_vtx[m.cell_ptr[c]:m.cell_ptr[c + 1]]
    return np.stack([m.x[ids], m.y[ids]], 1)


def test_training_polygons_match_oracle():
    print("[case] training polygons 0..299", flush=True)
    ctx = _ctx()
    feat, f64, mom, area = ctx.train_polygons(SEED, 0, 300, with_f64=True)
    f64, mom, area, feat = f64.cpu().numpy(), mom.cpu().numpy(), area.cpu().numpy(), feat.cpu().numpy()
    for i in range(300):
        v = L.random_polygon(i, SEED)
        x = L.features(v)
        m = v.shape[0]
        assert np.array_equal(f64[i, 24:], x[24:]), i           # vertex count: exact
        assert np.abs(f64[i, :24] - x[:24]).max() <= 4e-15, i    # sin/cos differ by ulps
        assert np.abs(feat[i] - x.astype(np.float32)).max() <= 1e-6
        M = L.polygon_moments(v)
        assert np.abs(mom[i] - M).max() <= 1e-13 * abs(M[0]), i
        assert abs(area[i] - L.polygon_area(v)) <= 1e-14 * area[i]
        assert m == int(x[24:].sum())
    # a later window of the same stream gives the same polygons
    _, g2, _, _ = ctx.train_polygons(SEED, 250, 10, with_f64=True)
    assert np.array_equal(g2.cpu().numpy(), f64[250:260])
    ctx.close()


def _mesh_with_rules(n, seed, p, init, iters=8):
    import paper_2007_04881_amd as D
    m = voronoi_mesh(n, seed, lloyd=1, p=p)
    ctx = _ctx()
    ctx.upload(m)
    ctx.pattern()
    st = ctx.qrule_build(init, iters, 1e-10)
    return m, ctx, st


def test_element_data_and_template_rules():
    import paper_2007_04881_amd as D
    print("[case] element data + template rules, 700 cells", flush=True)
    m, ctx, st = _mesh_with_rules(700, 91, 3, D.INIT_TEMPLATE)
    feat, mom, area = (t.cpu().numpy() for t in ctx.qrule_cell_data())
    nodes, w, ok, res, it = (t.cpu().numpy() for t in ctx.qrule_get())
    nv = np.diff(m.cell_ptr)
    assert st.n_cells == m.n_cells and st.n_eligible == int((nv <= 12).sum())
    assert st.n_accepted == int(ok.sum())
    assert st.n_accepted >= 0.95 * st.n_eligible, (st.n_accepted, st.n_eligible)
    worst = 0.0
    for c in range(m.n_cells):
        if nv[c] > 12:
            assert ok[c] == 0
            continue
        v = L.normalise(_cell_xy(m, c))
        x = L.features(v)
        assert np.array_equal(feat[c], x.astype(np.float32)), c
        M = L.polygon_moments(v)
        A = L.polygon_area(v)
        assert np.abs(mom[c] - M).max() <= 1e-13 * A
        assert abs(area[c] - A) <= 1e-14 * A
        if ok[c]:
            r = L.residual(nodes[c], w[c], M, A)   # re-judged by the oracle
            worst = max(worst, r)
            assert r <= 1e-10, (c, r, res[c])
    print(f"       accepted {st.n_accepted}/{st.n_eligible}, worst re-judged residual {worst:.2e}", flush=True)
    ctx.close()


def _random_blob(seed):
    return L.flatten(L.init_params(seed)).astype(np.float32)


def test_network_forward_matches_oracle():
    import torch
    print("[case] network forward, 333 rows", flush=True)
    polys = [L.random_polygon(i, 7) for i in range(333)]
    X = np.stack([L.features(v) for v in polys]).astype(np.float32)
    A = np.array([L.polygon_area(v) for v in polys])
    blob = _random_blob(3)
    ctx = _ctx()
    out = ctx.mlp_forward(torch.from_numpy(blob).cuda(), torch.from_numpy(X).cuda()).cpu().numpy()
    params = L.unflatten(blob.astype(np.float64))
    _, _, (_, _, ref, _) = L.forward(params, X.astype(np.float64), A)
    err = np.abs(out - ref).max() / np.abs(ref).max()
    print(f"       max relative error {err:.2e}", flush=True)
    assert err <= 1e-5
    ctx.close()


def test_loss_gradient_and_adam_match_oracle():
    import torch
    # 2,100 rows: the weight gradients take the split-K path (partials summed in order)
    print("[case] loss gradient, 2100 rows", flush=True)
    polys = [L.random_polygon(i, 8) for i in range(2100)]
    X = np.stack([L.features(v) for v in polys]).astype(np.float32).astype(np.float64)
    A = np.array([L.polygon_area(v) for v in polys])
    M = np.stack([L.polygon_moments(v) for v in polys])
    blob = _random_blob(5)
    ctx = _ctx()
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g, loss = ctx.mlp_loss_grad(dev(blob), dev(X.astype(np.float32)), dev(M), dev(A))
    g = g.cpu().numpy().astype(np.float64)
    params = L.unflatten(blob.astype(np.float64))
    ref = L.flatten(L.backward(params, X, M, A))
    lref = L.loss(params, X, M, A)
    assert abs(loss.item() / len(polys) - lref) <= 1e-5 * lref
    o = 0
    for k, p in enumerate(params):
        sl = slice(o, o + p.size)
        o += p.size
        rel = np.linalg.norm(g[sl] - ref[sl]) / np.linalg.norm(ref[sl])
        assert rel <= 1e-4, (k, rel)
    # one Adam step on the device against the oracle's
    p_d, m_d, v_d = dev(blob.copy()), torch.zeros(blob.size).cuda(), torch.zeros(blob.size).cuda()
    gd = dev(g.astype(np.float32))
    for t in (1, 2):
        ctx.adam_step(p_d, gd, m_d, v_d, t, lr=1e-3)
    p_ref, m_ref, v_ref = blob.astype(np.float64), np.zeros(blob.size), np.zeros(blob.size)
    g32 = g.astype(np.float32).astype(np.float64)
    for t in (1, 2):
        p_ref, m_ref, v_ref = L.adam_step(p_ref, g32, m_ref, v_ref, t, lr=1e-3)
    assert np.abs(p_d.cpu().numpy() - p_ref).max() <= 1e-6
    ctx.close()


@pytest.mark.parametrize("p,params,precision", [(3, POISSON, 0), (3, POISSON, 1), (2, CONST_DAR, 0),
                                                 (2, CONST_DAR, 1), (3, CONST_DAR, 1)])
def test_reduced_assembly_matches_plain_oracle(p, params, precision):
    import torch
    import paper_2007_04881_amd as D
    print(f"[case] reduced assembly p={p} prec={precision} {params['b']}", flush=True)
    m, ctx, st = _mesh_with_rules(600, 92, p, D.INIT_TEMPLATE)
    assert st.n_accepted >= 0.95 * st.n_eligible
    vals, rhs = ctx.outputs(precision)
    ctx.assemble(params, precision, vals, rhs, rule_mode=D.RULE_REDUCED)
    vp, rp_ = ctx.outputs(precision)
    ctx.assemble(params, precision, vp, rp_, rule_mode=D.RULE_PLAIN)
    rp, ci, vpt, dp = ctx.pattern_tensors()
    torch.cuda.synchronize()
    g = dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val_ptr=vpt.cpu().numpy(),
             dof_ptr=dp.cpu().numpy(), vals=vals.double().cpu().numpy(), rhs=rhs.double().cpu().numpy(),
             info=(ctx.info.n_rows, ctx.info.nnzb, ctx.info.n_vals, ctx.info.n_dofs))
    pat = oracle.pattern(m)
    check_pattern(g, pat)
    ov, orhs = oracle.assemble(m, oracle_problem(params), pat=pat)
    eb, er = block_errors(g, ov, orhs, pat)
    tol = 1e-8 if precision == 0 else 1e-5
    print(f"       worst block {eb:.3e}  worst rhs row {er:.3e}", flush=True)
    assert eb <= tol and er <= (1e-12 if precision == 0 else 1e-5)
    # the reduced rule was used: the diagonal blocks differ from the plain ones by rounding only
    if precision == 0:
        d = np.abs(g["vals"] - vp.double().cpu().numpy()).max()
        assert 0.0 < d <= 1e-8 * np.abs(ov).max()
    ctx.close()


def test_reduced_assembly_full_size_sampled():
    """The 262,144-cell p = 3 workload with template-initialised rules, FP32,
    sampled rows against the oracle's plain assembly."""
    import torch
    import paper_2007_04881_amd as D
    from meshgen import config_mesh, problem_params
    m = config_mesh(5)
    params = problem_params(5)
    print(f"[case] reduced assembly, {m.n_cells} cells", flush=True)
    ctx = _ctx()
    ctx.upload(m)
    ctx.pattern()
    st = ctx.qrule_build(D.INIT_TEMPLATE, 8, 1e-10)
    assert st.n_accepted >= 0.99 * st.n_eligible
    vals, rhs = ctx.outputs(D.F32)
    ctx.assemble(params, D.F32, vals, rhs, rule_mode=D.RULE_REDUCED)
    rp, ci, vp, dp = ctx.pattern_tensors()
    torch.cuda.synchronize()
    g = dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val_ptr=vp.cpu().numpy(),
             dof_ptr=dp.cpu().numpy(), vals=vals.double().cpu().numpy(), rhs=rhs.double().cpu().numpy(),
             info=(ctx.info.n_rows, ctx.info.nnzb, ctx.info.n_vals, ctx.info.n_dofs))
    ctx.close()
    pat = oracle.pattern(m)
    check_pattern(g, pat)
    rows = np.unique(np.concatenate([[0, m.n_cells - 1], np.random.default_rng(12).integers(0, m.n_cells, 300)]))
    ov, orhs = oracle.assemble(m, oracle_problem(params), rows=rows, pat=pat)
    eb, er = block_errors(g, ov, orhs, pat, rows=rows)
    print(f"       worst block {eb:.3e}  worst rhs row {er:.3e} over {len(rows)} rows", flush=True)
    assert eb <= 1e-5 and er <= 1e-5


def _diag_offdiag_errors(g, ov, pat):
    """Worst relative Frobenius error of the diagonal blocks and of the others."""
    worst = [0.0, 0.0]
    for r in range(len(pat.row_ptr) - 1):
        for k in range(pat.row_ptr[r], pat.row_ptr[r + 1]):
            s0, s1 = pat.val_ptr[k], pat.val_ptr[k + 1]
            ref = ov[s0:s1]
            e = np.linalg.norm(g["vals"][s0:s1] - ref) / max(np.linalg.norm(ref), 1e-300)
            d = 0 if pat.col_idx[k] == r else 1
            worst[d] = max(worst[d], e)
    return worst


def test_reduced_rules_with_variable_diffusion_converge():
    """With a(x) = 1 + 0.5 sin(2 pi x) cos(2 pi y) neither rule integrates
    a grad phi_i . grad phi_j exactly: the reduced assembly differs from the
    oracle's plain one by the two quadrature errors.  Both rules are exact to
    degree 6 and grad phi_i . grad phi_j has degree 2 (p - 1) = 4, so a's
    Taylor terms up to degree 2 are integrated exactly and the difference,
    relative to the block, falls like h^3 (8x per halving of h; at least 5x
    is required, pre-asymptotic): checked on meshes of 800 and 3,200 cells.
    The off-diagonal blocks and the load do not use the volume rule and match
    the oracle to rounding."""
    import torch
    import paper_2007_04881_amd as D
    var_a = dict(POISSON, a1=0.5)
    errs = []
    for n in (800, 3200):
        print(f"[case] reduced rules with variable a, {n} cells p = 3", flush=True)
        m, ctx, st = _mesh_with_rules(n, 96, 3, D.INIT_TEMPLATE)
        assert st.n_accepted >= 0.95 * st.n_eligible
        vals, rhs = ctx.outputs(D.F64)
        ctx.assemble(var_a, D.F64, vals, rhs, rule_mode=D.RULE_REDUCED)
        rp, ci, vp, dp = ctx.pattern_tensors()
        torch.cuda.synchronize()
        g = dict(row_ptr=rp.cpu().numpy(), col_idx=ci.cpu().numpy(), val_ptr=vp.cpu().numpy(),
                 dof_ptr=dp.cpu().numpy(), vals=vals.double().cpu().numpy(), rhs=rhs.double().cpu().numpy(),
                 info=(ctx.info.n_rows, ctx.info.nnzb, ctx.info.n_vals, ctx.info.n_dofs))
        ctx.close()
        pat = oracle.pattern(m)
        check_pattern(g, pat)
        ov, orhs = oracle.assemble(m, oracle_problem(var_a), pat=pat)
        ed, eo = _diag_offdiag_errors(g, ov, pat)
        _, er = block_errors(g, ov, orhs, pat)
        print(f"       diagonal blocks {ed:.3e}  off-diagonal {eo:.3e}  rhs rows {er:.3e}", flush=True)
        assert eo <= 1e-12 and er <= 1e-12
        errs.append(ed)
    assert 0.0 < errs[0] <= 1e-4
    assert errs[1] <= errs[0] / 5.0, errs


def test_training_lowers_the_loss_and_network_rules_are_accepted():
    import paper_2007_04881_amd as D
    print("[case] training 20000 polygons x 4 epochs", flush=True)
    ctx = _ctx()
    params, losses, st = ctx.mlp_train(20000, SEED, init_seed=1, epochs=4, batch=1024, lr=2e-3)
    print(f"       epoch losses {losses.tolist()} steps {st.steps} {st.ms:.0f} ms", flush=True)
    assert np.all(np.isfinite(losses)) and losses[-1] < 0.5 * losses[0]
    assert st.steps == 4 * 20
    m = voronoi_mesh(400, 93, lloyd=1, p=3)
    ctx.upload(m)
    ctx.pattern()
    s = ctx.qrule_build(D.INIT_NETWORK, 8, 1e-10)
    assert s.n_accepted >= 0.9 * s.n_eligible, (s.n_accepted, s.n_eligible)
    # the trained parameters reloaded give the same rules
    nodes1 = ctx.qrule_get()[0].cpu().numpy()
    ctx.mlp_load(params)
    ctx.qrule_build(D.INIT_NETWORK, 8, 1e-10)
    assert np.array_equal(nodes1, ctx.qrule_get()[0].cpu().numpy())
    ctx.close()


def test_reduced_rule_errors():
    import paper_2007_04881_amd as D
    ctx = _ctx()
    m = voronoi_mesh(60, 94, lloyd=1, p=3)
    ctx.upload(m)
    ctx.pattern()
    v, r = ctx.outputs(D.F64)
    with pytest.raises(D.DgpError) as e:
        ctx.assemble(POISSON, D.F64, v, r, rule_mode=D.RULE_REDUCED)
    assert e.value.status == -6
    with pytest.raises(D.DgpError) as e:
        ctx.qrule_build(D.INIT_NETWORK, 8, 1e-10)
    assert e.value.status == -6
    ctx.qrule_build(D.INIT_TEMPLATE, 8, 1e-10)
    with pytest.raises(D.DgpError) as e:
        ctx.mlp_load(np.zeros(10, np.float32))
    assert e.value.status == -1
    ctx.close()


def test_network_start_gains_over_the_template():
    """What the trained network adds: on the same mesh, rules built from the
    network start (each element from the network's or the template's rule,
    whichever has the smaller moment residual, at most 6 steps; elements not
    accepted then are refined again from the template, and their steps count
    both attempts) are accepted at least as often as from the template alone
    and need fewer refinement steps on average; every accepted network-start
    rule is re-judged by the oracle's moments."""
    import paper_2007_04881_amd as D
    print("[case] network vs template starts, 3000 cells p = 3", flush=True)
    ctx = _ctx()
    ctx.mlp_train(300000, SEED, init_seed=1, epochs=20, batch=2048, lr=2e-3)
    m = voronoi_mesh(3000, 95, lloyd=0, p=3)
    ctx.upload(m)
    ctx.pattern()

    def mean_steps(st):
        return sum(k * st.iters_hist[k] for k in range(16)) / max(st.n_accepted, 1)

    t = ctx.qrule_build(D.INIT_TEMPLATE, 8, 1e-10)
    n = ctx.qrule_build(D.INIT_NETWORK, 8, 1e-10)
    print(f"       template: accepted {t.n_accepted}/{t.n_eligible}, mean steps {mean_steps(t):.2f}", flush=True)
    print(f"       network:  accepted {n.n_accepted}/{n.n_eligible}, mean steps {mean_steps(n):.2f}, "
          f"network starts {n.n_start_network}, retried {n.n_retried} ({n.n_retry_accepted} accepted)", flush=True)
    assert n.n_accepted >= t.n_accepted
    assert mean_steps(n) < mean_steps(t)
    nodes, w, ok, res, it = (t_.cpu().numpy() for t_ in ctx.qrule_get())
    nv = np.diff(m.cell_ptr)
    for c in np.nonzero(ok)[0]:
        v = L.normalise(_cell_xy(m, c))
        assert nv[c] <= 12
        r = L.residual(nodes[c], w[c], L.polygon_moments(v), L.polygon_area(v))
        assert r <= 1e-10, (c, r)
    ctx.close()
