"""Pins of the oracle's space-time slab assembly (Section 2.3, equation
spacetime_dg) on prisms I_n x kappa over 2D polygonal meshes.

* Consistency: with constant coefficients and u = u_s(x, y) T(t) in the
  space-time polynomial space (u_s of degree <= 1 and T linear, or u_s
  quadratic and T constant), the exact coefficients c of u on every prism (its
  projection on the bounding box, where the basis is orthonormal) satisfy
  A c = F: the time derivative, the time jump with the exact u(t0), the
  spatial SIPG terms and the boundary data are all reproduced.
* Time terms alone (a = b = c = 0): integration by parts in time gives
  A + A^T = M(t1) + M(t0), the mass matrices of the prism's top and bottom,
  computed here by the divergence theorem on the polygon.
* Spatial terms: on the basis functions constant in time the slab matrix is
  the 2D matrix of the same mesh (same penalty) plus the bottom mass matrix
  divided by tau.
"""

import numpy as np
import pytest

import oracle
from meshgen import voronoi_mesh
from tests import polyexact as PE


def _coeffs_on_boxes(m, pat, u, t0, t1, p_of):
    """Coefficients of u(x, y, t) in each prism's basis: integrals of u phi_i over
    the bounding box (orthonormal basis there), by a tensor Gauss rule."""
    geo = oracle.geometry(m)
    xg, wg = np.polynomial.legendre.leggauss(8)
    c = np.zeros(pat.n_dofs)
    for r in range(m.n_cells):
        lo = np.array([geo["lo"][r, 0], geo["lo"][r, 1], t0])
        hi = np.array([geo["hi"][r, 0], geo["hi"][r, 1], t1])
        p = p_of(r)
        acc = 0.0
        for i, (a, wa) in enumerate(zip(xg, wg)):
            for b, wb in zip(xg, wg):
                for cc, wc in zip(xg, wg):
                    x = lo + (np.array([a, b, cc]) + 1) * (hi - lo) / 2
                    phi, _ = oracle.basis(3, p, lo, hi, x)
                    acc = acc + wa * wb * wc * u(*x) * phi
        c[pat.dof_ptr[r]:pat.dof_ptr[r + 1]] = acc * np.prod(hi - lo) / 8
    return c


@pytest.mark.parametrize("p,us,tau", [
    (1, (1.0, 2.0, -1.0, 0, 0, 0, 0, 0, 0, 0), (0.0, 0.0)),
    (2, (1.0, 2.0, -1.0, 0, 0, 0, 0, 0, 0, 0), (0.5, 0.0)),
    (2, (1.0, 2.0, -1.0, 0, 0.7, -0.5, 0, 1.0, 0, 0), (0.0, 0.0)),
    (3, (1.0, 2.0, -1.0, 0, 0.7, -0.5, 0, 1.0, 0, 0), (0.5, 0.0)),
])
def test_spacetime_reproduces_polynomials(p, us, tau):
    m = voronoi_mesh(25, 41, lloyd=2, p=p)
    prob = oracle.Problem(a0=1.3, a1=0.0, b=(0.4, -0.7, 0.0), c=0.9, u_kind=oracle.U_POLY, u_poly=us)
    t0, t1 = 0.3, 0.45
    pat = oracle.pattern_st(m)
    A, F = oracle.assemble_st(m, prob, t0, t1, tau=tau, pat=pat)
    T = lambda t: 1.0 + tau[0] * t + tau[1] * t * t
    u = lambda x, y, t: (us[0] + us[1] * x + us[2] * y + us[4] * x * x + us[5] * y * y + us[7] * x * y) * T(t)
    c = _coeffs_on_boxes(m, pat, u, t0, t1, lambda r: p)
    Ac = np.zeros(pat.n_dofs)
    for r in range(m.n_cells):
        nr = pat.dof_ptr[r + 1] - pat.dof_ptr[r]
        for k in range(pat.row_ptr[r], pat.row_ptr[r + 1]):
            cc = pat.col_idx[k]
            nc = pat.dof_ptr[cc + 1] - pat.dof_ptr[cc]
            blk = A[pat.val_ptr[k]:pat.val_ptr[k + 1]].reshape(nr, nc)
            Ac[pat.dof_ptr[r]:pat.dof_ptr[r + 1]] += blk @ c[pat.dof_ptr[cc]:pat.dof_ptr[cc + 1]]
    assert np.abs(Ac - F).max() <= 1e-11 * np.abs(F).max(), np.abs(Ac - F).max() / np.abs(F).max()


def _bottom_top_mass(m, r, p, t0, t1, t):
    """M(t)_ij = int_kappa phi_i(., t) phi_j(., t), phi_(a,b,c) = (2D basis
    function (a, b) on the cell's box) times sqrt((2c+1)/tau) P_c on [t0, t1],
    the polygon integrals by the divergence theorem."""
    geo = oracle.geometry(m)
    lo, hi = geo["lo"][r, :2], geo["hi"][r, :2]
    ids = m.cell_vtx[m.cell_ptr[r]:m.cell_ptr[r + 1]]
    xy_box, J = PE.to_box(np.stack([m.x[ids], m.y[ids]], 1), lo, hi)
    sp = dict(zip(PE.basis_exponents(2, p), PE.basis_polys_2d(p, lo, hi)))
    exps = PE.basis_exponents(3, p)
    tau = t1 - t0
    s = 2 * (t - t0) / tau - 1
    Lt = [np.polynomial.legendre.legval(s, [0] * c + [1]) * np.sqrt((2 * c + 1) / tau) for c in range(p + 1)]
    M = np.zeros((len(exps), len(exps)))
    for i, (a1, b1, c1) in enumerate(exps):
        for j, (a2, b2, c2) in enumerate(exps):
            M[i, j] = J * PE.polygon_integral(xy_box, PE.mul(sp[(a1, b1)], sp[(a2, b2)])) * Lt[c1] * Lt[c2]
    return M


@pytest.mark.parametrize("p", [1, 2, 3])
def test_time_terms_integrate_by_parts(p):
    m = voronoi_mesh(12, 43, lloyd=2, p=p)
    prob = oracle.Problem(a0=0.0, a1=0.0, b=(0.0, 0.0, 0.0), c=0.0)
    t0, t1 = 0.2, 0.5
    pat = oracle.pattern_st(m)
    A, _ = oracle.assemble_st(m, prob, t0, t1, pat=pat)
    for r in range(m.n_cells):
        nb = pat.dof_ptr[r + 1] - pat.dof_ptr[r]
        for k in range(pat.row_ptr[r], pat.row_ptr[r + 1]):
            blk = A[pat.val_ptr[k]:pat.val_ptr[k + 1]]
            if pat.col_idx[k] != r:
                assert np.abs(blk).max() == 0.0  # a = b = 0: no face terms
                continue
            D = blk.reshape(nb, nb)
            ref = _bottom_top_mass(m, r, p, t0, t1, t1) + _bottom_top_mass(m, r, p, t0, t1, t0)
            assert np.abs(D + D.T - ref).max() <= 1e-12 * np.abs(ref).max(), r


@pytest.mark.parametrize("p", [1, 2])
def test_time_constant_functions_see_the_2d_matrix(p):
    """Rows and columns of basis functions with time exponent 0: the 2D matrix
    (phi_st = phi_2d / sqrt(tau) there, integrated over tau) plus M_2D / tau
    from the time jump; the penalty is fixed so both sides use the same sigma."""
    m = voronoi_mesh(20, 44, lloyd=1, p=p)
    prob = oracle.Problem(a0=1.2, a1=0.4, b=(0.8, -0.3, 0.0), c=0.7, sigma_override=37.0)
    t0, t1 = 0.1, 0.35
    tau = t1 - t0
    pst = oracle.pattern_st(m)
    A3, _ = oracle.assemble_st(m, prob, t0, t1, pat=pst)
    p2 = oracle.pattern(m)
    A2, _ = oracle.assemble(m, prob, pat=p2)
    M2, _ = oracle.assemble(m, oracle.Problem(a0=0.0, c=1.0, term_mask=oracle.T_VOLUME), pat=p2)
    exps = PE.basis_exponents(3, p)
    sel = [i for i, e in enumerate(exps) if e[2] == 0]  # time exponent 0, in 2D order
    nb3, nb2 = len(exps), len(sel)
    for r in range(m.n_cells):
        for k in range(pst.row_ptr[r], pst.row_ptr[r + 1]):
            c = pst.col_idx[k]
            B3 = A3[pst.val_ptr[k]:pst.val_ptr[k + 1]].reshape(nb3, nb3)[np.ix_(sel, sel)]
            B2 = A2[p2.val_ptr[k]:p2.val_ptr[k + 1]].reshape(nb2, nb2)
            ref = B2 + (M2[p2.val_ptr[k]:p2.val_ptr[k + 1]].reshape(nb2, nb2) / tau if c == r else 0.0)
            assert np.abs(B3 - ref).max() <= 1e-12 * np.abs(ref).max(), (r, c)


def test_time_jump_reads_the_previous_slab():
    """(U_{n-1}^-, W^+): with U_{n-1} the exact coefficients of a space-time
    polynomial u on the previous slab's prisms, the load equals the one formed
    from u(t0) itself; a perturbed U_{n-1} changes only the bottom term."""
    p, us, tau = 2, (1.0, 2.0, -1.0, 0, 0, 0, 0, 0, 0, 0), (0.5, 0.0)
    m = voronoi_mesh(15, 45, lloyd=2, p=p)
    prob = oracle.Problem(a0=1.3, b=(0.4, -0.7, 0.0), c=0.9, u_kind=oracle.U_POLY, u_poly=us)
    tp0, t0, t1 = 0.1, 0.3, 0.45
    pat = oracle.pattern_st(m)
    T = lambda t: 1.0 + tau[0] * t
    u = lambda x, y, t: (us[0] + us[1] * x + us[2] * y) * T(t)
    prev = _coeffs_on_boxes(m, pat, u, tp0, t0, lambda r: p)
    _, F_exact = oracle.assemble_st(m, prob, t0, t1, tau=tau, pat=pat)
    _, F_prev = oracle.assemble_st(m, prob, t0, t1, tau=tau, prev=prev, tp0=tp0, pat=pat)
    assert np.abs(F_prev - F_exact).max() <= 1e-12 * np.abs(F_exact).max()
    bumped = prev.copy()
    bumped[pat.dof_ptr[4]] += 1.0  # the constant mode of element 4 on the previous slab
    _, F_b = oracle.assemble_st(m, prob, t0, t1, tau=tau, prev=bumped, tp0=tp0, pat=pat)
    changed = np.nonzero(np.abs(F_b - F_prev) > 1e-12 * np.abs(F_prev).max())[0]
    assert changed.min() >= pat.dof_ptr[4] and changed.max() < pat.dof_ptr[5]
