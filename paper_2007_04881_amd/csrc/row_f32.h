// 2D SIPG rows in FP32 with the plain (sub-triangulation) rules for rows of
// degree p <= 2, on meshes of one degree or (MX) among neighbours of any
// degree: the same terms and quadrature as the general row kernel (one wave
// per element row; fan sub-triangle points for the element block and the
// load, the Gauss points of every edge, grouped per neighbour, for the face
// terms of eq. dg-bilinear and dg-linear), laid out for register economy:
//  * what depends only on the element's vertices and edges is formed once per
//    row in the lanes that hold the loop: each vertex's box coordinates and
//    offset from the box centre and each fan sub-triangle's area (FP64,
//    rounded once to FP32), each edge's length, outward normal, penalty and
//    upwind weight, and the neighbour's box coordinates of the edge's ends;
//  * a point's lane fetches its vertices' or its edge's values (ds_bpermute)
//    and forms its box coordinates and coefficients in FP32; the manufactured
//    data (a, f, boundary values) stay FP64 (sin / cos by angle addition from
//    the box centre), for the sine solution only (problems with the
//    polynomial solution take the general row kernel: its coefficients would
//    hold scalar registers through the whole row);
//  * a transposed per-wave LDS table holds, per basis function, the test
//    terms of every point of the pass (columns 3 lane + a), then the
//    neighbour's trial terms (the cross blocks of every edge group of the pass
//    at once, one entry per lane and round; MX: in chunks of trial rows),
//    then the row's own trial terms and the load terms (p = 2: the element
//    block and load as 4 x 4 x 1 matrix products in 16 blocks; p = 1 keeps
//    rank-3 register updates into 12 accumulators and a reduce-scatter);
//  * sums across passes (rows of more than 64 points, edges shared twice
//    with one neighbour) are compensated (TwoSum).
// Included by the FP32 row kernels and by the single persistent launch over
// every degree bin, which must compute the rows the same way.
#pragma once

#include "asm_common.h"
#include "row_common.h"
#include "wave.h"

namespace dgp {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int P, bool MX>
struct F32Cfg {
    static_assert(P == 1 || P == 2, "FP32 rows of degree 1 or 2");
    static constexpr int NB = nb2d(P);
    static constexpr int NQT = Tri<4>::n;  // the degree-4 rule on each fan sub-triangle
    // MX: neighbours of any degree up to kMaxP (mixed meshes)
    static constexpr int PN = MX ? kMaxP : P;
    static constexpr int NBN = nb2d(PN);
    static constexpr int NG = 3;           // Gauss points per edge on one-degree meshes (max(p + 1, 3))
    // lanes per edge group: 4 on one-degree meshes; on mixed meshes 4 or 8 by
    // the edge's Gauss points (max(p, p') + 1, at least 3), 8-lane groups first
    static constexpr int FG = MX ? 8 : 4;
    static constexpr int CW = NB + 1;      // MX: neighbour trial rows per cross chunk (the trial rows and the load row)
    static constexpr bool EL = P == 2;     // element block and load through the table
    static constexpr int KS = 3 * 64 + 4;  // table row stride: 192 point terms + 4 (rows start 4 banks apart)
    // rows: test terms (NB), the neighbour's or the row's own trial terms (NB), load terms (1)
    static constexpr int LW = (2 * NB + 1) * KS;
};

// The manufactured data (the sine solution) at a point given by its offset
// (px, py) from the box centre (x0, y0), in FP64: sin / cos by angle addition from the centre's values
// when the element is small (near), else directly.  FP64 because the load f is a
// sum of terms up to tens of times larger than itself (FP32 data put the load
// rows of elements where f changes sign 6e-5 off).
__device__ __forceinline__ PointData data_near(const DevProblem &pr, bool near, double x0, double y0, double s0x,
                                               double c0x, double s0y, double c0y, float px, float py, bool need_f) {
    const double x = x0 + double(px), y = y0 + double(py);
    if (!near) return point_data<true>(pr, x, y, need_f);
    double sx, cx, sy, cy;
    sincospi_near(s0x, c0x, double(px), &sx, &cx);
    sincospi_near(s0y, c0y, double(py), &sy, &cy);
    return point_data_sc<true>(pr, x, y, sx, cx, sy, cy, need_f);
}

// a + b with its rounding error carried in e (TwoSum, Knuth)
__device__ __forceinline__ void two_sum_acc(float &s, float &e, float b) {
    const float t = s + b;
    const float z = t - s;
    e += (s - (t - z)) + (b - z);
    s = t;
}

// a * d/dxi phi_j + b and a * d/deta phi_j + b, with b alone when phi_j is
// constant in that direction (j is an unrolled index: the test folds away)
template <int P>
__device__ __forceinline__ float fma_gx(const Eval<float, P> &ev, int j, float a, float b) {
    return exp_a(j) > 0 ? fmaf(a, ev.g0[j], b) : b;
}
template <int P>
__device__ __forceinline__ float fma_gy(const Eval<float, P> &ev, int j, float a, float b) {
    return exp_b(j) > 0 ? fmaf(a, ev.g1[j], b) : b;
}

// Element row c (degree P, all neighbours of degree P) in one wave.
template <int P, bool ADV, bool MX>
__device__ __forceinline__ void row_f32(const AsmArgs &A, const int c, float *xs) {
    using C = F32Cfg<P, MX>;
    constexpr int NB = C::NB, NQT = C::NQT, NG = C::NG, FG = C::FG, KS = C::KS;
    const int lane = threadIdx.x & 63;
    RowHead h;
    if (!row_head(A, c, NB, h)) return;
    const DevMesh &m = A.m;
    const DevProblem &pr = A.pr;
    float *__restrict__ vals = static_cast<float *>(A.vals);
    float *__restrict__ rhs = static_cast<float *>(A.rhs);
    const int nv = h.nv;

    // ---- per row, FP64
    const CellGeo g = A.geo[c];
    const double lox = g.lox, loy = g.loy, hix = g.hix, hiy = g.hiy, ihx = g.ihx, ihy = g.ihy;
    const double xc = 0.5 * (lox + hix), yc = 0.5 * (loy + hiy);
    const double hxd = hix - lox, hyd = hiy - loy;
    // data by angle addition from the centre when pi |half diagonal| <= kNearT
    constexpr double kNearD2 = (2.0 * kNearT / kPi) * (2.0 * kNearT / kPi);
    const bool near = hxd * hxd + hyd * hyd <= kNearD2;
    const float cxf = float(2.0 * ihx), cyf = float(2.0 * ihy);          // box factors 2 / h
    const float cx2 = float(4.0 * ihx * ihx), cy2 = float(4.0 * ihy * ihy);
    const double s0x = g.sx, c0x = g.cx, s0y = g.sy, c0y = g.cy;
    const double isq = g.isq;

    // ---- per vertex / sub-triangle / edge (lane k < nv), FP64, rounded once
    const int kw = lane + 1 < nv ? lane + 1 : 0;  // the edge's end vertex
    const double xw = __shfl(h.ex, kw, 64), yw = __shfl(h.ey, kw, 64);
    const int vw = __shfl(h.vid, kw, 64);
    const double x0 = readlane_d(h.ex, 0), y0 = readlane_d(h.ey, 0);
    // vertex k: box coordinates and the data position
    const float v_xi = float(((h.ex - lox) - (hix - h.ex)) * ihx);
    const float v_eta = float(((h.ey - loy) - (hiy - h.ey)) * ihy);
    const float v_px = float(h.ex - xc), v_py = float(h.ey - yc);  // offset from the centre
    const float v_ax = float(h.ex), v_ay = float(h.ey);              // absolute (exact for 0 and 1)
    // sub-triangle (0, k, k + 1)
    const float t_area = float(0.5 * ((h.ex - x0) * (yw - y0) - (xw - x0) * (h.ey - y0)));
    // edge k, from its lower-id end a to b
    float e_nxi = 0.0f, e_neta = 0.0f, e_ndxi = 0.0f, e_ndeta = 0.0f;  // neighbour's box coordinates
    float e_len = 0.0f, e_nx = 0.0f, e_ny = 0.0f, e_hs = 0.0f;  // length (negative: a = end vertex), normal, sigma - upwind
    float e_bnx = 0.0f, e_bny = 0.0f, e_xsc = 0.0f;                    // neighbour box factor x normal, scale
    if (lane < nv) {
        const bool fwd = h.vid < vw;
        const double xa = fwd ? h.ex : xw, ya = fwd ? h.ey : yw;
        const double tx = (fwd ? xw : h.ex) - xa, ty = (fwd ? yw : h.ey) - ya;
        // length and normal in FP32 from the FP64 edge vector rounded once
        // (reciprocal square root: about one ulp, as the rounding of the values)
        const float txf = float(tx), tyf = float(ty);
        const float l2 = fmaf(txf, txf, tyf * tyf);
        const float il = __builtin_amdgcn_rsqf(l2);
        const float len = l2 * il;
        const float dl = fwd ? il : -il;
        const float nx = tyf * dl, ny = -txf * dl;  // outward for a counter-clockwise loop
        // b.n with its cancellation in FP64 (an edge nearly along b has a tiny
        // upwind weight, which must keep its relative accuracy)
        const float bn = float(pr.bx * ty - pr.by * tx) * dl;
        const float up = bn < 0.0f ? bn : 0.0f;
        e_len = fwd ? len : -len;
        e_nx = nx;
        e_ny = ny;
        double sigma;
        if (h.o >= 0) {
            const CellGeo go = A.geo[h.o];
            e_nxi = float(((xa - go.lox) - (go.hix - xa)) * go.ihx);
            e_neta = float(((ya - go.loy) - (go.hiy - ya)) * go.ihy);
            e_ndxi = float(2.0 * tx * go.ihx);
            e_ndeta = float(2.0 * ty * go.ihy);
            e_bnx = float(2.0 * go.ihx) * nx;
            e_bny = float(2.0 * go.ihy) * ny;
            e_xsc = float(isq * go.isq);
            sigma = pr.c_sigma * (g.pen > go.pen ? g.pen : go.pen);
            if (pr.penalty == 1) {
                const int F = m.cell_face[h.s0 + lane];
                sigma = pr.c_sigma * double(len) * fmax(A.pen_face[2 * F], A.pen_face[2 * F + 1]);
            }
        } else {
            sigma = pr.c_sigma * g.pen;
            if (pr.penalty == 1) sigma = pr.c_sigma * double(len) * A.pen_face[2 * m.cell_face[h.s0 + lane]];
        }
        e_hs = float(sigma - double(up));
    }
    // mixed meshes: the degree across each loop edge, and the groups reordered
    // so that those needing 8 lanes (a degree-4 neighbour: 5 Gauss points)
    // come first, each on an 8-lane boundary; group g then starts at lane
    // QF0 + 8 g (g < n2) or QF0 + 4 (n2 + g)
    int e_po = P, gtab = h.gtab, n2 = 0;
    if constexpr (MX) {
        if (lane < nv && h.o >= 0) e_po = m.cell_p[h.o];
        const bool lead = (h.gmask >> lane) & 1ull;
        const bool wide = lead && (P > e_po ? P : e_po) + 1 > 4;
        const uint64_t m2 = __ballot(wide), m1 = h.gmask & ~m2;
        n2 = __popcll(m2);
        const uint64_t below = (1ull << lane) - 1ull;
        const int gidx = wide ? __popcll(m2 & below) : n2 + __popcll(m1 & below);
        const int dst = lead ? gidx : h.ng + (lane - __popcll(h.gmask & below));
        gtab = __builtin_amdgcn_ds_permute(dst << 2, lane);
    }
    // vertex 0 (the fan apex), uniform
    const float xi0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v_xi)));
    const float eta0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v_eta)));
    const float px0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v_px)));
    const float py0 = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v_py)));

    // ---- the points
    const int QM = (nv - 2) * NQT;             // fan sub-triangle points
    const int QF0 = (QM + FG - 1) / FG * FG;   // edge groups start here
    const int Qtot = MX ? QF0 + 4 * (n2 + h.ng) : QF0 + FG * h.ng;
    // EL: lane e < NB (NB + 1) holds entry (e / (NB + 1), e mod (NB + 1)) of the
    // element block (column NB: the load), with its carried rounding error
    float acc_e = 0.0f, err_e = 0.0f;
    float acc[NB * NB + NB];                   // p = 1: element block and load, then the reduce-scatter
#pragma unroll
    for (int e = 0; e < NB * NB + NB; ++e) acc[e] = 0.0f;
    float *U = xs, *S = xs + NB * KS, *Rr = xs + 2 * NB * KS;
    const int k0 = 3 * lane;

    for (int base = 0; base < Qtot; base += 64) {
        const int q = base + lane;
        const bool edge_lane = q >= QF0 && q < Qtot;
        int gi, gq;  // the lane's edge group and its point in the group
        if constexpr (MX) {
            const int u = (q - QF0) >> 2;  // 4-lane unit (QF0 is a multiple of 8)
            gi = edge_lane ? (u < 2 * n2 ? u >> 1 : u - n2) : 0;
            gq = edge_lane ? (u < 2 * n2 ? (u & 1) << 2 : 0) + (q & 3) : 0;
        } else {
            gi = edge_lane ? (q - QF0) / FG : 0;
            gq = edge_lane ? (q - QF0) - gi * FG : 0;
        }
        const int fl = __shfl(gtab, gi, 64);  // the group's leading edge
        const int og = __shfl(h.o, fl, 64);
        const int gvoff = __shfl(h.voff, fl, 64);
        // the degree across the group's edges and their Gauss points
        const int po = MX ? __shfl(e_po, fl, 64) : P;
        const int ngf = MX ? max((P > po ? P : po) + 1, 3) : NG;
        const bool pass_has_edges = base + 64 > QF0 && base < Qtot;
        const int np = min(64, Qtot - base);
        for (int d = 0; d < h.maxdup; ++d) {
            // the lane's edge: the d-th of its group (edges towards one neighbour, in loop order)
            int fk = fl;
            if (d > 0) {
                int seen = 0;
                fk = -1;
                for (int k = 0; k < nv; ++k) {
                    const int ok = __shfl(h.o, k, 64);
                    if (og >= 0 && ok == og) {
                        if (seen == d) fk = k;
                        ++seen;
                    }
                }
            }
            const bool vol = d == 0 && q < QM;
            const bool epnt = edge_lane && gq < ngf && fk >= 0;
            // fetch: a fan point's vertices and sub-triangle, or an edge point's edge
            const int tri = vol ? q / NQT : 0;
            // s1, s2: the sub-triangle's second and third vertices, or the edge's start and end
            const int s1 = vol ? tri + 1 : (fk >= 0 ? fk : 0);
            const int s2 = vol ? tri + 2 : (s1 + 1 < nv ? s1 + 1 : 0);
            const float xi1 = __shfl(v_xi, s1, 64), eta1 = __shfl(v_eta, s1, 64);
            const float xi2 = __shfl(v_xi, s2, 64), eta2 = __shfl(v_eta, s2, 64);
            const float px1 = __shfl(v_px, s1, 64), py1 = __shfl(v_py, s1, 64);
            const float px2 = __shfl(v_px, s2, 64), py2 = __shfl(v_py, s2, 64);
            const float area = __shfl(t_area, s1, 64);
            const float ax1 = __shfl(v_ax, s1, 64), ay1 = __shfl(v_ay, s1, 64);
            const float ax2 = __shfl(v_ax, s2, 64), ay2 = __shfl(v_ay, s2, 64);
            const float a_nxi = __shfl(e_nxi, s1, 64), a_neta = __shfl(e_neta, s1, 64);
            const float a_ndxi = __shfl(e_ndxi, s1, 64), a_ndeta = __shfl(e_ndeta, s1, 64);
            const float a_len = __shfl(e_len, s1, 64), a_nx = __shfl(e_nx, s1, 64), a_ny = __shfl(e_ny, s1, 64);
            const float a_hs = __shfl(e_hs, s1, 64), a_bnx = __shfl(e_bnx, s1, 64), a_bny = __shfl(e_bny, s1, 64);
            const float a_xsc = __shfl(e_xsc, s1, 64);

            float xi = 0.0f, eta = 0.0f, xin = 0.0f, etan = 0.0f;
            float a0 = 0.0f, a1 = 0.0f, b0 = 0.0f, b1 = 0.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
            float x0c = 0.0f, x1c = 0.0f, r0 = 0.0f, r1 = 0.0f, r2 = 0.0f;
            // the point: box coordinates, weight, data position (offset from the
            // centre, or absolute on a boundary edge)
            float W = 0.0f, tq = 0.0f, ppx = 0.0f, ppy = 0.0f;
            if (vol) {
                const int qi = q - tri * NQT;
                const float l1 = float(Tri<4>::l(3 * qi + 1)), l2 = float(Tri<4>::l(3 * qi + 2));
                W = float(Tri<4>::w(qi)) * area;
                xi = fmaf(l1, xi1 - xi0, fmaf(l2, xi2 - xi0, xi0));
                eta = fmaf(l1, eta1 - eta0, fmaf(l2, eta2 - eta0, eta0));
                ppx = fmaf(l1, px1 - px0, fmaf(l2, px2 - px0, px0));
                ppy = fmaf(l1, py1 - py0, fmaf(l2, py2 - py0, py0));
            } else if (epnt) {
                const int gk = (MX ? c_gl_off[ngf - 1] : c_gl_off[NG - 1]) + gq;
                tq = float(c_gl_t[gk]);
                W = float(c_gl_w[gk]) * fabsf(a_len);
                // from the lower-id end a to b (both rows place the edge's points alike)
                const bool fwd = a_len > 0.0f;
                const float xia = fwd ? xi1 : xi2, xib = fwd ? xi2 : xi1, etaa = fwd ? eta1 : eta2,
                            etab = fwd ? eta2 : eta1;
                xi = fmaf(tq, xib - xia, xia);
                eta = fmaf(tq, etab - etaa, etaa);
                // data position: offset from the centre inside, absolute on the boundary
                // (exact vertex coordinates there, so boundary data vanish exactly where u does)
                const float pxa = og >= 0 ? (fwd ? px1 : px2) : (fwd ? ax1 : ax2);
                const float pxb = og >= 0 ? (fwd ? px2 : px1) : (fwd ? ax2 : ax1);
                const float pya = og >= 0 ? (fwd ? py1 : py2) : (fwd ? ay1 : ay2);
                const float pyb = og >= 0 ? (fwd ? py2 : py1) : (fwd ? ay2 : ay1);
                ppx = fmaf(tq, pxb - pxa, pxa);
                ppy = fmaf(tq, pyb - pya, pya);
            }
            // data: one evaluation shared by the element points and the interior edge points
            PointData dd{};
            if (vol || (epnt && og >= 0))
                dd = data_near(pr, near, xc, yc, s0x, c0x, s0y, c0y, ppx, ppy, true);
            else if (epnt)
                dd = point_data<true>(pr, double(ppx), double(ppy), false);
            if (vol) {
                const float Wa = W * float(dd.a);
                a0 = Wa * cx2;
                a1 = Wa * cy2;
                if (ADV) {
                    c0 = W * float(pr.bx) * cxf;
                    c1 = W * float(pr.by) * cyf;
                    c2 = W * float(pr.c);
                }
                r2 = float(double(W) * dd.f);
            } else if (epnt) {
                const float w = W;
                const float cnx = cxf * a_nx, cny = cyf * a_ny;
                if (og >= 0) {
                    const float ha = -0.5f * w * float(dd.a), hs = a_hs * w;
                    b0 = ha * cnx;
                    b1 = ha * cny;
                    c0 = ha * cnx;
                    c1 = ha * cny;
                    c2 = hs;
                    x0c = ha * a_bnx;
                    x1c = ha * a_bny;
                    xin = fmaf(tq, a_ndxi, a_nxi);
                    etan = fmaf(tq, a_ndeta, a_neta);
                } else if (og == -1) {
                    const float ha = -w * float(dd.a), hs = a_hs * w;
                    b0 = ha * cnx;
                    b1 = ha * cny;
                    c0 = ha * cnx;
                    c1 = ha * cny;
                    c2 = hs;
                    const float uu = float(dd.u);
                    r0 = ha * uu * cnx;
                    r1 = ha * uu * cny;
                    r2 = hs * uu;
                } else {
                    r2 = float(double(w) * dd.a * (dd.ux * double(a_nx) + dd.uy * double(a_ny)));
                }
            }
            Eval<float, P> ev;
            ev.at(xi, eta);
            // ---- element block and load
            if constexpr (!C::EL) {
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const float t0 = fma_gx(ev, j, a0, b0 * ev.v[j]);
                    const float t1 = fma_gy(ev, j, a1, b1 * ev.v[j]);
                    const float t2 = fma_gx(ev, j, c0, fma_gy(ev, j, c1, c2 * ev.v[j]));
#pragma unroll
                    for (int i = 0; i < NB; ++i)
                        acc[i * NB + j] = fma_gx(ev, i, t0, fma_gy(ev, i, t1, fmaf(ev.v[i], t2, acc[i * NB + j])));
                }
#pragma unroll
                for (int i = 0; i < NB; ++i)
                    acc[NB * NB + i] = fma_gx(ev, i, r0, fma_gy(ev, i, r1, fmaf(ev.v[i], r2, acc[NB * NB + i])));
            }
            // ---- the table: normalised test terms of every lane's point
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                U[i * KS + k0] = fma_gx(ev, i, float(kNorm[i]), 0.0f);
                U[i * KS + k0 + 1] = fma_gy(ev, i, float(kNorm[i]), 0.0f);
                U[i * KS + k0 + 2] = ev.v[i] * float(kNorm[i]);
            }
            if (pass_has_edges) {
                if constexpr (!MX) {
                    // cross blocks: the neighbour's normalised trial terms, scaled by its box factor
                    float Lx[P + 1], dLx[P + 1], Ly[P + 1], dLy[P + 1];
                    legendre<float, P>(xin, Lx, dLx);
                    legendre<float, P>(etan, Ly, dLy);
    #pragma unroll
                    for (int a = 1; a <= P; ++a) {
                        Lx[a] *= float(kSqrt2a1[a]);
                        dLx[a] *= float(kSqrt2a1[a]);
                        Ly[a] *= float(kSqrt2a1[a]);
                        dLy[a] *= float(kSqrt2a1[a]);
                    }
                    const float sb0 = -b0 * a_xsc, sb1 = -b1 * a_xsc, sx0 = x0c * a_xsc, sx1 = x1c * a_xsc,
                                sc2 = -c2 * a_xsc;
    #pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        // (a gradient component of a function constant in that direction is left out)
                        const float vj = Lx[exp_a(j)] * Ly[exp_b(j)];
                        float t2 = sc2 * vj;
                        if (exp_a(j) > 0) t2 = fmaf(sx0, dLx[exp_a(j)] * Ly[exp_b(j)], t2);
                        if (exp_b(j) > 0) t2 = fmaf(sx1, Lx[exp_a(j)] * dLy[exp_b(j)], t2);
                        S[j * KS + k0] = sb0 * vj;
                        S[j * KS + k0 + 1] = sb1 * vj;
                        S[j * KS + k0 + 2] = t2;
                    }
                    wave_sync();
                    // every interior group of the pass at once: entry e of the pass's
                    // groups (NB^2 per group, row-major inside it) goes to lane e mod 64
                    // of round e / 64; the lane sums u(i) s(j) over its group's 3 NG
                    // columns (16-byte aligned: 3 ql is a multiple of 12) and writes it
                    const int gfirst = base > QF0 ? (base - QF0) / FG : 0;
                    const int glast = min(h.ng, (base + 64 - QF0) / FG);
                    const int nent = (glast - gfirst) * (NB * NB);
                    // the lane's group: its block's value offset, or -1 (boundary edge,
                    // or no d-th edge towards this neighbour)
                    const int gv = edge_lane && og >= 0 && fk >= 0 ? gvoff : -1;
                    for (int e0 = 0; e0 < nent; e0 += 64) {
                        const int e = e0 + lane;
                        const int gl = e / (NB * NB);
                        const int ij = e - gl * (NB * NB);
                        const int ql = min(QF0 + (gfirst + gl) * FG - base, 63);  // the group's first lane
                        const int gvq = __shfl(gv, ql, 64);
                        if (e < nent && gvq >= 0) {
                            const int i = ij / NB, j = ij - NB * (ij / NB);
                            const float *uu = U + i * KS + 3 * ql;
                            const float *ss = S + j * KS + 3 * ql;
                            static_assert(3 * NG == 9 && KS % 4 == 0, "two float4 and one float per row");
                            const float4 ua = reinterpret_cast<const float4 *>(uu)[0], ub = reinterpret_cast<const float4 *>(uu)[1];
                            const float4 sa = reinterpret_cast<const float4 *>(ss)[0], sb = reinterpret_cast<const float4 *>(ss)[1];
                            float sum = uu[8] * ss[8];
                            sum = fmaf(ua.x, sa.x, fmaf(ua.y, sa.y, fmaf(ua.z, sa.z, fmaf(ua.w, sa.w, sum))));
                            sum = fmaf(ub.x, sb.x, fmaf(ub.y, sb.y, fmaf(ub.z, sb.z, fmaf(ub.w, sb.w, sum))));
                            float *dst = vals + h.pre_v + gvq + ij;
                            if (d == 0)
                                *dst = sum;
                            else
                                *dst += sum;
                        }
                    }
                } else {
                    // mixed degrees: the neighbour's normalised trial terms up to
                    // degree PN, scaled by its box factor, in chunks of CW trial rows
                    // (the trial rows and the load row of the table); every interior
                    // group of the pass at once, NB CW entries per group and chunk
                    // (entry (i, j) of block column j = chunk CW + jj), the group's
                    // 3 x (4 or 8) columns summed
                    constexpr int CW = C::CW, NBN = C::NBN, NCH = (NBN + CW - 1) / CW;
                    float Lx[C::PN + 1], dLx[C::PN + 1], Ly[C::PN + 1], dLy[C::PN + 1];
                    legendre<float, C::PN>(xin, Lx, dLx);
                    legendre<float, C::PN>(etan, Ly, dLy);
#pragma unroll
                    for (int a = 1; a <= C::PN; ++a) {
                        Lx[a] *= float(kSqrt2a1[a]);
                        dLx[a] *= float(kSqrt2a1[a]);
                        Ly[a] *= float(kSqrt2a1[a]);
                        dLy[a] *= float(kSqrt2a1[a]);
                    }
                    const float sb0 = -b0 * a_xsc, sb1 = -b1 * a_xsc, sx0 = x0c * a_xsc, sx1 = x1c * a_xsc,
                                sc2 = -c2 * a_xsc;
                    // groups whose units lie in this pass's units [ub, ue)
                    const int ub = max(base - QF0, 0) >> 2, ue = max(base + 64 - QF0, 0) >> 2;
                    const int gfirst = min(ub <= 2 * n2 ? (ub + 1) >> 1 : ub - n2, h.ng);
                    const int glast = min(ue <= 2 * n2 ? (ue + 1) >> 1 : ue - n2, h.ng);
                    const int nent = (glast - gfirst) * (NB * CW);
                    const int nbn = nb2d(po);
                    // the lane's group: its block's value offset and width, or -1
                    // (boundary edge, or no d-th edge towards this neighbour)
                    const int gv = edge_lane && og >= 0 && fk >= 0 ? (gvoff | (nbn << 16)) : -1;
                    const int wmax = __builtin_amdgcn_readfirstlane(wave_max_i(gv >= 0 ? nbn : 0));
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) {
                        if (ch * CW >= wmax) break;
                        if (ch > 0) wave_sync();  // the previous chunk's rows read before they are rewritten
#pragma unroll
                        for (int jj = 0; jj < CW; ++jj) {
                            const int j = ch * CW + jj;
                            if (j < NBN) {
                                const float vj = Lx[exp_a(j)] * Ly[exp_b(j)];
                                float t2 = sc2 * vj;
                                if (exp_a(j) > 0) t2 = fmaf(sx0, dLx[exp_a(j)] * Ly[exp_b(j)], t2);
                                if (exp_b(j) > 0) t2 = fmaf(sx1, Lx[exp_a(j)] * dLy[exp_b(j)], t2);
                                S[jj * KS + k0] = sb0 * vj;
                                S[jj * KS + k0 + 1] = sb1 * vj;
                                S[jj * KS + k0 + 2] = t2;
                            }
                        }
                        wave_sync();
                        for (int e0 = 0; e0 < nent; e0 += 64) {
                            const int e = e0 + lane;
                            const int gl = e / (NB * CW);
                            const int ij = e - gl * (NB * CW);
                            const int g = gfirst + gl;
                            const int ql = min(QF0 + (g < n2 ? 8 * g : 4 * (n2 + g)) - base, 63);  // the group's first lane
                            const int gvq = __shfl(gv, ql, 64);
                            const int i = ij / CW, j = ch * CW + (ij - CW * (ij / CW));
                            if (e < nent && gvq >= 0 && j < (gvq >> 16)) {
                                // 16-byte aligned: 3 ql is a multiple of 12
                                const float4 *uu = reinterpret_cast<const float4 *>(U + i * KS + 3 * ql);
                                const float4 *ss = reinterpret_cast<const float4 *>(S + (j - ch * CW) * KS + 3 * ql);
                                const int n4 = g < n2 ? 6 : 3;  // 3 x 8 or 3 x 4 columns
                                float sum = 0.0f;
                                for (int k = 0; k < n4; ++k) {
                                    const float4 ua = uu[k], sa = ss[k];
                                    sum = fmaf(ua.x, sa.x, fmaf(ua.y, sa.y, fmaf(ua.z, sa.z, fmaf(ua.w, sa.w, sum))));
                                }
                                float *dst = vals + h.pre_v + (gvq & 0xffff) + i * (gvq >> 16) + j;
                                if (d == 0)
                                    *dst = sum;
                                else
                                    *dst += sum;
                            }
                        }
                    }
                }
                wave_sync();  // cross entries read before the trial rows are rewritten
            }
            if constexpr (C::EL) {
                // element block and load of the pass: the row's own trial terms and
                // the load terms join the test terms in the table (the load terms as
                // trial row NB), and the matrix cores form the NB x (NB + 1) product
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    S[j * KS + k0] = fma_gx(ev, j, a0, b0 * ev.v[j]);
                    S[j * KS + k0 + 1] = fma_gy(ev, j, a1, b1 * ev.v[j]);
                    S[j * KS + k0 + 2] = fma_gx(ev, j, c0, fma_gy(ev, j, c1, c2 * ev.v[j]));
                }
                Rr[k0] = r0;
                Rr[k0 + 1] = r1;
                Rr[k0 + 2] = r2;
                wave_sync();
                // 4 x 4 x 1 matrix products in 16 blocks: block b takes the pass's
                // points b, b + 16, ...; its lane 4 b + r supplies test row r (rows
                // 0-3) and 4 + r (rows 4, 5) and trial row r (columns 0-3) and 4 + r
                // (columns 4, 5 and the load), one term a of the rank-3 form per
                // product.  Rows past the block (r >= 2 of the second test slice,
                // r = 3 of the second trial slice) read a valid table row: they only
                // feed output entries that are never read.
                const int bk = lane >> 2, rr = lane & 3;
                const float *ua = U + rr * KS, *ub = U + (4 + min(rr, 1)) * KS;
                const float *ta = S + rr * KS, *tb = S + (4 + min(rr, 2)) * KS;  // S row 6 is the load row
                f32x4 m00 = {0.0f, 0.0f, 0.0f, 0.0f}, m01 = m00, m10 = m00, m11 = m00;
                const int nr = (np + 15) >> 4;
                for (int k = 0; k < nr; ++k) {
                    const int col = 3 * (16 * k + bk);
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const float xa = ua[col + a], xb = ub[col + a], ya = ta[col + a], yb = tb[col + a];
                        m00 = __builtin_amdgcn_mfma_f32_4x4x1f32(xa, ya, m00, 0, 0, 0);
                        m01 = __builtin_amdgcn_mfma_f32_4x4x1f32(xa, yb, m01, 0, 0, 0);
                        m10 = __builtin_amdgcn_mfma_f32_4x4x1f32(xb, ya, m10, 0, 0, 0);
                        m11 = __builtin_amdgcn_mfma_f32_4x4x1f32(xb, yb, m11, 0, 0, 0);
                    }
                }
                wave_sync();  // every table read done before the partial sums overwrite the test rows
                // the 16 blocks' partial sums to LDS, entry-major (entry (4 s + x, 4 t + y)
                // of slice pair (s, t) at red[((2 s + t) 16 + 4 x + y) 16 + block]), then
                // lane e < NB (NB + 1) adds up its entry's 16 and carries it into its
                // running sum with TwoSum
                float *red = U;
#pragma unroll
                for (int x = 0; x < 4; ++x) {
                    red[((0 * 16) + 4 * x + rr) * 16 + bk] = m00[x];
                    red[((1 * 16) + 4 * x + rr) * 16 + bk] = m01[x];
                    red[((2 * 16) + 4 * x + rr) * 16 + bk] = m10[x];
                    red[((3 * 16) + 4 * x + rr) * 16 + bk] = m11[x];
                }
                wave_sync();
                if (lane < NB * (NB + 1)) {
                    const int ie = lane / (NB + 1), je = lane - (NB + 1) * ie;
                    const int sp = 2 * (ie >> 2) + (je >> 2);
                    const float4 *pp = reinterpret_cast<const float4 *>(red + (sp * 16 + 4 * (ie & 3) + (je & 3)) * 16);
                    const float4 q0 = pp[0], q1 = pp[1], q2 = pp[2], q3 = pp[3];
                    const float sum = ((q0.x + q0.y) + (q0.z + q0.w)) + ((q1.x + q1.y) + (q1.z + q1.w)) +
                                      (((q2.x + q2.y) + (q2.z + q2.w)) + ((q3.x + q3.y) + (q3.z + q3.w)));
                    two_sum_acc(acc_e, err_e, sum);
                }
                wave_sync();
            }
        }
    }
    if constexpr (C::EL) {
        const int i = lane / (NB + 1), j = lane - (NB + 1) * i;
        if (lane < NB * (NB + 1)) {
            const double v = double(acc_e) + double(err_e);
            if (j < NB)
                vals[h.pre_v + h.dvoff + i * NB + j] = float(v * (c_norm[j] * isq * isq));
            else
                rhs[h.pre_d + i] = float(v * isq);
        }
    } else {
        // reduce-scatter over the wave: lane e holds entry e (block row-major, then the load)
        constexpr int E = NB * NB + NB;
        float a64[64];
#pragma unroll
        for (int e = 0; e < 64; ++e) a64[e] = e < E ? acc[e] : 0.0f;
        WaveRS<float, 32, E>::run(a64, lane);
        if (lane < NB * NB) {
            const int i = lane / NB, j = lane - i * NB;
            vals[h.pre_v + h.dvoff + lane] = float(double(a64[0]) * (c_norm[i] * c_norm[j] * isq * isq));
        } else if (lane < E) {
            const int i = lane - NB * NB;
            rhs[h.pre_d + i] = float(double(a64[0]) * (c_norm[i] * isq));
        }
    }
}

}  // namespace
}  // namespace dgp
