// 2D SIPG assembly, one wave per element row (row-owner form, no atomics).
//
// A wave owns element row r.  Its lanes first hold the loop edges (start
// vertex, neighbour across the edge, the rank and value offset of the
// neighbour's block, as the preparation kernel recorded them), and the row's
// offsets come from the scanned tile sums plus the element's prefix inside its
// tile; with them the wave writes its row of the block pattern (Section 3.4,
// Approach 2: one block per distinct neighbour, columns ascending).  Then
// every lane takes one quadrature point of the row: a point of a fan
// sub-triangle (element term, first line of eq. dg-bilinear, and the load of
// eq. dg-linear) or a point of an edge (the face lines of both equations).
// Edges are handled in groups of FG lanes, one group per neighbour (every
// edge shared with it, in loop order) or per boundary edge, so each cross
// block is summed inside its group.
//
// Every term at a point is a rank-3 update in the row's test functions
// (u_0, u_1, u_2) = (d phi / d xi, d phi / d eta, phi):
//     D_ij += sum_a u_a(i) t_a(j),   t_0 = a0 g0 + b0 v,  t_1 = a1 g1 + b1 v,
//                                    t_2 = c0 g0 + c1 g1 + c2 v     (trial = own basis)
//     X_ij += sum_a u_a(i) s_a(j),   s from the neighbour's basis
//     F_i  += sum_a u_a(i) r_a
// with, written for the test functions phi_i of row r (dn = grad phi . n_r,
// primes = the neighbour's basis, bn = b . n_r, w the point weight):
//   element:  a0 = w a cx^2, a1 = w a cy^2, (c0, c1, c2) = w (b_x cx, b_y cy, c), r_2 = w f
//   interior: b0 = ha cnx, b1 = ha cny, (c0, c1, c2) = (ha cnx, ha cny, hs),
//             s_0 = -ha cnx v', s_1 = -ha cny v', s_2 = ha dn' - hs v',
//             ha = -w a / 2, hs = w (sigma - [bn < 0] bn)
//   boundary: as interior with ha = -w a and no cross block;
//             (r_0, r_1, r_2) = (cnx ga, cny ga, gs), ga = -w a g, gs = hs g
//   Neumann:  r_2 = w g_N
// (cx, cy = 2 / box sides; cnx = cx n_x).  Lanes accumulate the element block
// and the load in registers over their points; a reduce-scatter across the
// wave then leaves entry e in lane e (a coalesced write).  Cross blocks are
// summed column by column inside their group and written directly.  Large
// element blocks are built in column slices of JS columns to bound registers.
//
// Precision: positions, Jacobians, box factors, coefficients, the load and the
// penalty are FP64; the point coefficients are rounded once to T and the
// basis is evaluated in T.  The basis normalisation s_i s'_j is applied to the
// finished sums in FP64.
#include <type_traits>
#include <utility>

#include "asm_common.h"
#include "kernels.h"
#include "row_common.h"
#include "row_f32.h"
#include "wave.h"

namespace dgp {

namespace {

// Row stride (elements) of the matrix-core tables: a lane stores table rows
// 3 l + a, so with rows of 16 the lanes of one store start 48 elements apart
// and fall on 4 of the banks (an 8-way conflict per store); with rows of 17
// they start 51 apart, an odd stride, and every lane of a store has its own
// bank.  The matrix-instruction reads (16 consecutive columns of 4 rows) then
// meet at most one 2-way conflict.
constexpr int kMfStride = 17;

// P: degree of the row's element; PN: largest degree of its neighbours
template <typename T, int P, int PN>
struct RowCfg {
    static constexpr int NB = nb2d(P);
    static constexpr int NBN = nb2d(PN);
    static constexpr int NB2 = NB * NB;
    // MF: the element block is a matrix-core product (p >= 3: 10 x 10 and
    // 15 x 15 blocks fill enough of a 16 x 16 tile); no column slices then
    static constexpr bool MF = P >= 3;
    static constexpr int MFW = sizeof(T) == 4 ? 2 * 96 * kMfStride : 2 * 48 * kMfStride;  // LDS table per wave (T elements)
    static constexpr int JS = MF ? NB : sizeof(T) == 4 ? (P <= 2 ? NB : P == 3 ? 5 : 3) : (P == 1 ? 3 : P == 2 ? 3 : 2);
    static constexpr int NSL = (NB + JS - 1) / JS;
    static constexpr int ED = MF ? 0 : NB * JS;  // element-block entries per slice held in registers
    static constexpr int E = ED + NB;   // with the load vector
    static_assert(E <= 64, "one entry per lane after the reduction");
    static constexpr int PF = P > PN ? P : PN;
    static constexpr int NG = PF + 1 > 3 ? PF + 1 : 3;  // Gauss points per edge, at most
    static constexpr int FG = NG <= 4 ? 4 : 8;         // lanes per edge group
    static constexpr int TDEG = P <= 2 ? 4 : 2 * P;
    static constexpr int NQT = Tri<TDEG>::n;
    // waves per SIMD the register allocation must allow (measured: three waves
    // beat two for the FP32 p <= 2 kernels even with a small spill)
    static constexpr int MINW = (sizeof(T) == 4 && P <= 2 && PN <= 2) ? 3 : 1;
    // cross blocks through a per-wave LDS table (XL) instead of per-column group sums
    static constexpr bool XL = sizeof(T) == 4 && P <= 2 && PN <= 2;
    static constexpr int XW = 3 * (NB + NBN);  // table row per lane: test terms, then trial terms
    // EL: the element block and the load through a transposed per-wave LDS table
    // (rows: the test terms of each basis function, the trial terms, the load
    // terms; columns k = 3 (lane) + a), each lane forming one entry as a dot
    // product over the pass's points, instead of 42 register accumulators per lane
    // and a reduce-scatter across the wave (FP32, p = 2 rows among p = 2 neighbours)
    static constexpr bool EL = XL && P == 2 && PN == 2;
    static constexpr int KS = 3 * 64 + 4;  // row stride: 192 point terms + 4 (rows start 4 banks apart)
    // CM: cross blocks on the matrix cores (p >= 3, and the FP32 mixed-degree
    // kernels, whose neighbours may have larger blocks than the row's own; in
    // FP64 the staged trial terms cost those kernels a wave per SIMD: slower)
    static constexpr bool CM = !XL && (P >= 3 || (PN > P && sizeof(T) == 4));
    static constexpr int CMW = 2 * 3 * FG * kMfStride;  // its table per wave (T elements)
    // VU: edge groups of 4 or 8 lanes (units of 4), by the Gauss points each
    // edge needs (a row of degree < 4 needs 8 only towards degree-4
    // neighbours): 8-lane groups first, each starting on an 8-lane boundary,
    // so no group straddles a pass of 64 lanes
    static constexpr bool VU = CM && FG == 8 && P < 4 && PN > P;
    // one LDS region per wave serves every table (their phases are separated by wave barriers)
    static constexpr int LW0 = EL ? (2 * NB + 1) * KS : XL ? 64 * XW : 0, LW1 = MF ? MFW : 0, LW2 = CM ? CMW : 0;
    static constexpr int LW = LW0 > LW1 ? (LW0 > LW2 ? LW0 : LW2) : (LW1 > LW2 ? LW1 : LW2);
};


// Per-point coefficients of the rank-3 updates (see the file comment).
// The cross block reuses the edge's own coefficients: s_0 = -b0 v', s_1 = -b1 v',
// s_2 = x0 g0' + x1 g1' - c2 v' (lanes of element points or boundary edges
// form cross terms too, but their groups are never written).
template <typename T>
struct PointCoef {
    T a0, b0, a1, b1, c0, c1, c2;  // element block
    T x0, x1;                      // cross block (neighbour's box factors)
    T r0, r1, r2;                  // load
    __device__ __forceinline__ void zero() {
        a0 = b0 = a1 = b1 = c0 = c1 = c2 = x0 = x1 = r0 = r1 = r2 = T(0);
    }
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));
template <typename T>
using MfAcc = std::conditional_t<sizeof(T) == 4, f32x4, f64x4>;
__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Element block on the matrix cores: D_ij = sum over (point, a) of u_a(i) t_a(j)
// with the test terms u = (d/dxi, d/deta, value) of basis i and the trial terms
// t_a(j) of the rank-3 form.  The 64 points of a pass go through LDS in groups
// of lanes (two of 32 in FP32, four of 16 in FP64: 12 KB per wave either way),
// 3 rows of u and of t per lane, 16 columns (the basis index, padding unused);
// each group is K / 4 steps of the 16 x 16 x 4 matrix instruction (A: row
// lane % 16, k lane / 16; B: k lane / 16, column lane % 16).  Accumulator r of
// lane l holds D[4 (l / 16) + r][l % 16] in FP32 and D[4 r + l / 16][l % 16]
// in FP64 (mf_row).  Padding rows and columns only reach entries that are
// never written.
template <typename T>
__device__ __forceinline__ int mf_row(int lane, int r) {
    return sizeof(T) == 4 ? 4 * (lane >> 4) + r : 4 * r + (lane >> 4);
}

template <typename T, int P>
__device__ __forceinline__ void mf_element(T *lds, int lane, const Eval<T, P> &ev, const PointCoef<T> &pc,
                                           MfAcc<T> &acc) {
    constexpr int NB = nb2d(P);
    constexpr int NGR = sizeof(T) == 4 ? 2 : 4;  // lane groups staged in turn
    constexpr int LG = 64 / NGR;                 // lanes per group
    constexpr int KR = 3 * LG;                   // rows of u (and of t) per group
    T *U = lds, *Tt = lds + KR * kMfStride;
#pragma unroll
    for (int g = 0; g < NGR; ++g) {
        if (lane / LG == g) {
            const int k0 = 3 * (lane % LG);
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                U[(k0 + 0) * kMfStride + j] = ev.g0[j];
                U[(k0 + 1) * kMfStride + j] = ev.g1[j];
                U[(k0 + 2) * kMfStride + j] = ev.v[j];
                Tt[(k0 + 0) * kMfStride + j] = fmat(pc.a0, ev.g0[j], pc.b0 * ev.v[j]);
                Tt[(k0 + 1) * kMfStride + j] = fmat(pc.a1, ev.g1[j], pc.b1 * ev.v[j]);
                Tt[(k0 + 2) * kMfStride + j] = fmat(pc.c0, ev.g0[j], fmat(pc.c1, ev.g1[j], pc.c2 * ev.v[j]));
            }
        }
        wave_sync();
        const int r = lane >> 4, c = lane & 15;
#pragma unroll 4
        for (int s = 0; s < KR / 4; ++s)
            acc = mfma16(U[(4 * s + r) * kMfStride + c], Tt[(4 * s + r) * kMfStride + c], acc);
        wave_sync();  // the next group rewrites the table
    }
}

// Everything a slice of the row needs, computed once per row.
struct RowCtx {
    int lane, c, nv, vid, o, voff, dvoff, maxdup, QM, QF0, Qtot, QR;
    int gtab;  // lane g < number of groups: loop index of the g-th group's leading edge
    int ng;    // number of edge groups
    int n2;    // VU kernels: groups 0 .. n2 - 1 have 8 lanes, the others 4
    void *xs;  // the wave's cross-block table in LDS (XL kernels)
    bool red;
    uint64_t gmask;
    double ex, ey, x0, y0, isq, hx, hy, pen_r;  // x0, y0: the fan apex (first vertex)
    double lox, loy, hix, hiy, ihx, ihy;        // the box and 1 / its sides
    int64_t s0;                                 // the row's first loop entry (cell_ptr)
    int64_t pre_v, pre_d;
    Box bx;
    TrigCentre tc;
};

// Cross blocks of the edge groups in one pass of 64 points, through LDS.  Every
// lane stores its point's normalised test terms u_a(i) (a = 0, 1, 2: d/dxi,
// d/deta, value) and trial terms s_a(j) of the neighbour's normalised basis,
// already scaled by the neighbour's box factor (zero for lanes without an
// interior edge point).  Then each lane takes entries (group, i, j) of the
// pass and sums u(i) . s(j) over the group's points: no cross-lane reductions,
// and the entries of a block go out in row-major order.
template <typename T, int P, int PN>
__device__ __forceinline__ void cross_lds(const AsmArgs &A, const RowCtx &R, const Eval<T, P> &ev,
                                          const PointCoef<T> &pc, double xin, double etan, double xsc, int base,
                                          int d, int og, int gvoff, int fk) {
    using C = RowCfg<T, P, PN>;
    constexpr int NB = C::NB, NBN = C::NBN, XW = C::XW, FG = C::FG, NBX = NB * NBN;
    constexpr int NGP = C::NG;  // Gauss points per edge (all neighbours have degree P here)
    T *xs = static_cast<T *>(R.xs);
    {
        T Lx[PN + 1], dLx[PN + 1], Ly[PN + 1], dLy[PN + 1];
        legendre<T, PN>(T(xin), Lx, dLx);
        legendre<T, PN>(T(etan), Ly, dLy);
#pragma unroll
        for (int a = 1; a <= PN; ++a) {
            Lx[a] *= T(kSqrt2a1[a]);
            dLx[a] *= T(kSqrt2a1[a]);
            Ly[a] *= T(kSqrt2a1[a]);
            dLy[a] *= T(kSqrt2a1[a]);
        }
        const T xs_ = T(xsc);
        const T sb0 = -pc.b0 * xs_, sb1 = -pc.b1 * xs_, sx0 = pc.x0 * xs_, sx1 = pc.x1 * xs_, sc2 = -pc.c2 * xs_;
        T *row = xs + R.lane * XW;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            row[3 * i] = ev.g0[i] * T(kNorm[i]);
            row[3 * i + 1] = ev.g1[i] * T(kNorm[i]);
            row[3 * i + 2] = ev.v[i] * T(kNorm[i]);
        }
#pragma unroll
        for (int j = 0; j < NBN; ++j) {
            const T vj = Lx[exp_a(j)] * Ly[exp_b(j)];
            const T gj0 = dLx[exp_a(j)] * Ly[exp_b(j)], gj1 = Lx[exp_a(j)] * dLy[exp_b(j)];
            row[3 * NB + 3 * j] = sb0 * vj;
            row[3 * NB + 3 * j + 1] = sb1 * vj;
            row[3 * NB + 3 * j + 2] = fmat(sx0, gj0, fmat(sx1, gj1, sc2 * vj));
        }
    }
    wave_sync();
    // groups whose lanes lie in this pass (groups never straddle passes: 64 % FG == 0)
    const int gfirst = base > R.QF0 ? (base - R.QF0) / FG : 0;
    const int glast = min(R.ng, (base + 64 - R.QF0) / FG);
    const int nent = (glast - gfirst) * NBX;
    T *__restrict__ vals = static_cast<T *>(A.vals);
    for (int e0 = 0; e0 < nent; e0 += 64) {
        const int e = min(e0 + R.lane, nent - 1);
        const int gl = e / NBX, r = e - gl * NBX, i = r / NBN, j = r - i * NBN;
        const int ql = R.QF0 + (gfirst + gl) * FG - base;  // the group's first lane
        const int oge = __shfl(og, ql, 64), gvo = __shfl(gvoff, ql, 64), fke = __shfl(fk, ql, 64);
        const T *uu = xs + ql * XW + 3 * i;
        const T *ss = xs + ql * XW + 3 * NB + 3 * j;
        T sum = T(0);
#pragma unroll
        for (int p = 0; p < NGP; ++p)
            sum = fmat(uu[p * XW], ss[p * XW],
                       fmat(uu[p * XW + 1], ss[p * XW + 1], fmat(uu[p * XW + 2], ss[p * XW + 2], sum)));
        if (e0 + R.lane < nent && oge >= 0 && fke >= 0) {
            T *dst = vals + R.pre_v + gvo + i * NBN + j;
            if (d == 0)
                *dst = sum;
            else
                *dst += sum;
        }
    }
    wave_sync();  // the table is rewritten by the next point set
}

// The transposed table of the EL kernels, per wave: row i < NB holds the
// normalised test terms u_a(i) at column k = 3 (lane) + a; rows NB .. 2 NB - 1
// first hold the neighbour's trial terms s_a(j) (cross blocks), then the row's
// own trial terms t_a(j) (element block); row 2 NB the load terms r_a.  Every
// lane writes its point's columns (lanes without a point have zero
// coefficients, so their trial and load terms are zero).
//
// Cross blocks: each lane takes entries (group, i, j) of the pass and sums the
// 3 FG columns of its group's lanes: u(i) . s(j), written in row-major order.
template <typename T, int P, int PN>
__device__ __forceinline__ void cross_el(const AsmArgs &A, const RowCtx &R, const Eval<T, P> &ev,
                                         const PointCoef<T> &pc, double xin, double etan, double xsc, int base,
                                         int d, int og, int gvoff, int fk) {
    using C = RowCfg<T, P, PN>;
    constexpr int NB = C::NB, NBN = C::NBN, FG = C::FG, NBX = NB * NBN, KS = C::KS;
    constexpr int NGP = C::NG;  // Gauss points per edge (all neighbours have degree P here)
    static_assert(NGP <= FG, "one edge point per lane of a group");
    T *U = static_cast<T *>(R.xs), *S = U + NB * KS;
    const int k0 = 3 * R.lane;
    {
        T Lx[PN + 1], dLx[PN + 1], Ly[PN + 1], dLy[PN + 1];
        legendre<T, PN>(T(xin), Lx, dLx);
        legendre<T, PN>(T(etan), Ly, dLy);
#pragma unroll
        for (int a = 1; a <= PN; ++a) {
            Lx[a] *= T(kSqrt2a1[a]);
            dLx[a] *= T(kSqrt2a1[a]);
            Ly[a] *= T(kSqrt2a1[a]);
            dLy[a] *= T(kSqrt2a1[a]);
        }
        const T xs_ = T(xsc);
        const T sb0 = -pc.b0 * xs_, sb1 = -pc.b1 * xs_, sx0 = pc.x0 * xs_, sx1 = pc.x1 * xs_, sc2 = -pc.c2 * xs_;
#pragma unroll
        for (int j = 0; j < NBN; ++j) {
            const T vj = Lx[exp_a(j)] * Ly[exp_b(j)];
            const T gj0 = dLx[exp_a(j)] * Ly[exp_b(j)], gj1 = Lx[exp_a(j)] * dLy[exp_b(j)];
            S[j * KS + k0] = sb0 * vj;
            S[j * KS + k0 + 1] = sb1 * vj;
            S[j * KS + k0 + 2] = fmat(sx0, gj0, fmat(sx1, gj1, sc2 * vj));
        }
    }
    wave_sync();
    // groups whose lanes lie in this pass (groups never straddle passes: 64 % FG == 0)
    const int gfirst = base > R.QF0 ? (base - R.QF0) / FG : 0;
    const int glast = min(R.ng, (base + 64 - R.QF0) / FG);
    const int nent = (glast - gfirst) * NBX;
    T *__restrict__ vals = static_cast<T *>(A.vals);
    for (int e0 = 0; e0 < nent; e0 += 64) {
        const int e = min(e0 + R.lane, nent - 1);
        const int gl = e / NBX, r = e - gl * NBX, i = r / NBN, j = r - i * NBN;
        const int ql = R.QF0 + (gfirst + gl) * FG - base;  // the group's first lane (a multiple of 4)
        const int oge = __shfl(og, ql, 64), gvo = __shfl(gvoff, ql, 64), fke = __shfl(fk, ql, 64);
        const T *uu = U + i * KS + 3 * ql;
        const T *ss = S + j * KS + 3 * ql;
        T sum = T(0);
#pragma unroll
        for (int t = 0; t < 3 * NGP; ++t) sum = fmat(uu[t], ss[t], sum);
        if (e0 + R.lane < nent && oge >= 0 && fke >= 0) {
            T *dst = vals + R.pre_v + gvo + i * NBN + j;
            if (d == 0)
                *dst = sum;
            else
                *dst += sum;
        }
    }
}

// Writes the lane's normalised test terms (columns 3 lane .. 3 lane + 2 of rows 0 .. NB - 1).
template <typename T, int P, int PN>
__device__ __forceinline__ void el_test_terms(const RowCtx &R, const Eval<T, P> &ev) {
    using C = RowCfg<T, P, PN>;
    constexpr int NB = C::NB, KS = C::KS;
    T *U = static_cast<T *>(R.xs);
    const int k0 = 3 * R.lane;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        U[i * KS + k0] = ev.g0[i] * T(kNorm[i]);
        U[i * KS + k0 + 1] = ev.g1[i] * T(kNorm[i]);
        U[i * KS + k0 + 2] = ev.v[i] * T(kNorm[i]);
    }
}

// Element block and load of the pass: the lane's trial terms t_a(j) and load
// terms r_a go to rows NB .. 2 NB; then lane e < NB (NB + 1) adds entry
// (i, j) = (e / (NB + 1), e mod (NB + 1)) (j = NB: the load of row i) over the
// columns of the pass's np points to its accumulator.  load_only: only the load
// entries take part (the trial rows are not written).
template <typename T, int P, int PN>
__device__ __forceinline__ void elem_el(const RowCtx &R, const Eval<T, P> &ev, const PointCoef<T> &pc, int np,
                                        bool load_only, T &acc_e) {
    using C = RowCfg<T, P, PN>;
    constexpr int NB = C::NB, KS = C::KS;
    T *U = static_cast<T *>(R.xs), *Tt = U + NB * KS, *Rr = U + 2 * NB * KS;
    const int k0 = 3 * R.lane;
    if (!load_only) {
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            Tt[j * KS + k0] = fmat(pc.a0, ev.g0[j], pc.b0 * ev.v[j]);
            Tt[j * KS + k0 + 1] = fmat(pc.a1, ev.g1[j], pc.b1 * ev.v[j]);
            Tt[j * KS + k0 + 2] = fmat(pc.c0, ev.g0[j], fmat(pc.c1, ev.g1[j], pc.c2 * ev.v[j]));
        }
    }
    Rr[k0] = pc.r0;
    Rr[k0 + 1] = pc.r1;
    Rr[k0 + 2] = pc.r2;
    wave_sync();
    const int i = R.lane / (NB + 1), j = R.lane - (NB + 1) * i;
    if (R.lane < NB * (NB + 1) && (!load_only || j == NB)) {
        const float4 *uu = reinterpret_cast<const float4 *>(U + i * KS);
        const float4 *tt = reinterpret_cast<const float4 *>(j < NB ? Tt + j * KS : Rr);
        const int n4 = (3 * np + 3) >> 2;  // columns of the pass's points, in fours
        T s0 = T(0), s1 = T(0);
        int k = 0;
        for (; k + 1 < n4; k += 2) {
            const float4 a = uu[k], b = tt[k], c = uu[k + 1], e = tt[k + 1];
            s0 = fmat(a.x, b.x, fmat(a.y, b.y, fmat(a.z, b.z, fmat(a.w, b.w, s0))));
            s1 = fmat(c.x, e.x, fmat(c.y, e.y, fmat(c.z, e.z, fmat(c.w, e.w, s1))));
        }
        if (k < n4) {
            const float4 a = uu[k], b = tt[k];
            s0 = fmat(a.x, b.x, fmat(a.y, b.y, fmat(a.z, b.z, fmat(a.w, b.w, s0))));
        }
        acc_e += s0 + s1;
    }
    wave_sync();  // the table is rewritten by the next point set
}

// Cross blocks on the matrix cores (the p >= 3 and mixed-degree kernels): one edge group at a
// time, its FG lanes write 3 rows each of normalised test terms u_a(i) and of
// the neighbour's trial terms s_a(j) (normalised, scaled by its box factor;
// zero on lanes without a point) to LDS, and 3 FG / 4 steps of the 16 x 16 x 4
// instruction form the n_b(p) x n_b(p') block, written from the accumulator
// layout (mf_row).  Columns beyond the neighbour's n_b are not written.
template <typename T, int P, int PN>
__device__ __forceinline__ void cross_mf(const AsmArgs &A, const RowCtx &R, const Eval<T, P> &ev,
                                         const PointCoef<T> &pc, double xin, double etan, double xsc, int base,
                                         int d, int og, int gvoff, int fk, int nbo) {
    using C = RowCfg<T, P, PN>;
    constexpr int NB = C::NB, NBN = C::NBN, FG = C::FG, KR = 3 * FG;
    static_assert(KR % 4 == 0 && NB <= 16 && NBN <= 16, "one 16 x 16 tile per cross block");
    T *U = static_cast<T *>(R.xs), *S = U + KR * kMfStride;
    const int lane = R.lane;
    // this lane's trial terms (computed once, stored when its group's turn comes)
    T sv[3][NBN];
    {
        T Lx[PN + 1], dLx[PN + 1], Ly[PN + 1], dLy[PN + 1];
        legendre<T, PN>(T(xin), Lx, dLx);
        legendre<T, PN>(T(etan), Ly, dLy);
#pragma unroll
        for (int a = 1; a <= PN; ++a) {
            Lx[a] *= T(kSqrt2a1[a]);
            dLx[a] *= T(kSqrt2a1[a]);
            Ly[a] *= T(kSqrt2a1[a]);
            dLy[a] *= T(kSqrt2a1[a]);
        }
        const T xs_ = T(xsc);
        const T sb0 = -pc.b0 * xs_, sb1 = -pc.b1 * xs_, sx0 = pc.x0 * xs_, sx1 = pc.x1 * xs_, sc2 = -pc.c2 * xs_;
#pragma unroll
        for (int j = 0; j < NBN; ++j) {
            const T vj = Lx[exp_a(j)] * Ly[exp_b(j)];
            const T gj0 = dLx[exp_a(j)] * Ly[exp_b(j)], gj1 = Lx[exp_a(j)] * dLy[exp_b(j)];
            sv[0][j] = sb0 * vj;
            sv[1][j] = sb1 * vj;
            sv[2][j] = fmat(sx0, gj0, fmat(sx1, gj1, sc2 * vj));
        }
    }
    int gfirst, glast;
    if constexpr (C::VU) {
        // groups whose units lie in this pass's units [ub, ue)
        const int ub = max(base - R.QF0, 0) >> 2, ue = max(base + 64 - R.QF0, 0) >> 2;
        const int n2 = R.n2;
        gfirst = min(ub <= 2 * n2 ? (ub + 1) >> 1 : ub - n2, R.ng);
        glast = min(ue <= 2 * n2 ? (ue + 1) >> 1 : ue - n2, R.ng);
    } else {
        gfirst = base > R.QF0 ? (base - R.QF0) / FG : 0;
        glast = min(R.ng, (base + 64 - R.QF0) / FG);
    }
    T *__restrict__ vals = static_cast<T *>(A.vals);
    for (int g = gfirst; g < glast; ++g) {
        // the group's first lane and its lanes (uniform)
        const int ql = R.QF0 + (C::VU ? (g < R.n2 ? 8 * g : 4 * (R.n2 + g)) : g * FG) - base;
        const int fgl = C::VU ? (g < R.n2 ? 8 : 4) : FG;
        const int oge = __builtin_amdgcn_readlane(og, ql), fke = __builtin_amdgcn_readlane(fk, ql);
        if (oge < 0 || fke < 0) continue;
        if (lane >= ql && lane < ql + fgl) {
            const int k0 = 3 * (lane - ql);
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                U[(k0 + 0) * kMfStride + i] = ev.g0[i] * T(kNorm[i]);
                U[(k0 + 1) * kMfStride + i] = ev.g1[i] * T(kNorm[i]);
                U[(k0 + 2) * kMfStride + i] = ev.v[i] * T(kNorm[i]);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a)
#pragma unroll
                for (int j = 0; j < NBN; ++j) S[(k0 + a) * kMfStride + j] = sv[a][j];
        }
        wave_sync();
        MfAcc<T> acc = {T(0), T(0), T(0), T(0)};
        const int r4 = lane >> 4, c = lane & 15;
        const int ks = 3 * fgl / 4;  // matrix steps over the group's 3 fgl table rows
#pragma unroll
        for (int s = 0; s < KR / 4; ++s)
            if (s < ks) acc = mfma16(U[(4 * s + r4) * kMfStride + c], S[(4 * s + r4) * kMfStride + c], acc);
        wave_sync();  // the next group rewrites the table
        const int nbog = __builtin_amdgcn_readlane(nbo, ql), gvo = __builtin_amdgcn_readlane(gvoff, ql);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = mf_row<T>(lane, r);
            if (i < NB && c < nbog) {
                T *dst = vals + R.pre_v + gvo + i * nbog + c;
                if (d == 0)
                    *dst = acc[r];
                else
                    *dst += acc[r];
            }
        }
    }
}

template <typename T, int P, int PN, bool MX, bool ADV, int SL>
__device__ __forceinline__ void row_slice(const AsmArgs &A, const RowCtx &R) {
    using C = RowCfg<T, P, PN>;
    constexpr int NB = C::NB, JS = C::JS, FG = C::FG, ED = C::ED;
    constexpr int j0 = SL * JS;
    const DevMesh &m = A.m;
    const DevProblem &pr = A.pr;
    T *__restrict__ vals = static_cast<T *>(A.vals);
    T *__restrict__ rhs = static_cast<T *>(A.rhs);
    const int lane = R.lane, c = R.c, nv = R.nv, vid = R.vid, o = R.o, voff = R.voff;
    const int QM = R.QM, QF0 = R.QF0, Qtot = R.Qtot;
    const double ex = R.ex, ey = R.ey;
    const Box &bx = R.bx;
    const TrigCentre &tc = R.tc;
    using R_ = Tri<C::TDEG>;

    T acc[64];
#pragma unroll
    for (int e = 0; e < 64; ++e) acc[e] = T(0);  // [0, ED): element block slice, [ED, ED + NB): load
    T acc_e = T(0);                              // EL kernels: the lane's entry of the element block or load
    MfAcc<T> accm = {T(0), T(0), T(0), T(0)};   // MF kernels: the element block on the matrix cores

    for (int base = 0; base < Qtot; base += 64) {
        const int q = base + lane;
        const bool edge_lane = q >= QF0 && q < Qtot;
        int gi, gq;  // the lane's edge group and its point in the group
        if constexpr (C::VU) {
            const int u = (q - QF0) >> 2;  // 4-lane unit (QF0 is a multiple of 8)
            gi = edge_lane ? (u < 2 * R.n2 ? u >> 1 : u - R.n2) : 0;
            gq = edge_lane ? (u < 2 * R.n2 ? (u & 1) << 2 : 0) + (q & 3) : 0;
        } else {
            gi = edge_lane ? (q - QF0) / FG : 0;
            gq = edge_lane ? (q - QF0) - gi * FG : 0;
        }
        // leader edge of the lane's group
        const int fl = __shfl(R.gtab, gi, 64);
        const int og = __shfl(o, fl, 64);
        const int gvoff = __shfl(voff, fl, 64);
        const bool cross = edge_lane && og >= 0;
        Box bo{0.0, 0.0, 0.0, 0.0};
        double pen_o = 0.0, xsc = 0.0;
        double olox = 0.0, oloy = 0.0, ohix = 0.0, ohiy = 0.0, oihx = 0.0, oihy = 0.0;  // the neighbour's box
        int po = P;  // degree across the edge (the row's own on the boundary)
        if (cross) {
            const CellGeo go = A.geo[og];
            bo = box_of(go);
            olox = go.lox;
            oloy = go.loy;
            ohix = go.hix;
            ohiy = go.hiy;
            oihx = go.ihx;
            oihy = go.ihy;
            po = MX ? (int)m.cell_p[og] : P;
            pen_o = go.pen;  // abar p^2 / h at the neighbour's degree
            xsc = R.isq * go.isq;
        }
        const int nbo = nb2d(po);
        const int ngf = (P > po ? P : po) + 1 > 3 ? (P > po ? P : po) + 1 : 3;  // this edge's Gauss points
        const bool pass_has_edges = base + 64 > QF0 && base < Qtot;

        for (int d = 0; d < R.maxdup; ++d) {
            // the lane's point: an element point (d == 0) or point gq of the d-th edge of its group
            int fk = fl;
            if (d > 0) {
                int seen = 0;
                fk = -1;
                for (int k = 0; k < nv; ++k) {
                    const int ok = __shfl(o, k, 64);
                    if (og >= 0 && ok == og) {
                        if (seen == d) fk = k;
                        ++seen;
                    }
                }
            }
            const bool vol = d == 0 && q < QM;
            const bool epnt = edge_lane && gq < ngf && fk >= 0;
            const int tri = vol && !R.red ? q / C::NQT : 0;
            const int s1 = vol ? tri + 1 : (fk >= 0 ? fk : 0);
            const int s2 = vol ? tri + 2 : (fk >= 0 ? (fk + 1 == nv ? 0 : fk + 1) : 0);
            const double X0 = R.x0, Y0 = R.y0;
            const double X1 = __shfl(ex, s1, 64), Y1 = __shfl(ey, s1, 64);
            const double X2 = __shfl(ex, s2, 64), Y2 = __shfl(ey, s2, 64);
            const int V1 = __shfl(vid, s1, 64), V2 = __shfl(vid, s2, 64);

            PointCoef<T> pc;
            pc.zero();
            double xi = 0.0, eta = 0.0, xin = 0.0, etan = 0.0;
            // the lane's point and weight: a fan sub-triangle point, or point gq
            // of its edge (canonical order: lower vertex id first)
            const bool vpt = vol && !R.red;
            // the point is (rx, ry) + (dxq, dyq) with (rx, ry) a vertex of the loop: its box
            // coordinates come from the offset, not from absolute coordinates (which carry
            // rounding of the size of the coordinates, large on small cells)
            double px = 0.0, py = 0.0, W = 0.0, nx = 0.0, ny = 0.0, up = 0.0, flen = 0.0;
            double rx = 0.0, ry = 0.0, dxq = 0.0, dyq = 0.0;
            if (vpt) {
                const int qi = q - tri * C::NQT;
                const double area = 0.5 * ((X1 - X0) * (Y2 - Y0) - (X2 - X0) * (Y1 - Y0));
                const double l1 = R_::l(3 * qi + 1), l2 = R_::l(3 * qi + 2);
                rx = X0;
                ry = Y0;
                dxq = l1 * (X1 - X0) + l2 * (X2 - X0);
                dyq = l1 * (Y1 - Y0) + l2 * (Y2 - Y0);
                px = X0 + dxq;
                py = Y0 + dyq;
                W = R_::w(qi) * area;
            } else if (epnt) {
                const bool fwd = V1 < V2;
                const double xa = fwd ? X1 : X2, ya = fwd ? Y1 : Y2;
                const double tx = (fwd ? X2 : X1) - xa, ty = (fwd ? Y2 : Y1) - ya;
                const double len = sqrt(tx * tx + ty * ty);
                flen = len;
                const double dl = (fwd ? 1.0 : -1.0) / len;
                nx = ty * dl;  // outward for a CCW loop
                ny = -tx * dl;
                const double bn = pr.bx * nx + pr.by * ny;
                up = bn < 0.0 ? bn : 0.0;
                const int goff = c_gl_off[ngf - 1];
                const double tq = c_gl_t[goff + gq];
                W = c_gl_w[goff + gq] * len;
                rx = xa;
                ry = ya;
                dxq = tq * tx;
                dyq = tq * ty;
                px = xa + dxq;
                py = ya + dyq;
            }
            // box coordinates ((r - lo) - (hi - r) + 2 d) / (hi - lo) of the own and the neighbour's box
            const double xib = ((rx - R.lox) - (R.hix - rx) + 2.0 * dxq) * R.ihx;
            const double etab = ((ry - R.loy) - (R.hiy - ry) + 2.0 * dyq) * R.ihy;
            // coefficient and load data, one evaluation for the element points
            // and the interior edge points (sin/cos by angle addition from the centre)
            PointData pdn{};
            if (vpt || (epnt && og >= 0)) pdn = point_data_near(pr, tc, px, py, SL == 0);
            if (vpt) {
                xi = xib;
                eta = etab;
                pc.a0 = T(W * bx.cx * bx.cx * pdn.a);
                pc.a1 = T(W * bx.cy * bx.cy * pdn.a);
                if (ADV) {
                    pc.c0 = T(W * pr.bx * bx.cx);
                    pc.c1 = T(W * pr.by * bx.cy);
                    pc.c2 = T(W * pr.c);
                }
                pc.r2 = T(W * pdn.f);
            } else if (vol) {
                // reduced rule: node q of the element's accepted rule (box coordinates)
                xi = A.qr_nodes[(int64_t)c * 2 * kQrNodes + 2 * q];
                eta = A.qr_nodes[(int64_t)c * 2 * kQrNodes + 2 * q + 1];
                const double W = A.qr_w[(int64_t)c * kQrNodes + q] * 0.25 * R.hx * R.hy;
                const double a = coef_a_near(pr, tc, bx.mx + xi / bx.cx, bx.my + eta / bx.cy);
                pc.a0 = T(W * bx.cx * bx.cx * a);
                pc.a1 = T(W * bx.cy * bx.cy * a);
                if (ADV) {
                    pc.c0 = T(W * pr.bx * bx.cx);
                    pc.c1 = T(W * pr.by * bx.cy);
                    pc.c2 = T(W * pr.c);
                }
            } else if (epnt) {
                const double w = W;
                const double cnx = bx.cx * nx, cny = bx.cy * ny;
                xi = xib;
                eta = etab;
                if (og >= 0) {
                    double sigma = pr.c_sigma * (R.pen_r > pen_o ? R.pen_r : pen_o);
                    if (pr.penalty == 1) {
                        const int F = m.cell_face[R.s0 + fk];
                        sigma = pr.c_sigma * flen * fmax(A.pen_face[2 * F], A.pen_face[2 * F + 1]);
                    }
                    const double ha = -0.5 * w * pdn.a, hs = (sigma - up) * w;
                    pc.b0 = T(ha * cnx);
                    pc.b1 = T(ha * cny);
                    pc.c0 = T(ha * cnx);
                    pc.c1 = T(ha * cny);
                    pc.c2 = T(hs);
                    pc.x0 = T(ha * bo.cx * nx);
                    pc.x1 = T(ha * bo.cy * ny);
                    xin = ((rx - olox) - (ohix - rx) + 2.0 * dxq) * oihx;
                    etan = ((ry - oloy) - (ohiy - ry) + 2.0 * dyq) * oihy;
                } else if (og == -1) {
                    double sigma = pr.c_sigma * R.pen_r;
                    if (pr.penalty == 1) sigma = pr.c_sigma * flen * A.pen_face[2 * m.cell_face[R.s0 + fk]];
                    const PointData pd = point_data(pr, px, py, false);
                    const double ha = -w * pd.a, hs = (sigma - up) * w;
                    pc.b0 = T(ha * cnx);
                    pc.b1 = T(ha * cny);
                    pc.c0 = T(ha * cnx);
                    pc.c1 = T(ha * cny);
                    pc.c2 = T(hs);
                    pc.r0 = T(ha * pd.u * cnx);
                    pc.r1 = T(ha * pd.u * cny);
                    pc.r2 = T(hs * pd.u);
                } else {
                    const PointData pd = point_data(pr, px, py, false);
                    pc.r2 = T(w * pd.a * (pd.ux * nx + pd.uy * ny));
                }
            }
            Eval<T, P> ev;
            ev.at(T(xi), T(eta));
            if constexpr (C::MF) mf_element<T, P>(static_cast<T *>(R.xs), lane, ev, pc, accm);
#pragma unroll
            for (int jj = 0; jj < (C::MF || C::EL ? 0 : JS); ++jj) {
                const int j = j0 + jj;
                if (j < NB) {
                    const T t0 = fmat(pc.a0, ev.g0[j], pc.b0 * ev.v[j]);
                    const T t1 = fmat(pc.a1, ev.g1[j], pc.b1 * ev.v[j]);
                    const T t2 = fmat(pc.c0, ev.g0[j], fmat(pc.c1, ev.g1[j], pc.c2 * ev.v[j]));
#pragma unroll
                    for (int i = 0; i < NB; ++i)
                        acc[i * JS + jj] = fmat(ev.g0[i], t0, fmat(ev.g1[i], t1, fmat(ev.v[i], t2, acc[i * JS + jj])));
                }
            }
            if (SL == 0 && !C::EL) {
#pragma unroll
                for (int i = 0; i < NB; ++i)
                    acc[ED + i] = fmat(ev.g0[i], pc.r0, fmat(ev.g1[i], pc.r1, fmat(ev.v[i], pc.r2, acc[ED + i])));
            }
            if constexpr (C::EL) {
                el_test_terms<T, P, PN>(R, ev);
                if (pass_has_edges) {
                    cross_el<T, P, PN>(A, R, ev, pc, xin, etan, xsc, base, d, og, gvoff, fk);
                    wave_sync();  // cross entries read before the trial rows are rewritten
                }
                elem_el<T, P, PN>(R, ev, pc, min(64, Qtot - base), false, acc_e);
            } else if constexpr (C::XL) {
                if (pass_has_edges) cross_lds<T, P, PN>(A, R, ev, pc, xin, etan, xsc, base, d, og, gvoff, fk);
            } else if constexpr (C::CM) {
                if (pass_has_edges) cross_mf<T, P, PN>(A, R, ev, pc, xin, etan, xsc, base, d, og, gvoff, fk, nbo);
            } else if (pass_has_edges) {
                // cross block, one column at a time: the group's lanes sum the column
                // (butterfly inside the group) and lane gq writes the entries i = gq mod FG
                T Lx[PN + 1], dLx[PN + 1], Ly[PN + 1], dLy[PN + 1];
                legendre<T, PN>(T(xin), Lx, dLx);
                legendre<T, PN>(T(etan), Ly, dLy);
                T *dst = vals + R.pre_v + gvoff;
                const bool wr = cross && fk >= 0;
                // trial columns of the neighbour's block: all of them, in slices of the row's width
                constexpr int NSX = (C::NBN + JS - 1) / JS;
#pragma unroll
                for (int sx = (SL < NSX ? SL : NSX); sx < (SL + 1 < C::NSL ? SL + 1 : NSX); ++sx)
#pragma unroll
                for (int jj = 0; jj < JS; ++jj) {
                    const int j = sx * JS + jj;
                    if (j < C::NBN && j < nbo) {
                        const T vj = Lx[exp_a(j)] * Ly[exp_b(j)];
                        const T gj0 = dLx[exp_a(j)] * Ly[exp_b(j)], gj1 = Lx[exp_a(j)] * dLy[exp_b(j)];
                        const T u0 = -pc.b0 * vj, u1 = -pc.b1 * vj;
                        const T u2 = fmat(pc.x0, gj0, fmat(pc.x1, gj1, -pc.c2 * vj));
                        T col[NB];
#pragma unroll
                        for (int i = 0; i < NB; ++i) col[i] = fmat(ev.g0[i], u0, fmat(ev.g1[i], u1, ev.v[i] * u2));
#pragma unroll
                        for (int i = 0; i < NB; ++i) col[i] = group_sum<FG>(col[i]);
                        if (wr) {
                            const T csc = T(kNorm[j] * xsc);
#pragma unroll
                            for (int i = 0; i < NB; ++i)
                                if (i % FG == gq) {
                                    const T v = col[i] * T(kNorm[i]) * csc;
                                    if (d == 0)
                                        dst[i * nbo + j] = v;
                                    else
                                        dst[i * nbo + j] += v;
                                }
                        }
                    }
                }
            }
        }
    }
    // load-only points of rows with a reduced rule (fan sub-triangles)
    if constexpr (C::EL) {
        for (int base = 0; base < R.QR; base += 64) {
            const int q = base + lane;
            const bool in = q < R.QR;
            const int tri = in ? q / C::NQT : 0;
            const double X0 = R.x0, Y0 = R.y0;
            const double X1 = __shfl(ex, tri + 1, 64), Y1 = __shfl(ey, tri + 1, 64);
            const double X2 = __shfl(ex, tri + 2, 64), Y2 = __shfl(ey, tri + 2, 64);
            PointCoef<T> pc;
            pc.zero();
            double xi = 0.0, eta = 0.0;
            if (in) {
                const int qi = q - tri * C::NQT;
                const double area = 0.5 * ((X1 - X0) * (Y2 - Y0) - (X2 - X0) * (Y1 - Y0));
                const double l1 = R_::l(3 * qi + 1), l2 = R_::l(3 * qi + 2);
                const double dxq = l1 * (X1 - X0) + l2 * (X2 - X0), dyq = l1 * (Y1 - Y0) + l2 * (Y2 - Y0);
                const PointData pd = point_data_near(pr, tc, X0 + dxq, Y0 + dyq, true);
                pc.r2 = T(R_::w(qi) * area * pd.f);
                xi = ((X0 - R.lox) - (R.hix - X0) + 2.0 * dxq) * R.ihx;
                eta = ((Y0 - R.loy) - (R.hiy - Y0) + 2.0 * dyq) * R.ihy;
            }
            Eval<T, P> ev;
            ev.at(T(xi), T(eta));
            el_test_terms<T, P, PN>(R, ev);
            elem_el<T, P, PN>(R, ev, pc, min(64, R.QR - base), true, acc_e);
        }
    } else if (SL == 0) {
        for (int base = 0; base < R.QR; base += 64) {
            const int q = base + lane;
            const int tri = q < R.QR ? q / C::NQT : 0;
            const double X0 = R.x0, Y0 = R.y0;
            const double X1 = __shfl(ex, tri + 1, 64), Y1 = __shfl(ey, tri + 1, 64);
            const double X2 = __shfl(ex, tri + 2, 64), Y2 = __shfl(ey, tri + 2, 64);
            if (q < R.QR) {
                const int qi = q - tri * C::NQT;
                const double area = 0.5 * ((X1 - X0) * (Y2 - Y0) - (X2 - X0) * (Y1 - Y0));
                const double l1 = R_::l(3 * qi + 1), l2 = R_::l(3 * qi + 2);
                const double dxq = l1 * (X1 - X0) + l2 * (X2 - X0), dyq = l1 * (Y1 - Y0) + l2 * (Y2 - Y0);
                const double px = X0 + dxq, py = Y0 + dyq;
                const PointData pd = point_data_near(pr, tc, px, py, true);
                const T wf = T(R_::w(qi) * area * pd.f);
                T Lx[P + 1], dLx[P + 1], Ly[P + 1], dLy[P + 1];
                legendre<T, P>(T(((X0 - R.lox) - (R.hix - X0) + 2.0 * dxq) * R.ihx), Lx, dLx);
                legendre<T, P>(T(((Y0 - R.loy) - (R.hiy - Y0) + 2.0 * dyq) * R.ihy), Ly, dLy);
#pragma unroll
                for (int i = 0; i < NB; ++i) acc[ED + i] = fmat(wf, Lx[exp_a(i)] * Ly[exp_b(i)], acc[ED + i]);
            }
        }
    }
    if constexpr (C::EL) {
        // lane e < NB (NB + 1) holds entry (i, j) = (e / (NB + 1), e mod (NB + 1)),
        // the test normalisation applied (j = NB: the load of row i)
        const int i = lane / (NB + 1), j = lane - (NB + 1) * i;
        if (lane < NB * (NB + 1)) {
            if (j < NB)
                vals[R.pre_v + R.dvoff + i * NB + j] = T(double(acc_e) * (c_norm[j] * R.isq * R.isq));
            else
                rhs[R.pre_d + i] = T(double(acc_e) * R.isq);
        }
        return;
    }
    // element block slice and load: reduce-scatter over the wave, lane e writes entry e
    WaveRS<T, 32, (SL == 0 ? C::E : ED)>::run(acc, lane);
    if (lane < ED) {
        const int i = lane / JS, j = j0 + (lane - i * JS);
        if (j < NB) vals[R.pre_v + R.dvoff + i * NB + j] = T(double(acc[0]) * (c_norm[i] * c_norm[j] * R.isq * R.isq));
    } else if (SL == 0 && lane < C::E) {
        const int i = lane - ED;
        rhs[R.pre_d + i] = T(double(acc[0]) * (c_norm[i] * R.isq));
    }
    if constexpr (C::MF) {
        const int j = lane & 15;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = mf_row<T>(lane, r);
            if (i < NB && j < NB)
                vals[R.pre_v + R.dvoff + i * NB + j] = T(double(accm[r]) * (c_norm[i] * c_norm[j] * R.isq * R.isq));
        }
    }
}

template <typename T, int P, int PN, bool MX, bool ADV, int... SL>
__device__ __forceinline__ void row_slices(const AsmArgs &A, const RowCtx &R, std::integer_sequence<int, SL...>) {
    (row_slice<T, P, PN, MX, ADV, SL>(A, R), ...);
}

}  // namespace

// MX: neighbours may have other degrees than P (up to PN); otherwise all have degree P = PN
// ALT = 1 asks the register allocator for one more wave per SIMD than the
// measured default (dgp_autotune picks between the two per degree and precision)
// Element row c of degree P in one wave (pattern row and values); wlds: the
// wave's LDS region of RowCfg<T, P, PN>::LW elements.
template <typename T, int P, int PN, bool MX, bool ADV>
__device__ __forceinline__ void row_body(const AsmArgs &A, const int c, T *wlds) {
    using C = RowCfg<T, P, PN>;
    constexpr int NB = C::NB, FG = C::FG;
    const int lane = threadIdx.x & 63;
    RowHead h;
    if (!row_head(A, c, NB, h)) return;
    const int nv = h.nv;
    const int ng = h.ng;

    const CellGeo g = A.geo[c];
    RowCtx R;
    R.bx = box_of(g);
    R.bx.mx = uniform(R.bx.mx);
    R.bx.my = uniform(R.bx.my);
    R.bx.cx = uniform(R.bx.cx);
    R.bx.cy = uniform(R.bx.cy);
    R.isq = uniform(g.isq);
    R.hx = uniform(g.hix - g.lox);
    R.hy = uniform(g.hiy - g.loy);
    R.tc = trig_centre_of(g);
    R.tc.x0 = uniform(R.tc.x0);
    R.tc.y0 = uniform(R.tc.y0);
    R.tc.sx = uniform(R.tc.sx);
    R.tc.cx = uniform(R.tc.cx);
    R.tc.sy = uniform(R.tc.sy);
    R.tc.cy = uniform(R.tc.cy);
    R.tc.near = __builtin_amdgcn_readfirstlane(R.tc.near);
    R.pen_r = uniform(g.pen);
    R.lox = uniform(g.lox);
    R.loy = uniform(g.loy);
    R.hix = uniform(g.hix);
    R.hiy = uniform(g.hiy);
    R.ihx = uniform(g.ihx);
    R.ihy = uniform(g.ihy);
    R.s0 = h.s0;
    R.red = A.reduced && A.qr_ok[c];
    R.QM = R.red ? kQrNodes : (nv - 2) * C::NQT;  // points of the element matrix
    R.QF0 = (R.QM + FG - 1) / FG * FG;            // edge groups start here
    R.Qtot = R.QF0 + FG * ng;
    R.n2 = 0;
    R.gtab = h.gtab;
    if constexpr (C::VU) {
        // the groups that need 8 lanes (more than 4 Gauss points: a degree-4
        // neighbour) first, each in loop order; the others after them
        const bool lead = (h.gmask >> lane) & 1ull;
        const int po = (lead && h.o >= 0) ? (int)A.m.cell_p[h.o] : P;
        const bool wide = lead && (P > po ? P : po) + 1 > 4;
        const uint64_t m2 = __ballot(wide), m1 = h.gmask & ~m2;
        const int n2 = __popcll(m2);
        const uint64_t below = (1ull << lane) - 1ull;
        const int gidx = wide ? __popcll(m2 & below) : n2 + __popcll(m1 & below);
        const int dst = lead ? gidx : ng + (lane - __popcll(h.gmask & below));
        R.gtab = __builtin_amdgcn_ds_permute(dst << 2, lane);
        R.n2 = n2;
        R.Qtot = R.QF0 + 4 * (2 * n2 + (ng - n2));
    }
    R.QR = R.red ? (nv - 2) * C::NQT : 0;         // load-only points (reduced rule)
    R.lane = lane;
    R.c = c;
    R.nv = nv;
    R.vid = h.vid;
    R.o = h.o;
    R.voff = h.voff;
    R.dvoff = h.dvoff;
    R.maxdup = h.maxdup;
    R.ng = ng;
    R.xs = C::LW > 0 ? wlds : nullptr;
    R.gmask = h.gmask;
    R.ex = h.ex;
    R.ey = h.ey;
    R.x0 = readlane_d(h.ex, 0);
    R.y0 = readlane_d(h.ey, 0);
    R.pre_v = h.pre_v;
    R.pre_d = h.pre_d;
    row_slices<T, P, PN, MX, ADV>(A, R, std::make_integer_sequence<int, C::NSL>{});
}

template <typename T, int P, int PN, bool MX, bool ADV, int ALT>
__global__ void __launch_bounds__(256, (RowCfg<T, P, PN>::MINW + ALT)) k_row2d(AsmArgs A) {
    using C = RowCfg<T, P, PN>;
    __shared__ T xlds[C::LW > 0 ? 4 * C::LW : 1];
    // the row index is uniform across the wave: keep it (and what derives from it) in scalar registers
    const int wid = xcd_block(blockIdx.x, gridDim.x) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wid >= A.n_rows) return;
    const int c = A.rows ? __builtin_amdgcn_readfirstlane(A.rows[wid]) : wid;
    row_body<T, P, PN, MX, ADV>(A, c, xlds + (threadIdx.x >> 6) * C::LW);
}

// One persistent launch over the rows of every degree of a mixed-degree mesh:
// A.rows lists them bin by bin, (degree, fan sub-triangle count) descending,
// so the costliest rows start first; wave w of the grid takes items w,
// w + W, w + 2W, ... (W waves in the grid) and dispatches on the row's degree
// to the same per-degree body as k_row2d (identical arithmetic per row).  No
// queue counter: the assignment is static, so the launch needs no reset and
// every wave exits after its last item.
template <typename T, int P>
constexpr int lw_mixed() {
    return RowCfg<T, P, kMaxP>::LW;
}
template <typename T>
constexpr int lw_fused() {
    constexpr int a = lw_mixed<T, 1>(), b = lw_mixed<T, 2>(), c = lw_mixed<T, 3>(), d = lw_mixed<T, 4>();
    constexpr int ab = a > b ? a : b, cd = c > d ? c : d;
    // FP32: also the FP32 row body's table (rows of degree <= 2)
    constexpr int e = sizeof(T) == 4 ? F32Cfg<2, true>::LW : 0;
    constexpr int abcd = ab > cd ? ab : cd;
    return abcd > e ? abcd : e;
}

template <typename T, bool ADV>
__global__ void __launch_bounds__(256) k_row2d_fused(AsmArgs A) {
    constexpr int LW = lw_fused<T>();
    __shared__ T xlds[4 * (LW > 0 ? LW : 1)];
    T *wlds = xlds + (threadIdx.x >> 6) * LW;
    const int w0 = blockIdx.x * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int nw = gridDim.x * 4;
    for (int it = w0; it < A.n_rows; it += nw) {
        const int c = __builtin_amdgcn_readfirstlane(A.rows[it]);
        const int p = __builtin_amdgcn_readfirstlane((int)A.m.cell_p[c]);
        // FP32 rows of degree <= 2 with the plain rules and the sine solution: the
        // body of the FP32 row kernel (row_f32.h), as their per-degree launch runs them
        constexpr bool F32 = sizeof(T) == 4;
        if (p == 4)
            row_body<T, 4, kMaxP, true, ADV>(A, c, wlds);
        else if (p == 3)
            row_body<T, 3, kMaxP, true, ADV>(A, c, wlds);
        else if (p == 2) {
            if constexpr (F32) {
                if (!A.reduced && A.pr.u_kind == 0)
                    row_f32<2, ADV, true>(A, c, wlds);
                else
                    row_body<T, 2, kMaxP, true, ADV>(A, c, wlds);
            } else {
                row_body<T, 2, kMaxP, true, ADV>(A, c, wlds);
            }
        } else {
            if constexpr (F32) {
                if (!A.reduced && A.pr.u_kind == 0)
                    row_f32<1, ADV, true>(A, c, wlds);
                else
                    row_body<T, 1, kMaxP, true, ADV>(A, c, wlds);
            } else {
                row_body<T, 1, kMaxP, true, ADV>(A, c, wlds);
            }
        }
        wave_sync();  // the next row reuses the wave's LDS region
    }
}

template <typename T, int P, int PN, bool MX>
static void launch_row(const AsmArgs &a, int alt, hipStream_t st) {
    const bool adv = a.pr.bx != 0.0 || a.pr.by != 0.0 || a.pr.c != 0.0;
    const int nb = (a.n_rows + 3) / 4;
    if (nb <= 0) return;
    if (adv) {
        if (alt)
            hipLaunchKernelGGL((k_row2d<T, P, PN, MX, true, 1>), dim3(nb), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_row2d<T, P, PN, MX, true, 0>), dim3(nb), dim3(256), 0, st, a);
    } else {
        if (alt)
            hipLaunchKernelGGL((k_row2d<T, P, PN, MX, false, 1>), dim3(nb), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_row2d<T, P, PN, MX, false, 0>), dim3(nb), dim3(256), 0, st, a);
    }
}

template <typename T, bool ADV>
static void launch_fused_t(const AsmArgs &a, hipStream_t st) {
    // as many work-groups as stay resident at once (the loop does the rest)
    static int blocks = 0;
    if (blocks == 0) {
        int dev = 0, per_cu = 0, n_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_row2d_fused<T, ADV>, 256, 0) != hipSuccess ||
            per_cu < 1 || n_cu < 1) {
            per_cu = 1;
            n_cu = 256;
        }
        blocks = per_cu * n_cu;
    }
    const int need = (a.n_rows + 3) / 4;
    hipLaunchKernelGGL((k_row2d_fused<T, ADV>), dim3(blocks < need ? blocks : need), dim3(256), 0, st, a);
}

void launch_row2d_fused(const AsmArgs &a, int precision, hipStream_t st) {
    if (a.n_rows <= 0) return;
    const bool adv = a.pr.bx != 0.0 || a.pr.by != 0.0 || a.pr.c != 0.0;
    if (precision == 0) {
        if (adv)
            launch_fused_t<double, true>(a, st);
        else
            launch_fused_t<double, false>(a, st);
    } else {
        if (adv)
            launch_fused_t<float, true>(a, st);
        else
            launch_fused_t<float, false>(a, st);
    }
}

// Bytes of per-lane scratch (register spills) of the row kernel for these
// template arguments; the tuner leaves configurations that spill untried.
template <typename T, int P, int PN, bool MX>
static size_t spill_bytes(int alt, bool adv) {
    hipFuncAttributes fa;
    const void *f = adv ? (alt ? (const void *)k_row2d<T, P, PN, MX, true, 1> : (const void *)k_row2d<T, P, PN, MX, true, 0>)
                        : (alt ? (const void *)k_row2d<T, P, PN, MX, false, 1> : (const void *)k_row2d<T, P, PN, MX, false, 0>);
    if (hipFuncGetAttributes(&fa, f) != hipSuccess) return 0;
    return fa.localSizeBytes;
}

size_t row2d_spill_bytes(const AsmArgs &a, int precision, int p, bool mixed, int alt) {
    const bool adv = a.pr.bx != 0.0 || a.pr.by != 0.0 || a.pr.c != 0.0;
    if (row2d_f32_applies(a, precision, p)) return row2d_f32_spill_bytes(p, mixed, alt, adv);
#define DGP_SP(T, PP) \
    if (p == PP) return mixed ? spill_bytes<T, PP, kMaxP, true>(alt, adv) : spill_bytes<T, PP, PP, false>(alt, adv);
    if (precision == 0) {
        DGP_SP(double, 1) DGP_SP(double, 2) DGP_SP(double, 3) DGP_SP(double, 4)
    } else {
        DGP_SP(float, 1) DGP_SP(float, 2) DGP_SP(float, 3) DGP_SP(float, 4)
    }
#undef DGP_SP
    return 0;
}

bool launch_row2d(const AsmArgs &a, int precision, int p, bool mixed, int alt, hipStream_t st) {
    if (row2d_f32_applies(a, precision, p)) {
        launch_row2d_f32(a, p, mixed, alt, st);
        return true;
    }
#define DGP_ROW(T, PP)                                      \
    if (p == PP) {                                          \
        if (mixed)                                          \
            launch_row<T, PP, kMaxP, true>(a, alt, st);     \
        else                                                \
            launch_row<T, PP, PP, false>(a, alt, st);       \
        return true;                                        \
    }
    if (precision == 0) {
        DGP_ROW(double, 1) DGP_ROW(double, 2) DGP_ROW(double, 3) DGP_ROW(double, 4)
    } else {
        DGP_ROW(float, 1) DGP_ROW(float, 2) DGP_ROW(float, 3) DGP_ROW(float, 4)
    }
#undef DGP_ROW
    return false;
}

}  // namespace dgp
