// 3D SIPG assembly on polyhedra, one wave per element row (row-owner form,
// no atomics).  The row's cell is a union of tetrahedra; its faces are
// triangles, grouped by neighbour by the preparation kernel.
//
// Element term (first line of eq. dg-bilinear, constant a, b, c) and load
// (eq. dg-linear).  Lanes take the cell's tetrahedra and the 11 points of the
// degree-4 rule on each.  Every integrand of the element block is a
// polynomial in the box coordinates xi of degree <= 2p, so instead of the
// n_b x n_b block the lanes accumulate, in FP64, the Legendre moments
//     M_k = sum_q w_q P_k1(xi_q) P_k2(eta_q) P_k3(zeta_q),   |k| <= MDEG,
// with MDEG = 2p - 2 (diffusion only), 2p - 1 (with advection) or 2p (with
// reaction), plus the load moments sum_q w_q f(x_q) P_a P_b P_c of the basis
// exponents.  This is the same quadrature sum regrouped: the products of
// basis functions (and derivatives) are expanded in tensor Legendre
// polynomials with the one-dimensional linearisation coefficients c_lin, and
//     D_ij = s_i s_j sum_k M_k [ a sum_d (2/h_d)^2 L''_d + sum_d b_d (2/h_d) L'_d + c L ]_ij,k.
//
// Face terms (the face lines of both equations).  Lanes take the points of
// the 6-point degree-4 rule on the group's triangles, evaluate the row's basis
// (and the neighbour's, for interior groups) in T and add rank-2 updates,
//     D_ij += u_i (hs u_j + ha g_j) + g_i (ha u_j)          (symmetric, packed)
//     X_ij += u_i (ha g'_j - hs v_j) - g_i (ha v_j)
//     F_i  += g_i (ha g_D) + u_i (hs g_D)                   (Dirichlet)
//     F_i  += u_i w g_N                                      (Neumann)
// with u, g = n . grad (unnormalised basis values and normal derivatives of
// the row), v, g' the neighbour's, w the point weight, theta = 1/2 inside
// and 1 on the boundary, ha = -w theta a, hs = w (sigma - [b.n < 0] b.n).
// A reduce-scatter over the wave leaves entry e of a sum in lane e: each
// cross block is written after its group; the face part of the diagonal block
// and of the load after the last group, added to the element part.  The basis
// normalisation s_i s'_j is applied to the finished sums in FP64.
#include <type_traits>
#include <utility>

#include "dgp3d.h"
#include "kernels.h"
#include "rules_data.h"
#include "wave.h"

namespace dgp {

namespace {

// Coefficient of P_k in P_a P_b (t = 0), P_a' P_b (t = 1), P_a' P_b' (t = 2)
// on [-1, 1], for a, b <= 2 and k <= 4, from the power forms of P_0..P_4 and
// c_k = (2k + 1)/2 int_{-1}^{1} f P_k.
struct Lin1D {
    double v[3][3][3][5];
};
constexpr Lin1D make_lin() {
    const double pw[5][5] = {{1, 0, 0, 0, 0}, {0, 1, 0, 0, 0}, {-0.5, 0, 1.5, 0, 0}, {0, -1.5, 0, 2.5, 0},
                             {0.375, 0, -3.75, 0, 4.375}};
    const double dpw[3][5] = {{0, 0, 0, 0, 0}, {1, 0, 0, 0, 0}, {0, 3, 0, 0, 0}};
    Lin1D L{};
    for (int t = 0; t < 3; ++t)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double f[9] = {};
                for (int i = 0; i < 5; ++i)
                    for (int j = 0; j < 5; ++j) {
                        const double fa = t >= 1 ? (i < 5 ? dpw[a][i] : 0.0) : pw[a][i];
                        const double fb = t == 2 ? dpw[b][j] : pw[b][j];
                        f[i + j] += fa * fb;
                    }
                for (int k = 0; k < 5; ++k) {
                    double s = 0.0;
                    for (int i = 0; i < 9; ++i)
                        for (int l = 0; l < 5; ++l)
                            if ((i + l) % 2 == 0) s += f[i] * pw[k][l] * 2.0 / (i + l + 1);
                    L.v[t][a][b][k] = 0.5 * (2 * k + 1) * s;
                }
            }
    return L;
}
__constant__ Lin1D c_lin = make_lin();

// sqrt((2a+1)(2b+1)(2c+1)) of basis function i
__constant__ double c_norm3[10] = {1.0,
                                   1.7320508075688772935,
                                   1.7320508075688772935,
                                   1.7320508075688772935,
                                   2.2360679774997896964,
                                   3.0,
                                   3.0,
                                   2.2360679774997896964,
                                   3.0,
                                   2.2360679774997896964};

// Tensor Legendre indices (k1, k2, k3) with k1 + k2 + k3 <= D, graded.
template <int D>
struct MomIdx {
    static constexpr int N = (D + 1) * (D + 2) * (D + 3) / 6;
    int k[N][3];
};
template <int D>
constexpr MomIdx<D> make_mom() {
    MomIdx<D> r{};
    int n = 0;
    for (int t = 0; t <= D; ++t)
        for (int a = t; a >= 0; --a)
            for (int b = t - a; b >= 0; --b) {
                r.k[n][0] = a;
                r.k[n][1] = b;
                r.k[n][2] = t - a - b;
                ++n;
            }
    return r;
}

// the same indices for degree <= 4 as a table (graded, so degree <= D is a prefix)
constexpr MomIdx<4> kMom4 = make_mom<4>();
__constant__ MomIdx<4> c_mom4 = kMom4;

// packed upper-triangle index of (i <= j) in an n x n symmetric block
__host__ __device__ constexpr int pk(int n, int i, int j) { return i * n - i * (i - 1) / 2 + (j - i); }

// wavefront sum of the ROCm device library (DPP; declared by HIP's headers only
// under HIP_ENABLE_EXTRA_WARP_SYNC_TYPES)
extern "C" __device__ __attribute__((const)) double __ockl_wfred_add_f64(double);
__device__ __forceinline__ double wave_sum(double v) { return __ockl_wfred_add_f64(v); }

// Manufactured data in 3D (constant a): u, grad u and f = -a lap u + b . grad u + c u
struct Trig3 {
    double x0[3], s[3], c[3];
    bool near;
};
__device__ __forceinline__ void exact3(const DevProblem &pr, const Trig3 &t, const double *x, double *u, double *gu,
                                       double *f) {
    double lap;
    if (pr.u_kind == 0) {
        double s[3], c[3];
        for (int d = 0; d < 3; ++d) {
            if (t.near)
                sincospi_near(t.s[d], t.c[d], x[d] - t.x0[d], &s[d], &c[d]);
            else
                sincospi(x[d], &s[d], &c[d]);
        }
        *u = s[0] * s[1] * s[2];
        gu[0] = kPi * c[0] * s[1] * s[2];
        gu[1] = kPi * s[0] * c[1] * s[2];
        gu[2] = kPi * s[0] * s[1] * c[2];
        lap = -3.0 * kPi * kPi * (*u);
    } else {
        // read here at an offset (zero) hidden from the compiler, so that the ten
        // coefficients are not hoisted into scalar registers for the whole kernel
        int z;
        asm volatile("s_mov_b32 %0, 0" : "=s"(z));
        const double *q = pr.u + z;
        *u = q[0] + q[1] * x[0] + q[2] * x[1] + q[3] * x[2] + q[4] * x[0] * x[0] + q[5] * x[1] * x[1] +
             q[6] * x[2] * x[2] + q[7] * x[0] * x[1] + q[8] * x[0] * x[2] + q[9] * x[1] * x[2];
        gu[0] = q[1] + 2 * q[4] * x[0] + q[7] * x[1] + q[8] * x[2];
        gu[1] = q[2] + 2 * q[5] * x[1] + q[7] * x[0] + q[9] * x[2];
        gu[2] = q[3] + 2 * q[6] * x[2] + q[8] * x[0] + q[9] * x[1];
        lap = 2 * (q[4] + q[5] + q[6]);
    }
    if (f) *f = -pr.a0 * lap + pr.bx * gu[0] + pr.by * gu[1] + pr.bz * gu[2] + pr.c * (*u);
}

// The load f alone at a volume point.  Without advection f = (3 pi^2 a + c) u
// for the sine solution, so no gradient is formed.  SHORT: sin/cos(pi d) near
// the centre from their series through t^7 / t^8 (|t| <= 0.2: truncation below
// 2e-12), enough for the FP32 kernels; otherwise as exact3.
template <bool SHORT>
__device__ __forceinline__ double load3(const DevProblem &pr, const Trig3 &t, const double *x) {
    if (pr.u_kind != 0 || !t.near) {
        double u, gu[3], f;
        exact3(pr, t, x, &u, gu, &f);
        return f;
    }
    double s[3], c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        if (SHORT) {
            const double tt = kPi * (x[d] - t.x0[d]), t2 = tt * tt;
            const double st = tt * (1.0 + t2 * (-1.0 / 6 + t2 * (1.0 / 120 + t2 * (-1.0 / 5040))));
            const double ct = 1.0 + t2 * (-0.5 + t2 * (1.0 / 24 + t2 * (-1.0 / 720 + t2 * (1.0 / 40320))));
            s[d] = t.s[d] * ct + t.c[d] * st;
            c[d] = t.c[d] * ct - t.s[d] * st;
        } else {
            sincospi_near(t.s[d], t.c[d], x[d] - t.x0[d], &s[d], &c[d]);
        }
    }
    const double u = s[0] * s[1] * s[2];
    if (pr.bx == 0.0 && pr.by == 0.0 && pr.bz == 0.0) return (3.0 * kPi * kPi * pr.a0 + pr.c) * u;
    const double g0 = kPi * c[0] * s[1] * s[2], g1 = kPi * s[0] * c[1] * s[2], g2 = kPi * s[0] * s[1] * c[2];
    return 3.0 * kPi * kPi * pr.a0 * u + pr.bx * g0 + pr.by * g1 + pr.bz * g2 + pr.c * u;
}

// unnormalised basis values u_i = P_a P_b P_c and normal derivatives
// g_i = sum_d nc_d d/dxi_d (P_a P_b P_c), nc_d = n_d (2 / h_d), of the first N
// functions (degree <= 2: P_1 = t, P_2 = (3t^2 - 1)/2, P_2' = 3t)
template <typename T, int N>
__device__ __forceinline__ void basis3(const T *xi, const T *nc, T *u, T *g) {
    static_assert(N == 1 || N == 4 || N == 10, "degree <= 2");
    const T x = xi[0], y = xi[1], z = xi[2];
    u[0] = T(1);
    g[0] = T(0);
    if (N > 1) {
        u[1] = x;
        u[2] = y;
        u[3] = z;
        g[1] = nc[0];
        g[2] = nc[1];
        g[3] = nc[2];
    }
    if (N > 4) {
        u[4] = T(1.5) * x * x - T(0.5);
        u[5] = x * y;
        u[6] = x * z;
        u[7] = T(1.5) * y * y - T(0.5);
        u[8] = y * z;
        u[9] = T(1.5) * z * z - T(0.5);
        g[4] = T(3) * x * nc[0];
        g[5] = nc[0] * y + nc[1] * x;
        g[6] = nc[0] * z + nc[2] * x;
        g[7] = T(3) * y * nc[1];
        g[8] = nc[1] * z + nc[2] * y;
        g[9] = T(3) * z * nc[2];
    }
}

// A face triangle as seen from cell c: first vertex, edges, unit normal out of
// c and area.  One lane computes it (one chain of dependent loads per face)
// and stores it in LDS, where the six lanes of its points read it.
struct FaceLds {
    double p0[3], e1[3], e2[3], n[3], area;
    double pen, theta;  // the face group's penalty and consistency factor (diagonal sweep)
    int code;           // neighbour id, or -1 Dirichlet, -2 Neumann (diagonal sweep)
};
__device__ __forceinline__ void face_stage(const DevMesh &m, int c, int F, FaceLds &f) {
    const int iv0 = m.face_vtx[3 * F], iv1 = m.face_vtx[3 * F + 1], iv2 = m.face_vtx[3 * F + 2];
    const int io = m.face_opp[F];
    const bool left = m.face_cell[2 * F] == c;
    const double p0[3] = {m.x[iv0], m.y[iv0], m.z[iv0]};
    const double p1[3] = {m.x[iv1], m.y[iv1], m.z[iv1]};
    const double p2[3] = {m.x[iv2], m.y[iv2], m.z[iv2]};
    const double po[3] = {m.x[io], m.y[io], m.z[io]};
    const double e1[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
    const double e2[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
    const double cr[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double len = sqrt(cr[0] * cr[0] + cr[1] * cr[1] + cr[2] * cr[2]);
    // the left cell's outward normal points away from its tetrahedron's opposite vertex
    double sg = (cr[0] * (po[0] - p0[0]) + cr[1] * (po[1] - p0[1]) + cr[2] * (po[2] - p0[2])) > 0.0 ? -1.0 : 1.0;
    if (!left) sg = -sg;
    const double il = sg / len;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        f.p0[d] = p0[d];
        f.e1[d] = e1[d];
        f.e2[d] = e2[d];
        f.n[d] = cr[d] * il;
    }
    f.area = 0.5 * len;
}

// A face group of the row with what its points need: the neighbour's box
// factors, the penalty, the range in the grouped face list.  Filled once per
// row, one lane per group, so the sweeps read it from LDS instead of chains
// of dependent loads.
struct GroupLds {
    double ncx[3], nctr[3], nisq, pen;
    int start, count, code, rank_voff, nbo, pad;
};

// Point pi of the staged faces (6-point rule, face pi / 6): position, normal, weight.
struct FacePt {
    double x[3], n[3], w;
};
__device__ __forceinline__ void face_point(const FaceLds *fl, int pi, FacePt &fp) {
    const int fk = pi / DGP_TRI4_N, q = pi - DGP_TRI4_N * fk;
    const FaceLds &f = fl[fk];
    const double l1 = c_tri4_l[3 * q + 1], l2 = c_tri4_l[3 * q + 2];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        fp.x[d] = f.p0[d] + l1 * f.e1[d] + l2 * f.e2[d];
        fp.n[d] = f.n[d];
    }
    fp.w = c_tri4_w[q] * f.area;
}

// The row's box, offsets and face groups (all wave-uniform).
struct Row3 {
    int c, ng, drank, dvoff;
    int64_t fs, pre_b, pre_v, pre_d;
    double lo[3], hi[3], cx[3], ctr[3], isq;
};
__device__ __forceinline__ void row_begin(const Asm3Args &A, int c, Row3 &R) {
    const CellGeo3 &G = A.geo[c];
    R.c = c;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        R.lo[d] = G.lo[d];
        R.hi[d] = G.hi[d];
        R.cx[d] = uniform(2.0 / (R.hi[d] - R.lo[d]));
        R.ctr[d] = uniform(0.5 * (R.lo[d] + R.hi[d]));
    }
    R.isq = uniform(1.0 / G.sqrt_box);
    R.fs = A.m.cell_face_ptr[c];
    R.ng = G.n_groups;
    const int t0 = c / kPrepTile3D;
    const int4 cr = reinterpret_cast<const int4 *>(A.cnt)[c];
    R.pre_b = A.tile_off[3 * t0] + cr.x;
    R.pre_v = A.tile_off[3 * t0 + 1] + cr.y;
    R.pre_d = A.tile_off[3 * t0 + 2] + cr.z;
    R.drank = cr.w & 255;
    R.dvoff = cr.w >> 8;
}
__device__ __forceinline__ Trig3 row_trig(const CellGeo3 &G, const Row3 &R) {
    Trig3 tc;
    double r2 = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        tc.x0[d] = R.ctr[d];
        tc.s[d] = uniform(G.s[d]);
        tc.c[d] = uniform(G.c[d]);
        r2 += 0.25 * (R.hi[d] - R.lo[d]) * (R.hi[d] - R.lo[d]);
    }
    tc.near = kPi * sqrt(r2) <= kNearT;
    return tc;
}

}  // namespace

// Element part of the diagonal block and the load, written (the face kernel adds its part).
template <typename T, int P, int MDEG>
__global__ void __launch_bounds__(256, 2) k_vol3d(Asm3Args A) {
    constexpr int NB = nb3d(P);
    constexpr int MX = MDEG > P ? MDEG : P;  // Legendre degree needed at volume points
    constexpr MomIdx<MDEG> KM = make_mom<MDEG>();
    constexpr int NM = MomIdx<MDEG>::N;
    static_assert(NB * NB <= 128, "one or two entries per lane");
    __shared__ double s_mom[4][NM];

    const DevMesh &m = A.m;
    const DevProblem &pr = A.pr;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wid = xcd_block(blockIdx.x, gridDim.x) * 4 + wv;  // XCD x: one contiguous range of the row order
    if (wid >= A.n_rows) return;
    const int c = A.rows ? __builtin_amdgcn_readfirstlane(A.rows[wid]) : wid;
    Row3 R;
    row_begin(A, c, R);
    const Trig3 tc = row_trig(A.geo[c], R);
    const double *cx = R.cx, *ctr = R.ctr;
    const double isq = R.isq;

    // ---- element term: moments over the tetrahedra (FP64)
    double mom[NM], momf[NB], vol = 0.0;
#pragma unroll
    for (int k = 0; k < NM; ++k) mom[k] = 0.0;
#pragma unroll
    for (int i = 0; i < NB; ++i) momf[i] = 0.0;
    const int64_t ts = m.cell_ptr[c] >> 2;
    const int nt = (int)((m.cell_ptr[c + 1] >> 2) - ts);
    for (int t = lane; t < nt; t += 64) {
        const int4 id = reinterpret_cast<const int4 *>(m.cell_vtx)[ts + t];
        const int ids[4] = {id.x, id.y, id.z, id.w};
        double v[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            v[k][0] = m.x[ids[k]];
            v[k][1] = m.y[ids[k]];
            v[k][2] = m.z[ids[k]];
        }
        double e[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int d = 0; d < 3; ++d) e[k][d] = v[k + 1][d] - v[0][d];
        const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                           e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                           e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
        const double tv = fabs(det) / 6.0;
        vol += tv;
#pragma unroll 1
        for (int q = 0; q < DGP_TET4_N; ++q) {
            double x[3], L[3][MX + 1];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                x[d] = c_tet4_l[4 * q] * v[0][d] + c_tet4_l[4 * q + 1] * v[1][d] + c_tet4_l[4 * q + 2] * v[2][d] +
                       c_tet4_l[4 * q + 3] * v[3][d];
                const double xi = (x[d] - ctr[d]) * cx[d];
                L[d][0] = 1.0;
                if (MX >= 1) L[d][1] = xi;
#pragma unroll
                for (int n = 1; n < MX; ++n)
                    L[d][n + 1] = (double(2 * n + 1) / (n + 1)) * xi * L[d][n] - (double(n) / (n + 1)) * L[d][n - 1];
            }
            const double w = c_tet4_w[q] * tv;
            double wx[MX + 1];
#pragma unroll
            for (int k = 0; k <= MX; ++k) wx[k] = w * L[0][k];
#pragma unroll
            for (int k = 0; k < NM; ++k) mom[k] += wx[KM.k[k][0]] * (L[1][KM.k[k][1]] * L[2][KM.k[k][2]]);
            const double wf = w * load3<sizeof(T) == 4>(pr, tc, x);
#pragma unroll
            for (int i = 0; i < NB; ++i)
                momf[i] += wf * L[0][exp3(i, 0)] * L[1][exp3(i, 1)] * L[2][exp3(i, 2)];
        }
    }
#pragma unroll
    for (int k = 0; k < NM; ++k) {
        const double t = wave_sum(mom[k]);
        if (lane == 0) s_mom[wv][k] = t;
    }
    wave_sync();
#pragma unroll
    for (int i = 0; i < NB; ++i) momf[i] = wave_sum(momf[i]);
    vol = wave_sum(vol);
    if (lane == 0) const_cast<CellGeo3 *>(A.geo)[c].vol = vol;

    // element block entries e = lane, lane + 64 (row-major), FP64
    const double st[3] = {pr.a0 * cx[0] * cx[0], pr.a0 * cx[1] * cx[1], pr.a0 * cx[2] * cx[2]};
    const double ad[3] = {pr.bx * cx[0], pr.by * cx[1], pr.bz * cx[2]};
    auto entry = [&](int e) {
        const int i = e / NB, j = e % NB;
        int ie[3], je[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            ie[d] = exp3(i, d);
            je[d] = exp3(j, d);
        }
        double acc = 0.0;
#pragma unroll 1
        for (int k = 0; k < NM; ++k) {
            const int kk[3] = {c_mom4.k[k][0], c_mom4.k[k][1], c_mom4.k[k][2]};
            double m0[3], m1[3], m2[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                m0[d] = c_lin.v[0][ie[d]][je[d]][kk[d]];
                m1[d] = c_lin.v[1][je[d]][ie[d]][kk[d]];
                m2[d] = c_lin.v[2][ie[d]][je[d]][kk[d]];
            }
            const double sv = st[0] * m2[0] * m0[1] * m0[2] + st[1] * m0[0] * m2[1] * m0[2] + st[2] * m0[0] * m0[1] * m2[2];
            const double av = ad[0] * m1[0] * m0[1] * m0[2] + ad[1] * m0[0] * m1[1] * m0[2] + ad[2] * m0[0] * m0[1] * m1[2];
            acc += s_mom[wv][k] * (sv + av + pr.c * m0[0] * m0[1] * m0[2]);
        }
        return acc * c_norm3[i] * c_norm3[j] * isq * isq;
    };
    const double dvol0 = lane < NB * NB ? entry(lane) : 0.0;
    const double dvol1 = (NB * NB > 64 && lane + 64 < NB * NB) ? entry(lane + 64) : 0.0;
    double fvol = 0.0;
#pragma unroll
    for (int i = 0; i < NB; ++i)
        if (lane == i) fvol = momf[i] * c_norm3[i] * isq;


    T *vals = static_cast<T *>(A.vals);
    if (lane < NB * NB) vals[R.pre_v + R.dvoff + lane] = T(dvol0);
    if (NB * NB > 64 && lane + 64 < NB * NB) vals[R.pre_v + R.dvoff + lane + 64] = T(dvol1);
    if (lane < NB) static_cast<T *>(A.rhs)[R.pre_d + lane] = T(fvol);
}

// Pattern row (if A.write_pattern) and, with A.values, the face terms: cross
// blocks written, the face part of the diagonal block and of the load added
// to what the element kernel wrote.
template <typename T, int P>
__global__ void __launch_bounds__(256, (sizeof(T) == 4 ? 2 : 1)) k_face3d(Asm3Args A) {
    __shared__ FaceLds s_face[4][64];
    __shared__ GroupLds s_group[4][kMaxGroups3D];
    constexpr int NB = nb3d(P), NBN = nb3d(kMaxP3D);
    constexpr int NPK = NB * (NB + 1) / 2;  // packed symmetric entries
    constexpr int NXE = NB * NBN;           // cross-block entries (neighbour basis up to degree 2)
    constexpr int NCH = (NXE + 31) / 32;    // cross-block chunks of 32 entries (one per half-wave lane)
    static_assert(NCH <= 4, "at most four chunks");
    static_assert(NPK <= 64 && NB * NB <= 128, "one or two entries per lane");

    const DevMesh &m = A.m;
    const DevProblem &pr = A.pr;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int wid = xcd_block(blockIdx.x, gridDim.x) * 4 + wv;  // XCD x: one contiguous range of the row order
    if (wid >= A.n_rows) return;
    const int c = A.rows ? __builtin_amdgcn_readfirstlane(A.rows[wid]) : wid;
    Row3 R;
    row_begin(A, c, R);
    const CellGeo3 &G = A.geo[c];
    FaceLds *sf = s_face[wv];
    const double *cx = R.cx, *ctr = R.ctr;
    const double isq = R.isq;
    const int64_t fs = R.fs, pre_b = R.pre_b, pre_v = R.pre_v, pre_d = R.pre_d;
    const int ng = R.ng, drank = R.drank, dvoff = R.dvoff;
    if (A.write_pattern) {
        for (int k = lane; k < ng; k += 64) {
            const FaceGroup gr = A.grp[fs + k];
            if (gr.code >= 0) {
                A.col_idx[pre_b + (gr.rank_voff & 255)] = gr.code;
                A.val_ptr[pre_b + (gr.rank_voff & 255)] = pre_v + (gr.rank_voff >> 8);
            }
        }
        if (lane == 0) {
            A.col_idx[pre_b + drank] = c;
            A.val_ptr[pre_b + drank] = pre_v + dvoff;
            A.row_ptr[c] = pre_b;
            A.dof_ptr[c] = pre_d;
            if (c == m.n_cells - 1) {
                const int n_tiles = (m.n_cells + kPrepTile3D - 1) / kPrepTile3D;
                const int64_t nnzb = A.tile_off[3 * n_tiles];
                A.row_ptr[c + 1] = nnzb;
                A.val_ptr[nnzb] = A.tile_off[3 * n_tiles + 1];
                A.dof_ptr[c + 1] = A.tile_off[3 * n_tiles + 2];
            }
        }
    }
    if (!A.values) return;
    const Trig3 tc = row_trig(G, R);

    // ---- face terms in two sweeps over the groups, so that the cross block
    // and the diagonal block are never live together: first every interior
    // group's cross block (reduced and written after the group), then the face
    // part of the diagonal block (packed) and of the load over all groups,
    // reduced once.
    const double a = pr.a0;
    const double pen_r = uniform(G.abar * (P * P) / G.h);
    T *vals = static_cast<T *>(A.vals);
    GroupLds *sg = s_group[wv];
    for (int gi = lane; gi < ng; gi += 64) {
        const FaceGroup gr = A.grp[fs + gi];
        GroupLds e;
        e.start = gr.start;
        e.count = gr.count;
        e.code = gr.code;
        e.rank_voff = gr.rank_voff;
        e.pad = 0;
        e.pen = pr.c_sigma * pen_r;
        e.nbo = 0;
        e.nisq = 0.0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            e.ncx[d] = 1.0;
            e.nctr[d] = 0.0;
        }
        if (gr.code >= 0) {
            const CellGeo3 &Gn = A.geo[gr.code];
            const int pn = m.cell_p[gr.code];
            e.nbo = nb3d(pn);
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                e.ncx[d] = 2.0 / (Gn.hi[d] - Gn.lo[d]);
                e.nctr[d] = 0.5 * (Gn.lo[d] + Gn.hi[d]);
            }
            e.nisq = 1.0 / Gn.sqrt_box;
            e.pen = pr.c_sigma * fmax(pen_r, Gn.abar * (pn * pn) / Gn.h);
        }
        sg[gi] = e;
    }
    wave_sync();
    // Sweep A: two interior groups at a time, one per half-wave (lanes 0-31 and
    // 32-63), so the reduce-scatter of a cross block runs over 32 lanes and two
    // blocks share each reduction step.  Interior groups come first in a row's
    // group list (neighbours ascending), boundary groups last.
    int n_in = 0;
    while (n_in < ng && A.grp[fs + n_in].code >= 0) ++n_in;
    const int h = lane >> 5, hl = lane & 31;
    FaceLds *sfh = sf + 32 * h;
    for (int gp = 0; gp < n_in; gp += 2) {
        const int gi = gp + h;
        const bool gvalid = gi < n_in;
        const GroupLds &gg = sg[gvalid ? gi : gp];
        const int nbo = gg.nbo;
        double ncx[3], nctr[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            ncx[d] = gg.ncx[d];
            nctr[d] = gg.nctr[d];
        }
        const double nisq = gg.nisq;
        const double pen = gg.pen;
        const int gstart = gg.start, grank_voff = gg.rank_voff;
        const int cnt = gvalid ? gg.count : 0;
        const int cmax = max(__builtin_amdgcn_readlane(cnt, 0), __builtin_amdgcn_readlane(cnt, 32));
        T xa[NCH][64];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int k = 0; k < 32; ++k) xa[ch][k] = T(0);
        for (int f0 = 0; f0 < cmax; f0 += 32) {
            const int nfc = min(32, cnt - f0);
            if (hl < nfc) face_stage(m, c, A.forder[fs + gstart + f0 + hl], sfh[hl]);
            wave_sync();
            for (int pi = hl; pi < DGP_TRI4_N * nfc; pi += 32) {
                FacePt fp;
                face_point(sfh, pi, fp);
                const double bn = pr.bx * fp.n[0] + pr.by * fp.n[1] + pr.bz * fp.n[2];
                const T tha = T(-fp.w * 0.5 * a), ths = T(fp.w * (pen - (bn < 0.0 ? bn : 0.0)));
                T xi[3], nc[3], u[NB], g[NB], v[NBN], gv[NBN];
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    xi[d] = T((fp.x[d] - ctr[d]) * cx[d]);
                    nc[d] = T(fp.n[d] * cx[d]);
                }
                basis3<T, NB>(xi, nc, u, g);
#pragma unroll
                for (int d = 0; d < 3; ++d) {
                    xi[d] = T((fp.x[d] - nctr[d]) * ncx[d]);
                    nc[d] = T(fp.n[d] * ncx[d]);
                }
                basis3<T, NBN>(xi, nc, v, gv);
                // X_ij += u_i (ha g'_j - hs v_j) + g_i (-ha v_j)   (u_0 = 1, g_0 = 0)
#pragma unroll
                for (int j = 0; j < NBN; ++j) {
                    const T tx = tha * gv[j] - ths * v[j];
                    const T ux = -tha * v[j];
#pragma unroll
                    for (int i = 0; i < NB; ++i) {
                        const int e = i * NBN + j;
                        T &acc = xa[e / 32][e % 32];
                        if (i == 0) {
                            acc += tx;
                        } else {
                            acc = fma(u[i], tx, acc);
                            acc = fma(g[i], ux, acc);
                        }
                    }
                }
            }
            wave_sync();
        }
        // entry e = 32 ch + (lane & 31) of the degree-2 neighbour basis; the
        // neighbour's first nbo functions are its basis of degree p_n
        auto reduce_write = [&](auto chc) {
            constexpr int ch = decltype(chc)::value;
            if constexpr (ch < NCH) {
                WaveRS<T, 16, (NXE - 32 * ch < 32 ? NXE - 32 * ch : 32)>::run(xa[ch], lane);
                const int e = 32 * ch + hl;
                if (gvalid && e < NXE) {
                    const int i = e / NBN, j = e % NBN;
                    if (j < nbo)
                        vals[pre_v + (grank_voff >> 8) + i * nbo + j] =
                            T(double(xa[ch][0]) * (c_norm3[i] * isq) * (c_norm3[j] * nisq));
                }
            }
        };
        reduce_write(std::integral_constant<int, 0>{});
        reduce_write(std::integral_constant<int, 1>{});
        reduce_write(std::integral_constant<int, 2>{});
        reduce_write(std::integral_constant<int, 3>{});
    }

    // Sweep B: the face part of the diagonal block and of the load, over the
    // row's faces in chunks of 64 regardless of group boundaries (each staged
    // face carries its group's penalty, weight factor and boundary code).
    T dp[64], rf[64];
#pragma unroll
    for (int k = 0; k < NPK; ++k) dp[k] = T(0);
#pragma unroll
    for (int k = 0; k < NB; ++k) rf[k] = T(0);
    const int nfr = (int)(m.cell_face_ptr[c + 1] - fs);
    for (int f0 = 0; f0 < nfr; f0 += 64) {
        const int nfc = min(64, nfr - f0);
        const int k = f0 + lane;
        if (lane < nfc) {
            int gi = 0;  // the group holding face k (groups are consecutive ranges)
            while (gi + 1 < ng && sg[gi + 1].start <= k) ++gi;
            face_stage(m, c, A.forder[fs + k], sf[lane]);
            sf[lane].pen = sg[gi].pen;
            sf[lane].theta = sg[gi].code >= 0 ? 0.5 : 1.0;
            sf[lane].code = sg[gi].code;
        }
        wave_sync();
        for (int pi = lane; pi < DGP_TRI4_N * nfc; pi += 64) {
            FacePt fp;
            face_point(sf, pi, fp);
            const FaceLds &fl = sf[pi / DGP_TRI4_N];
            const int code = fl.code;
            const double bn = pr.bx * fp.n[0] + pr.by * fp.n[1] + pr.bz * fp.n[2];
            const double ha = -fp.w * fl.theta * a, hs = fp.w * (fl.pen - (bn < 0.0 ? bn : 0.0));
            T xi[3], nc[3], u[NB], g[NB];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                xi[d] = T((fp.x[d] - ctr[d]) * cx[d]);
                nc[d] = T(fp.n[d] * cx[d]);
            }
            basis3<T, NB>(xi, nc, u, g);
            if (code != -2) {
                // D_ij += u_i (hs u_j + ha g_j) + g_i (ha u_j), i <= j
                const T tha = T(ha), ths = T(hs);
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const T tj = ths * u[j] + tha * g[j];
                    const T sj = tha * u[j];
#pragma unroll
                    for (int i = 0; i <= j; ++i) {
                        T &acc = dp[pk(NB, i, j)];
                        if (i == 0) {
                            acc += tj;
                        } else {
                            acc = fma(u[i], tj, acc);
                            acc = fma(g[i], sj, acc);
                        }
                    }
                }
            }
            if (code < 0) {
                // boundary data with sin/cos taken directly, not by angle addition
                // from the centre: on a boundary where the manufactured u vanishes
                // (sin(pi k) = 0) the direct evaluation is exactly zero, where angle
                // addition leaves a rounding residue that the large penalty carries
                // into the load of elements whose load is itself tiny (corners)
                Trig3 tb = tc;
                tb.near = false;
                double ue, gu[3];
                exact3(pr, tb, fp.x, &ue, gu, nullptr);
                if (code == -1) {
                    const T r0 = T(ha * ue), r1 = T(hs * ue);
#pragma unroll
                    for (int i = 0; i < NB; ++i) rf[i] = fma(g[i], r0, fma(u[i], r1, rf[i]));
                } else {
                    const T gn = T(fp.w * a * (gu[0] * fp.n[0] + gu[1] * fp.n[1] + gu[2] * fp.n[2]));
#pragma unroll
                    for (int i = 0; i < NB; ++i) rf[i] = fma(u[i], gn, rf[i]);
                }
            }
        }
        wave_sync();
    }
    WaveRS<T, 32, NPK>::run(dp, lane);
    WaveRS<T, 32, NB>::run(rf, lane);
    const double dself = double(dp[0]), fself = double(rf[0]);

    // ---- face part added to the element part of the diagonal block and the load
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const int e = lane + 64 * r;
        const int ee = e < NB * NB ? e : 0;
        const int i = ee / NB, j = ee % NB;
        const int src = i <= j ? pk(NB, i, j) : pk(NB, j, i);
        const double face = __shfl(dself, src, 64);
        if (r * 64 < NB * NB && e < NB * NB) {
            T &dst = vals[pre_v + dvoff + e];
            dst = T(double(dst) + face * c_norm3[i] * c_norm3[j] * isq * isq);
        }
    }
    if (lane < NB) {
        T &dst = static_cast<T *>(A.rhs)[pre_d + lane];
        dst = T(double(dst) + fself * c_norm3[lane] * isq);
    }
}

namespace {

template <typename T, int P>
bool launch_p(const Asm3Args &a, int mdeg, hipStream_t st) {
    const dim3 grid((a.n_rows + 3) / 4), block(256);
    if (a.values) {
        if (mdeg == 2 * P - 2)
            hipLaunchKernelGGL((k_vol3d<T, P, 2 * P - 2>), grid, block, 0, st, a);
        else if (mdeg == 2 * P - 1)
            hipLaunchKernelGGL((k_vol3d<T, P, 2 * P - 1>), grid, block, 0, st, a);
        else if (mdeg == 2 * P)
            hipLaunchKernelGGL((k_vol3d<T, P, 2 * P>), grid, block, 0, st, a);
        else
            return false;
    }
    hipLaunchKernelGGL((k_face3d<T, P>), grid, block, 0, st, a);
    return true;
}

template <typename T>
bool launch_t(const Asm3Args &a, int p, int mdeg, hipStream_t st) {
    if (p == 1) return launch_p<T, 1>(a, mdeg, st);
    if (p == 2) return launch_p<T, 2>(a, mdeg, st);
    return false;
}

}  // namespace

bool launch_row3d(const Asm3Args &a, int precision, int p, hipStream_t st) {
    if (a.n_rows <= 0) return true;
    // highest Legendre degree of the element integrands: 2p - 2 (diffusion),
    // 2p - 1 (advection), 2p (reaction)
    const int mdeg = a.pr.c != 0.0 ? 2 * p : (a.pr.bx != 0.0 || a.pr.by != 0.0 || a.pr.bz != 0.0) ? 2 * p - 1 : 2 * p - 2;
    return precision == 0 ? launch_t<double>(a, p, mdeg, st) : launch_t<float>(a, p, mdeg, st);
}

}  // namespace dgp
