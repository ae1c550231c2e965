// 2D SIPG assembly, row-owner form (no floating-point atomics).
//
// A work-group owns a chunk of consecutive element rows (cut by the runtime
// so that the chunk's quadrature tasks fit the work-group).  It
//   1. gathers everything its rows need -- element geometry, loop vertices,
//      the neighbour across each edge and its geometry -- in two rounds of
//      independent loads, into LDS;
//   2. derives the exclusive prefix of its first row from the scanned tile
//      sums of the preparation kernels, and writes its rows of the block
//      pattern (Section 3.4, Approach 2: one block per distinct neighbour,
//      columns ascending);
//   3. runs the quadrature tasks of its rows, each a few points of one fan
//      sub-triangle (element term, first line of eq. dg-bilinear, and the load
//      of eq. dg-linear) or one face (the face lines of both equations),
//      written for the test functions phi_i of row r (dn = grad phi . n_r,
//      primes = the neighbour's basis, bn = b . n_r):
//        element:  D_ij += w [a grad phi_j . grad phi_i + (b . grad phi_j) phi_i + c phi_j phi_i]
//        interior: D_ij += w [-a/2 dn_j phi_i - a/2 dn_i phi_j + sigma phi_j phi_i] - [bn<0] w bn phi_j phi_i
//                  X_ij += w [-a/2 dn'_j phi_i + a/2 dn_i phi'_j - sigma phi'_j phi_i] + [bn<0] w bn phi'_j phi_i
//        boundary: D_ij += w [-a dn_j phi_i - a dn_i phi_j + sigma phi_j phi_i] - [bn<0] w bn phi_j phi_i
//                  F_i  += w [-g a dn_i + sigma g phi_i] - [bn<0] w bn g phi_i
//      keeping each task's partial blocks in LDS;
//   4. writes its rows -- a contiguous range of the value array -- with
//      consecutive lanes on consecutive entries, each entry the sum of its
//      partials in task order (deterministic).
//
// Precision: positions, Jacobians, bounding-box scaling, coefficients, the load
// and the penalty are FP64; per-point weights are formed in FP64 and rounded
// once to T.  Coefficient and load data at a point come from sin/cos at the
// element's centre by angle addition (a short series in the offset), boundary
// data from direct evaluation.  The basis is evaluated without its
// normalisation s_i = sqrt((2a+1)(2b+1)/|B|): every term is bilinear, so
// s_i s'_j is applied to the finished sum.
#include "dgp_common.h"
#include "kernels.h"
#include "rules_data.h"

namespace dgp {

namespace {

template <typename T>
__device__ __forceinline__ T fmat(T a, T b, T c) {
    return fma(a, b, c);
}

template <int DEG>
struct Tri;
template <>
struct Tri<4> {
    static constexpr int n = DGP_TRI4_N;
    __device__ static double l(int i) { return c_tri4_l[i]; }
    __device__ static double w(int i) { return c_tri4_w[i]; }
};
template <>
struct Tri<6> {
    static constexpr int n = DGP_TRI6_N;
    __device__ static double l(int i) { return c_tri6_l[i]; }
    __device__ static double w(int i) { return c_tri6_w[i]; }
};
template <>
struct Tri<8> {
    static constexpr int n = DGP_TRI8_N;
    __device__ static double l(int i) { return c_tri8_l[i]; }
    __device__ static double w(int i) { return c_tri8_w[i]; }
};

// Basis of one element at a point, without normalisation.
template <typename T, int P>
struct Eval {
    static constexpr int NB = nb2d(P);
    T v[NB], g0[NB], g1[NB];  // P_a P_b, dP_a/dxi P_b, P_a dP_b/deta
    __device__ __forceinline__ void at(T xi, T eta) {
        T Lx[P + 1], dLx[P + 1], Ly[P + 1], dLy[P + 1];
        legendre<T, P>(xi, Lx, dLx);
        legendre<T, P>(eta, Ly, dLy);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            v[i] = Lx[exp_a(i)] * Ly[exp_b(i)];
            g0[i] = dLx[exp_a(i)] * Ly[exp_b(i)];
            g1[i] = Lx[exp_a(i)] * dLy[exp_b(i)];
        }
    }
};

struct Box {
    double mx, my, cx, cy;  // centre and chain factors 2/h of the bounding box
};

__device__ __forceinline__ Box box_of(const CellGeo &g) {
    Box b;
    b.mx = 0.5 * (g.lox + g.hix);
    b.my = 0.5 * (g.loy + g.hiy);
    b.cx = 2.0 / (g.hix - g.lox);
    b.cy = 2.0 / (g.hiy - g.loy);
    return b;
}

// Element-term contribution of one point of weight W (physical frame):
// D_ij += W [a grad phi_j . grad phi_i + (b . grad phi_j) phi_i + c phi_j phi_i]
template <typename T, int P, bool ADV>
__device__ __forceinline__ void vol_matrix(T (&D)[nb2d(P) * nb2d(P)], const Eval<T, P> &ev, double W, double a_,
                                           const Box &bx, const DevProblem &pr) {
    constexpr int NB = nb2d(P);
    const T a = T(a_);
    const T wxx = T(W * bx.cx * bx.cx) * a, wyy = T(W * bx.cy * bx.cy) * a;
    const T wbx = T(W * pr.bx * bx.cx), wby = T(W * pr.by * bx.cy), wc = T(W * pr.c);
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        const T h0 = wxx * ev.g0[j], h1 = wyy * ev.g1[j];
        if (ADV) {
            const T h2 = fmat(wbx, ev.g0[j], fmat(wby, ev.g1[j], wc * ev.v[j]));
#pragma unroll
            for (int i = 0; i < NB; ++i)
                D[i * NB + j] = fmat(ev.g0[i], h0, fmat(ev.g1[i], h1, fmat(ev.v[i], h2, D[i * NB + j])));
        } else {
#pragma unroll
            for (int i = 0; i < NB; ++i) D[i * NB + j] = fmat(ev.g0[i], h0, fmat(ev.g1[i], h1, D[i * NB + j]));
        }
    }
}

// sqrt((2a+1)(2b+1)) of basis function i: its normalisation times sqrt(|B|)
__constant__ double c_norm[15] = {1.0, 1.7320508075688772, 1.7320508075688772, 2.23606797749979, 3.0,
                                  2.23606797749979, 2.6457513110645907, 3.872983346207417, 3.872983346207417,
                                  2.6457513110645907, 3.0, 4.58257569495584, 5.0, 4.58257569495584, 3.0};

// largest k in [0, n) with start[k] <= v (start ascending, start[0] = 0)
__device__ __forceinline__ int find_owner(const int *start, int n, int v) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= v)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

}  // namespace

template <typename T, int P>
struct AsmCfg {
    static constexpr int NB = nb2d(P);
    static constexpr int NB2 = NB * NB;
    static constexpr int WG = (sizeof(T) == 8 && P >= 3) ? 64 : 128;
    // large blocks: accumulate the self and cross blocks of a face in two passes
    static constexpr bool SPLIT = (int)sizeof(T) * NB2 > 4 * 36;
    static constexpr int SLOTS = WG;          // tasks per chunk
    static constexpr int FSLOTS = WG / 2;     // faces (loop edges) per chunk
    static constexpr int MAXC = 64;           // elements per chunk
    static constexpr int MAXB = FSLOTS + MAXC;  // blocks per chunk (at most one per face plus the diagonals)
    static constexpr int TDEG = P <= 2 ? 4 : 2 * P;
    static constexpr int NQT = Tri<TDEG>::n;  // points per sub-triangle
    static constexpr int VC = TDEG == 8 ? 4 : 3;
    static constexpr int NCH = NQT / VC;      // point chunks per sub-triangle
    static constexpr int NG = P + 1 > 3 ? P + 1 : 3;
    static constexpr int RVC = 4;                 // reduced-rule points per task
    static constexpr int RT = kQrNodes / RVC;     // reduced-rule tasks per row
    static constexpr int LD = SLOTS + 1;      // odd strides: conflict-free LDS columns
    static constexpr int LDF = FSLOTS + 1;
};

void assemble_limits(int precision, int p, AsmLimits *lim) {
#define DGP_LIM(T, PP)                        \
    if (p == PP) {                            \
        using C = AsmCfg<T, PP>;              \
        lim->slots = C::SLOTS;                \
        lim->fslots = C::FSLOTS;              \
        lim->maxc = C::MAXC;                  \
        lim->tasks_per_triangle = C::NCH;     \
        lim->reduced_tasks = C::RT;           \
        return;                               \
    }
    if (precision == 0) {
        DGP_LIM(double, 1) DGP_LIM(double, 2) DGP_LIM(double, 3)
    } else {
        DGP_LIM(float, 1) DGP_LIM(float, 2) DGP_LIM(float, 3)
    }
#undef DGP_LIM
    lim->slots = lim->fslots = lim->maxc = lim->tasks_per_triangle = lim->reduced_tasks = 0;
}

template <typename T, int P, bool ADV>
__global__ void __launch_bounds__((AsmCfg<T, P>::WG)) k_assemble2d(AsmArgs A) {
    using C = AsmCfg<T, P>;
    constexpr int NB = C::NB, NB2 = C::NB2, LD = C::LD, LDF = C::LDF;
    const DevMesh &m = A.m;
    const DevProblem &pr = A.pr;
    T *__restrict__ vals = static_cast<T *>(A.vals);
    T *__restrict__ rhs = static_cast<T *>(A.rhs);

    __shared__ T Dp[NB2 * LD];
    __shared__ T Xp[NB2 * LDF];
    __shared__ T Rp[NB * LD];
    __shared__ int s_task[C::MAXC + 1], s_face[C::MAXC + 1], s_blk[C::MAXC + 1], s_out[C::MAXC + 1];
    __shared__ int s_dof[C::MAXC + 1];
    __shared__ int s_red[C::MAXC];             // the row's volume matrix uses its reduced rule
    __shared__ CellGeo s_geo[C::MAXC];
    __shared__ double s_isq[C::MAXC];          // 1 / sqrt|B| of the element
    __shared__ TrigCentre s_trig[C::MAXC];     // sin/cos at the element's box centre
    __shared__ double s_vx[C::FSLOTS], s_vy[C::FSLOTS];  // loop vertices of the chunk
    __shared__ int s_vid[C::FSLOTS];           // their global ids (canonical edge order)
    __shared__ int s_fnb[C::FSLOTS];           // neighbour across each loop edge (-1 Dirichlet, -2 Neumann)
    __shared__ char s_first[C::FSLOTS];        // first edge of the row towards that neighbour
    __shared__ CellGeo s_fgeo[C::FSLOTS];      // the neighbour's geometry
    __shared__ double s_fisq[C::FSLOTS];       // and 1 / sqrt|B| of it
    __shared__ int s_bcol[C::MAXB], s_bface[C::MAXB];
    __shared__ unsigned long long s_pre[3];

    const int tid = threadIdx.x;
    const int c0 = A.chunks[2 * blockIdx.x], v0 = A.chunks[2 * blockIdx.x + 1];
    const int nc = A.chunks[2 * blockIdx.x + 2] - c0;
    const int nloop = A.chunks[2 * blockIdx.x + 3] - v0;

    // ---- 1. gather: element data, loop vertices, neighbours, row prefix
    if (tid < 3) s_pre[tid] = 0;
    int my_cnt[3] = {0, 0, 0};
    int my_nv = 0;
    if (tid < nc) {
        const int c = c0 + tid;
        s_face[tid] = (int)(m.cell_ptr[c] - v0);
        my_nv = (int)(m.cell_ptr[c + 1] - m.cell_ptr[c]);
        const CellGeo g = A.geo[c];
        s_geo[tid] = g;
        s_isq[tid] = 1.0 / g.sqrt_box;
        const double hx = g.hix - g.lox, hy = g.hiy - g.loy;
        s_trig[tid] = trig_centre(pr, 0.5 * (g.lox + g.hix), 0.5 * (g.loy + g.hiy), 0.5 * sqrt(hx * hx + hy * hy));
        my_cnt[0] = A.cnt[4 * c];
        my_cnt[1] = A.cnt[4 * c + 1];
        my_cnt[2] = A.cnt[4 * c + 2];
        s_red[tid] = A.reduced && A.qr_ok[c];
    }
    const int n_red = A.reduced ? C::RT : 0;
    if (tid == 0) s_face[nc] = nloop;
    for (int e = tid; e < nloop; e += C::WG) {
        const int vi = m.cell_vtx[v0 + e];
        const int o = A.nbr[v0 + e];
        s_vid[e] = vi;
        s_vx[e] = m.x[vi];
        s_vy[e] = m.y[vi];
        s_fnb[e] = o;
        if (o >= 0) {
            const CellGeo g = A.geo[o];
            s_fgeo[e] = g;
            s_fisq[e] = 1.0 / g.sqrt_box;
        }
    }
    __syncthreads();  // s_pre zeroed
    {
        // exclusive prefix at c0: the tile's offset plus the rows of its tile before c0
        const int t0 = c0 / kPrepTile;
        unsigned long long part[3] = {0, 0, 0};
        if (tid < 3) part[tid] = (unsigned long long)A.tile_off[3 * t0 + tid];
        for (int c = t0 * kPrepTile + tid; c < c0; c += C::WG)
            for (int q = 0; q < 3; ++q) part[q] += (unsigned long long)A.cnt[4 * c + q];
        for (int q = 0; q < 3; ++q)
            if (part[q]) atomicAdd(&s_pre[q], part[q]);  // LDS integer sums: order-independent
    }
    // prefix sums over the chunk's rows (wave 0, one lane per row, nc <= 64)
    if (tid < 64) {
        int v[4] = {tid < nc ? (my_nv - 2) * C::NCH + n_red + my_nv : 0, my_cnt[0], my_cnt[1], my_cnt[2]};
        int incl[4] = {v[0], v[1], v[2], v[3]};
        for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int o = __shfl_up(incl[q], off, 64);
                if (tid >= off) incl[q] += o;
            }
        }
        if (tid < nc) {
            s_task[tid + 1] = incl[0];
            s_blk[tid + 1] = incl[1];
            s_out[tid + 1] = incl[2];
            s_dof[tid + 1] = incl[3];
        }
        if (tid == 0) s_task[0] = s_blk[0] = s_out[0] = s_dof[0] = 0;
    }
    __syncthreads();

    // ---- 2. the chunk's rows of the block pattern
    const int64_t pre_b = (int64_t)s_pre[0], pre_v = (int64_t)s_pre[1], pre_d = (int64_t)s_pre[2];
    for (int e = tid; e < nloop; e += C::WG) {
        const int k = find_owner(s_face, nc, e);
        const int o = s_fnb[e];
        bool first = o >= 0 && o != c0 + k;
        for (int e2 = s_face[k]; e2 < e; ++e2)
            if (s_fnb[e2] == o) first = false;
        s_first[e] = first ? 1 : 0;
    }
    __syncthreads();
    for (int e = tid; e < nloop; e += C::WG) {
        if (!s_first[e]) continue;
        const int k = find_owner(s_face, nc, e);
        const int o = s_fnb[e];
        int rank = c0 + k < o ? 1 : 0;
        for (int e2 = s_face[k]; e2 < s_face[k + 1]; ++e2)
            if (s_first[e2] && s_fnb[e2] < o) ++rank;
        const int b = s_blk[k] + rank;
        s_bcol[b] = o;
        s_bface[b] = e;
        if (A.write_pattern) {
            A.col_idx[pre_b + b] = o;
            A.val_ptr[pre_b + b] = pre_v + s_out[k] + (int64_t)rank * NB2;
        }
    }
    if (tid < nc) {
        const int c = c0 + tid;
        int rank = 0;
        for (int e2 = s_face[tid]; e2 < s_face[tid + 1]; ++e2)
            if (s_first[e2] && s_fnb[e2] < c) ++rank;
        const int b = s_blk[tid] + rank;
        s_bcol[b] = c;
        s_bface[b] = -1;
        if (A.write_pattern) {
            A.col_idx[pre_b + b] = c;
            A.val_ptr[pre_b + b] = pre_v + s_out[tid] + (int64_t)rank * NB2;
            A.row_ptr[c] = pre_b + s_blk[tid];
            A.dof_ptr[c] = pre_d + s_dof[tid];
        }
        if (A.write_pattern && c == m.n_cells - 1) {
            A.row_ptr[c + 1] = pre_b + s_blk[tid + 1];
            A.dof_ptr[c + 1] = pre_d + s_dof[tid + 1];
            A.val_ptr[pre_b + s_blk[tid + 1]] = pre_v + s_out[tid + 1];
        }
    }

    if (A.values) {
        __syncthreads();
        // ---- 3. quadrature tasks
        const int n_tasks = s_task[nc];
        for (int t = tid; t < n_tasks; t += C::WG) {
            const int k = find_owner(s_task, nc, t);
            const int lt = t - s_task[k];
            const int nv = s_face[k + 1] - s_face[k];
            const int lb = s_face[k];  // loop entries of row k in the chunk's arrays
            const CellGeo gc = s_geo[k];
            const Box bx = box_of(gc);
            const TrigCentre tc = s_trig[k];
            T D[NB2], R[NB];
#pragma unroll
            for (int e = 0; e < NB2; ++e) D[e] = T(0);
#pragma unroll
            for (int e = 0; e < NB; ++e) R[e] = T(0);

            const int nvol = (nv - 2) * C::NCH;
            if (lt < nvol) {
                // element term: points [chunk*VC, chunk*VC + VC) of sub-triangle tri (the
                // matrix part only when the row has no accepted reduced rule)
                const bool mat = !s_red[k];
                const int tri = lt / C::NCH, chunk = lt - tri * C::NCH;
                const double x0 = s_vx[lb], y0 = s_vy[lb];
                const double x1 = s_vx[lb + tri + 1], y1 = s_vy[lb + tri + 1];
                const double x2 = s_vx[lb + tri + 2], y2 = s_vy[lb + tri + 2];
                const double area = 0.5 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0));
                using R_ = Tri<C::TDEG>;
#pragma unroll
                for (int qq = 0; qq < C::VC; ++qq) {
                    const int q = chunk * C::VC + qq;
                    const double l0 = R_::l(3 * q), l1 = R_::l(3 * q + 1), l2 = R_::l(3 * q + 2);
                    const double px = l0 * x0 + l1 * x1 + l2 * x2;
                    const double py = l0 * y0 + l1 * y1 + l2 * y2;
                    const double W = R_::w(q) * area;
                    const PointData pd = point_data_near(pr, tc, px, py, true);
                    Eval<T, P> ev;
                    ev.at(T((px - bx.mx) * bx.cx), T((py - bx.my) * bx.cy));
                    if (mat) vol_matrix<T, P, ADV>(D, ev, W, pd.a, bx, pr);
                    const T wf = T(W * pd.f);
#pragma unroll
                    for (int i = 0; i < NB; ++i) R[i] = fmat(wf, ev.v[i], R[i]);
                }
            } else if (lt < nvol + n_red) {
                // element matrix with the row's reduced rule: nodes [chunk*RVC, chunk*RVC + RVC)
                if (s_red[k]) {
                    const int64_t cg = c0 + k;
                    const int chunk = lt - nvol;
                    const double jac = 0.25 * (gc.hix - gc.lox) * (gc.hiy - gc.loy);
#pragma unroll
                    for (int qq = 0; qq < C::RVC; ++qq) {
                        const int q = chunk * C::RVC + qq;
                        const double xi = A.qr_nodes[cg * 2 * kQrNodes + 2 * q];
                        const double eta = A.qr_nodes[cg * 2 * kQrNodes + 2 * q + 1];
                        const double W = A.qr_w[cg * kQrNodes + q] * jac;
                        const double a = coef_a_near(pr, tc, bx.mx + xi / bx.cx, bx.my + eta / bx.cy);
                        Eval<T, P> ev;
                        ev.at(T(xi), T(eta));
                        vol_matrix<T, P, ADV>(D, ev, W, a, bx, pr);
                    }
                }
            } else {
                // face f: edge (v_f, v_f+1) of the loop, points in canonical order (lower vertex id first)
                const int f = lt - nvol - n_red;
                const int e = lb + f, en = lb + (f + 1 == nv ? 0 : f + 1);
                const bool fwd = s_vid[e] < s_vid[en];
                const double xa = fwd ? s_vx[e] : s_vx[en], ya = fwd ? s_vy[e] : s_vy[en];
                const double tx = (fwd ? s_vx[en] : s_vx[e]) - xa, ty = (fwd ? s_vy[en] : s_vy[e]) - ya;
                const double len = sqrt(tx * tx + ty * ty);
                const double dir = fwd ? 1.0 : -1.0;
                const double nx = dir * ty / len, ny = -dir * tx / len;  // outward for a CCW loop
                const double bn = pr.bx * nx + pr.by * ny;
                const double up = bn < 0.0 ? bn : 0.0;
                const T cnx = T(bx.cx * nx), cny = T(bx.cy * ny);
                const int goff = c_gl_off[C::NG - 1];
                const int o = s_fnb[e];
                if (o >= 0) {
                    const CellGeo go = s_fgeo[e];
                    const Box bo = box_of(go);
                    const double s1 = gc.abar * P * P / gc.h, s2 = go.abar * P * P / go.h;
                    const double sigma = pr.c_sigma * (s1 > s2 ? s1 : s2);
                    const T conx = T(bo.cx * nx), cony = T(bo.cy * ny);
                    if (!C::SPLIT) {
                        T X[NB2];
#pragma unroll
                        for (int i = 0; i < NB2; ++i) X[i] = T(0);
#pragma unroll
                        for (int q = 0; q < C::NG; ++q) {
                            const double tq = c_gl_t[goff + q], w = c_gl_w[goff + q] * len;
                            const double px = xa + tq * tx, py = ya + tq * ty;
                            const T a = T(coef_a_near(pr, tc, px, py));
                            Eval<T, P> e1, e2;
                            e1.at(T((px - bx.mx) * bx.cx), T((py - bx.my) * bx.cy));
                            e2.at(T((px - bo.mx) * bo.cx), T((py - bo.my) * bo.cy));
                            const T ha = T(-0.5 * w) * a, hs = T((sigma - up) * w);
                            T dn[NB];
#pragma unroll
                            for (int i = 0; i < NB; ++i) dn[i] = fmat(cnx, e1.g0[i], cny * e1.g1[i]);
#pragma unroll
                            for (int j = 0; j < NB; ++j) {
                                const T A1 = fmat(ha, dn[j], hs * e1.v[j]), B1 = ha * e1.v[j];
                                const T dnoj = fmat(conx, e2.g0[j], cony * e2.g1[j]);
                                const T A2 = fmat(ha, dnoj, -hs * e2.v[j]), B2 = -ha * e2.v[j];
#pragma unroll
                                for (int i = 0; i < NB; ++i) {
                                    D[i * NB + j] = fmat(e1.v[i], A1, fmat(dn[i], B1, D[i * NB + j]));
                                    X[i * NB + j] = fmat(e1.v[i], A2, fmat(dn[i], B2, X[i * NB + j]));
                                }
                            }
                        }
#pragma unroll
                        for (int i = 0; i < NB2; ++i) Xp[i * LDF + e] = X[i];
                    } else {
                        // pass 1: self block
#pragma unroll 1
                        for (int q = 0; q < C::NG; ++q) {
                            const double tq = c_gl_t[goff + q], w = c_gl_w[goff + q] * len;
                            const double px = xa + tq * tx, py = ya + tq * ty;
                            const T a = T(coef_a_near(pr, tc, px, py));
                            Eval<T, P> e1;
                            e1.at(T((px - bx.mx) * bx.cx), T((py - bx.my) * bx.cy));
                            const T ha = T(-0.5 * w) * a, hs = T((sigma - up) * w);
                            T dn[NB];
#pragma unroll
                            for (int i = 0; i < NB; ++i) dn[i] = fmat(cnx, e1.g0[i], cny * e1.g1[i]);
#pragma unroll
                            for (int j = 0; j < NB; ++j) {
                                const T A1 = fmat(ha, dn[j], hs * e1.v[j]), B1 = ha * e1.v[j];
#pragma unroll
                                for (int i = 0; i < NB; ++i)
                                    D[i * NB + j] = fmat(e1.v[i], A1, fmat(dn[i], B1, D[i * NB + j]));
                            }
                        }
#pragma unroll
                        for (int i = 0; i < NB2; ++i) {
                            Dp[i * LD + t] = D[i];
                            D[i] = T(0);  // reused as the cross-block accumulator
                        }
                        // pass 2: cross block
#pragma unroll 1
                        for (int q = 0; q < C::NG; ++q) {
                            const double tq = c_gl_t[goff + q], w = c_gl_w[goff + q] * len;
                            const double px = xa + tq * tx, py = ya + tq * ty;
                            const T a = T(coef_a_near(pr, tc, px, py));
                            Eval<T, P> e1, e2;
                            e1.at(T((px - bx.mx) * bx.cx), T((py - bx.my) * bx.cy));
                            e2.at(T((px - bo.mx) * bo.cx), T((py - bo.my) * bo.cy));
                            const T ha = T(-0.5 * w) * a, hs = T((sigma - up) * w);
#pragma unroll
                            for (int j = 0; j < NB; ++j) {
                                const T dnoj = fmat(conx, e2.g0[j], cony * e2.g1[j]);
                                const T A2 = fmat(ha, dnoj, -hs * e2.v[j]), B2 = -ha * e2.v[j];
#pragma unroll
                                for (int i = 0; i < NB; ++i)
                                    D[i * NB + j] = fmat(e1.v[i], A2,
                                                         fmat(fmat(cnx, e1.g0[i], cny * e1.g1[i]), B2, D[i * NB + j]));
                            }
                        }
#pragma unroll
                        for (int i = 0; i < NB2; ++i) Xp[i * LDF + e] = D[i];
#pragma unroll
                        for (int i = 0; i < NB; ++i) Rp[i * LD + t] = R[i];
                        continue;  // the self partial is stored already
                    }
                } else if (o == -1) {
                    // Dirichlet boundary face (carries the inflow term where b . n < 0)
                    const double sigma = pr.c_sigma * gc.abar * P * P / gc.h;
#pragma unroll
                    for (int q = 0; q < C::NG; ++q) {
                        const double tq = c_gl_t[goff + q], w = c_gl_w[goff + q] * len;
                        const double px = xa + tq * tx, py = ya + tq * ty;
                        const PointData pd = point_data(pr, px, py, false);
                        Eval<T, P> e1;
                        e1.at(T((px - bx.mx) * bx.cx), T((py - bx.my) * bx.cy));
                        const T ha = T(-w * pd.a), hs = T((sigma - up) * w);
                        const T ga = T(-w * pd.a * pd.u), gs = T((sigma - up) * w * pd.u);
                        T dn[NB];
#pragma unroll
                        for (int i = 0; i < NB; ++i) dn[i] = fmat(cnx, e1.g0[i], cny * e1.g1[i]);
#pragma unroll
                        for (int j = 0; j < NB; ++j) {
                            const T A1 = fmat(ha, dn[j], hs * e1.v[j]), B1 = ha * e1.v[j];
#pragma unroll
                            for (int i = 0; i < NB; ++i)
                                D[i * NB + j] = fmat(e1.v[i], A1, fmat(dn[i], B1, D[i * NB + j]));
                        }
#pragma unroll
                        for (int i = 0; i < NB; ++i) R[i] = fmat(dn[i], ga, fmat(e1.v[i], gs, R[i]));
                    }
                } else {
                    // Neumann face: g_N = n . (a grad u), right-hand side only
#pragma unroll
                    for (int q = 0; q < C::NG; ++q) {
                        const double tq = c_gl_t[goff + q], w = c_gl_w[goff + q] * len;
                        const double px = xa + tq * tx, py = ya + tq * ty;
                        const PointData pd = point_data(pr, px, py, false);
                        Eval<T, P> e1;
                        e1.at(T((px - bx.mx) * bx.cx), T((py - bx.my) * bx.cy));
                        const T gn = T(w * pd.a * (pd.ux * nx + pd.uy * ny));
#pragma unroll
                        for (int i = 0; i < NB; ++i) R[i] = fmat(gn, e1.v[i], R[i]);
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < NB2; ++i) Dp[i * LD + t] = D[i];
#pragma unroll
            for (int i = 0; i < NB; ++i) Rp[i * LD + t] = R[i];
        }
        __syncthreads();

        // ---- 4a. diagonal blocks: sum the row's task partials (fixed order) into its first slot
        for (int idx = tid; idx < nc * NB2; idx += C::WG) {
            const int k = idx / NB2, ij = idx - k * NB2;
            const int t0 = s_task[k], t1 = s_task[k + 1];
            T sum = Dp[ij * LD + t0];
            for (int t = t0 + 1; t < t1; ++t) sum += Dp[ij * LD + t];
            Dp[ij * LD + t0] = sum;
        }
        for (int idx = tid; idx < nc * NB; idx += C::WG) {
            const int k = idx / NB, i = idx - k * NB;
            T sum = T(0);
            for (int t = s_task[k]; t < s_task[k + 1]; ++t) sum += Rp[i * LD + t];
            rhs[pre_d + s_dof[k] + i] = T(double(sum) * c_norm[i] * s_isq[k]);
        }
        __syncthreads();
        // ---- 4b. the rows, one wave per row: consecutive lanes on consecutive entries
        constexpr int NW = C::WG / 64;
        const int lane = tid & 63, wave = tid >> 6;
        for (int k = wave; k < nc; k += NW) {
            const int n = s_out[k + 1] - s_out[k];
            T *dst = vals + pre_v + s_out[k];
            const double isq = s_isq[k];
            const int t0 = s_task[k];
            for (int e = lane; e < n; e += 64) {
                const int r = e / NB2, ij = e - r * NB2;
                const int i = ij / NB, j = ij - i * NB;
                const int b = s_blk[k] + r;
                const int f0 = s_bface[b];
                T sum;
                double scale;
                if (f0 < 0) {
                    sum = Dp[ij * LD + t0];
                    scale = isq * isq;
                } else {
                    const int col = s_bcol[b];
                    sum = Xp[ij * LDF + f0];
                    for (int f = f0 + 1; f < s_face[k + 1]; ++f)
                        if (s_fnb[f] == col) sum += Xp[ij * LDF + f];
                    scale = isq * s_fisq[f0];
                }
                dst[e] = T(double(sum) * (c_norm[i] * c_norm[j] * scale));
            }
        }
    }
}

template <typename T, int P>
static void launch_one(const AsmArgs &a, int n_chunks, hipStream_t st) {
    using C = AsmCfg<T, P>;
    const bool adv = a.pr.bx != 0.0 || a.pr.by != 0.0 || a.pr.c != 0.0;
    if (adv)
        hipLaunchKernelGGL((k_assemble2d<T, P, true>), dim3(n_chunks), dim3(C::WG), 0, st, a);
    else
        hipLaunchKernelGGL((k_assemble2d<T, P, false>), dim3(n_chunks), dim3(C::WG), 0, st, a);
}

bool launch_assemble2d(const AsmArgs &a, int n_chunks, int precision, int p, hipStream_t st) {
#define DGP_CASE(T, PP)                     \
    if (p == PP) {                          \
        launch_one<T, PP>(a, n_chunks, st); \
        return true;                        \
    }
    if (precision == 0) {
        DGP_CASE(double, 1)
        DGP_CASE(double, 2)
        DGP_CASE(double, 3)
    } else {
        DGP_CASE(float, 1)
        DGP_CASE(float, 2)
        DGP_CASE(float, 3)
    }
#undef DGP_CASE
    return false;
}

}  // namespace dgp
