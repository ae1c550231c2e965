// 2D SIPG assembly, row-owner form (no floating-point atomics).
//
// A work-group owns a run of consecutive element rows (a chunk chosen by the
// runtime so that its quadrature tasks fit the work-group).  Each row's work is
// split into tasks of a few quadrature points:
//   * element term (first line of eq. dg-bilinear; load term of eq. dg-linear)
//     on a fan sub-triangle (v0, v_t+1, v_t+2), one chunk of its rule points;
//   * one face of the element: interior-face consistency/symmetry/penalty/
//     upwind couplings (self block and cross block), or the boundary terms
//     of both equations.
// Written for the test functions phi_i of row r (dn = grad phi . n_r,
// primes = the neighbour's basis, bn = b . n_r, [bn<0] = inflow part of the
// boundary of r):
//   element:  D_ij += w [a grad phi_j . grad phi_i + (b . grad phi_j) phi_i + c phi_j phi_i]
//   interior: D_ij += w [-a/2 dn_j phi_i - a/2 dn_i phi_j + sigma phi_j phi_i] - [bn<0] w bn phi_j phi_i
//             X_ij += w [-a/2 dn'_j phi_i + a/2 dn_i phi'_j - sigma phi'_j phi_i] + [bn<0] w bn phi'_j phi_i
//   boundary: D_ij += w [-a dn_j phi_i - a dn_i phi_j + sigma phi_j phi_i] - [bn<0] w bn phi_j phi_i
//             F_i  += w [-g a dn_i + sigma g phi_i] - [bn<0] w bn g phi_i
// Each task accumulates its partial block(s) in registers and stores them in
// LDS.  The work-group then writes its rows -- a contiguous range of the value
// array -- with consecutive lanes on consecutive entries, each entry the sum of
// its partials in task order (deterministic).
//
// Precision: positions, Jacobians, bounding-box scaling and the penalty are
// FP64; per-point weights are formed in FP64 and rounded once to T.  In the
// FP32 path the coefficient and load functions are evaluated in FP32 after an
// exact FP64 argument reduction.  The basis is evaluated without its
// normalisation s_i = sqrt((2a+1)(2b+1)/|B|): every term is bilinear, so
// s_i s'_j is applied to the finished sum.
#include <type_traits>

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

// ---- coefficient evaluation in precision T ----------------------------------
// The load f and the boundary data are always evaluated in FP64 (f is a sum
// of terms that cancel where u is small); the diffusion coefficient on faces
// is evaluated in T.
// sin(pi x), cos(pi x) in FP32 after reducing x by whole periods in FP64.
__device__ __forceinline__ void sincospi_red(double x, float *s, float *c) {
    const double k = rint(x);
    float sf, cf;
    sincospif((float)(x - k), &sf, &cf);
    const bool odd = ((long long)k) & 1;
    *s = odd ? -sf : sf;
    *c = odd ? -cf : cf;
}

template <typename T>
struct Coef;

template <>
struct Coef<double> {
    __device__ static double a(const DevProblem &pr, double x, double y) { return coef_a(pr, x, y); }
    __device__ static PointData data(const DevProblem &pr, double x, double y, bool need_f) {
        return point_data(pr, x, y, need_f);
    }
};

template <>
struct Coef<float> {
    __device__ static float a(const DevProblem &pr, double x, double y) {
        if (pr.a1 == 0.0) return (float)pr.a0;
        float s2x, c2x, s2y, c2y;
        sincospi_red(2.0 * x, &s2x, &c2x);
        sincospi_red(2.0 * y, &s2y, &c2y);
        return (float)pr.a0 + (float)pr.a1 * s2x * c2y;
    }
    // the formulas of point_data (dgp_common.h) in FP32
    __device__ static PointData data(const DevProblem &pr, double x, double y, bool need_f) {
        if (pr.u_kind != 0) return point_data(pr, x, y, need_f);  // polynomial data: cheap in FP64
        PointData d;
        float sx, cx, sy, cy;
        sincospi_red(x, &sx, &cx);
        sincospi_red(y, &sy, &cy);
        const float pi = (float)kPi;
        float a = (float)pr.a0, ax = 0.f, ay = 0.f;
        if (pr.a1 != 0.0) {
            const float s2x = 2.f * sx * cx, c2x = cx * cx - sx * sx;
            const float s2y = 2.f * sy * cy, c2y = cy * cy - sy * sy;
            const float a1 = (float)pr.a1;
            a += a1 * s2x * c2y;
            ax = 2.f * pi * a1 * c2x * c2y;
            ay = -2.f * pi * a1 * s2x * s2y;
        }
        const float u = sx * sy, ux = pi * cx * sy, uy = pi * sx * cy, lap = -2.f * pi * pi * u;
        d.a = a;
        d.u = u;
        d.ux = ux;
        d.uy = uy;
        d.f = need_f ? (double)(-(ax * ux + ay * uy) - a * lap + (float)pr.bx * ux + (float)pr.by * uy +
                                (float)pr.c * u)
                     : 0.0;
        return d;
    }
};

// sqrt((2a+1)(2b+1)) of basis function i: its normalisation times sqrt(|B|)
__constant__ double c_norm[15] = {1.0, 1.7320508075688772, 1.7320508075688772, 2.23606797749979, 3.0,
                                  2.23606797749979, 2.6457513110645907, 3.872983346207417, 3.872983346207417,
                                  2.6457513110645907, 3.0, 4.58257569495584, 5.0, 4.58257569495584, 3.0};
__device__ __forceinline__ double norm_num(int i) { return c_norm[i]; }

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
    static constexpr int WG = (sizeof(T) == 4 && P <= 2) ? 256 : (sizeof(T) == 8 && P >= 3) ? 64 : 128;
    // large blocks: accumulate the self and cross blocks of a face in two passes
    static constexpr bool SPLIT = (int)sizeof(T) * NB2 > 4 * 36;
    static constexpr int SLOTS = WG;          // tasks per chunk
    static constexpr int FSLOTS = WG / 2;     // face tasks per chunk
    static constexpr int MAXC = 64;           // elements per chunk
    static constexpr int MAXB = MAXC * 12;    // blocks per chunk
    static constexpr int TDEG = P <= 2 ? 4 : 2 * P;
    static constexpr int NQT = Tri<TDEG>::n;  // points per sub-triangle
    static constexpr int VC = TDEG == 8 ? 4 : 3;
    static constexpr int NCH = NQT / VC;      // point chunks per sub-triangle
    static constexpr int NG = P + 1 > 3 ? P + 1 : 3;
    static constexpr int LD = SLOTS + 1;      // odd strides: conflict-free LDS columns
    static constexpr int LDF = FSLOTS + 1;
};

void assemble_limits(int precision, int p, AsmLimits *lim) {
#define DGP_LIM(T, PP)                                 \
    if (p == PP) {                                     \
        using C = AsmCfg<T, PP>;                       \
        lim->slots = C::SLOTS;                         \
        lim->fslots = C::FSLOTS;                       \
        lim->maxc = C::MAXC;                           \
        lim->maxb = C::MAXB;                           \
        lim->tasks_per_triangle = C::NCH;              \
        return;                                        \
    }
    if (precision == 0) {
        DGP_LIM(double, 1) DGP_LIM(double, 2) DGP_LIM(double, 3)
    } else {
        DGP_LIM(float, 1) DGP_LIM(float, 2) DGP_LIM(float, 3)
    }
#undef DGP_LIM
    lim->slots = lim->fslots = lim->maxc = lim->maxb = lim->tasks_per_triangle = 0;
}

template <typename T, int P, bool ADV>
__global__ void __launch_bounds__((AsmCfg<T, P>::WG))
    k_assemble2d(DevMesh m, DevProblem pr, const CellGeo *__restrict__ geo, const int64_t *__restrict__ row_ptr,
                 const int32_t *__restrict__ col_idx, const int64_t *__restrict__ val_ptr,
                 const int64_t *__restrict__ dof_ptr, const int32_t *__restrict__ chunks, T *__restrict__ vals,
                 T *__restrict__ rhs) {
    using C = AsmCfg<T, P>;
    constexpr int NB = C::NB, NB2 = C::NB2, LD = C::LD, LDF = C::LDF;

    __shared__ T Dp[NB2 * LD];
    __shared__ T Xp[NB2 * LDF];
    __shared__ T Rp[NB * LD];
    __shared__ int s_task[C::MAXC + 1], s_face[C::MAXC + 1], s_blk[C::MAXC + 1], s_out[C::MAXC + 1];
    __shared__ int s_cs[C::MAXC], s_nv[C::MAXC];
    __shared__ CellGeo s_geo[C::MAXC];
    __shared__ int64_t s_rp[C::MAXC];
    __shared__ int s_fnb[C::FSLOTS];
    __shared__ double s_fsqb[C::FSLOTS];  // 1 / sqrt|B| of the neighbour across the face
    __shared__ double s_isq[C::MAXC];      // 1 / sqrt|B| of the element
    __shared__ int s_bcol[C::MAXB], s_bface[C::MAXB];

    const int tid = threadIdx.x;
    const int c0 = chunks[blockIdx.x];
    const int nc = chunks[blockIdx.x + 1] - c0;

    // ---- per-element setup and prefix sums (wave 0, one lane per element, nc <= 64)
    if (tid < 64) {
        int v[4] = {0, 0, 0, 0};
        if (tid < nc) {
            const int c = c0 + tid;
            const int64_t s = m.cell_ptr[c];
            const int nv = (int)(m.cell_ptr[c + 1] - s);
            s_cs[tid] = (int)s;
            s_nv[tid] = nv;
            s_geo[tid] = geo[c];
            s_isq[tid] = 1.0 / geo[c].sqrt_box;
            const int64_t rp = row_ptr[c];
            s_rp[tid] = rp;
            const int nblk = (int)(row_ptr[c + 1] - rp);
            v[0] = (nv - 2) * C::NCH + nv;
            v[1] = nv;
            v[2] = nblk;
            v[3] = nblk * NB2;
        }
        int incl[4] = {v[0], v[1], v[2], v[3]};
        for (int off = 1; off < 64; off <<= 1) {
            int o[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) o[q] = __shfl_up(incl[q], off, 64);
            if (tid >= off)
#pragma unroll
                for (int q = 0; q < 4; ++q) incl[q] += o[q];
        }
        if (tid < nc) {
            s_task[tid + 1] = incl[0];
            s_face[tid + 1] = incl[1];
            s_blk[tid + 1] = incl[2];
            s_out[tid + 1] = incl[3];
        }
        if (tid == 0) s_task[0] = s_face[0] = s_blk[0] = s_out[0] = 0;
    }
    __syncthreads();
    const int n_tasks = s_task[nc], n_fslots = s_face[nc], n_blk = s_blk[nc];

    // ---- face slots: neighbour and its normalisation
    for (int f = tid; f < n_fslots; f += C::WG) {
        const int k = find_owner(s_face, nc, f);
        const int F = m.cell_face[s_cs[k] + (f - s_face[k])];
        const int o = other_cell(m, F, c0 + k);
        s_fnb[f] = o;
        s_fsqb[f] = o >= 0 ? 1.0 / geo[o].sqrt_box : 0.0;
    }
    __syncthreads();
    // ---- blocks: column and the first face towards it
    for (int b = tid; b < n_blk; b += C::WG) {
        const int k = find_owner(s_blk, nc, b);
        const int col = col_idx[s_rp[k] + (b - s_blk[k])];
        s_bcol[b] = col;
        int first = -1;
        if (col != c0 + k)
            for (int f = s_face[k]; f < s_face[k + 1]; ++f)
                if (s_fnb[f] == col) {
                    first = f;
                    break;
                }
        s_bface[b] = first;
    }

    // ---- quadrature tasks
    for (int t = tid; t < n_tasks; t += C::WG) {
        const int k = find_owner(s_task, nc, t);
        const int lt = t - s_task[k];
        const int nv = s_nv[k];
        const int64_t s = s_cs[k];
        const CellGeo gc = s_geo[k];
        const Box bx = box_of(gc);
        T D[NB2], R[NB];
#pragma unroll
        for (int e = 0; e < NB2; ++e) D[e] = T(0);
#pragma unroll
        for (int e = 0; e < NB; ++e) R[e] = T(0);

        if (lt < (nv - 2) * C::NCH) {
            // element term: points [chunk*VC, chunk*VC + VC) of sub-triangle tri
            const int tri = lt / C::NCH, chunk = lt - tri * C::NCH;
            const int iv0 = m.cell_vtx[s], iv1 = m.cell_vtx[s + tri + 1], iv2 = m.cell_vtx[s + tri + 2];
            const double x0 = m.x[iv0], y0 = m.y[iv0];
            const double x1 = m.x[iv1], y1 = m.y[iv1], x2 = m.x[iv2], y2 = m.y[iv2];
            const double area = 0.5 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0));
            using R_ = Tri<C::TDEG>;
#pragma unroll
            for (int qq = 0; qq < C::VC; ++qq) {
                const int q = chunk * C::VC + qq;
                const double l0 = R_::l(3 * q), l1 = R_::l(3 * q + 1), l2 = R_::l(3 * q + 2);
                const double px = l0 * x0 + l1 * x1 + l2 * x2;
                const double py = l0 * y0 + l1 * y1 + l2 * y2;
                const double W = R_::w(q) * area;
                const PointData pd = point_data(pr, px, py, true);
                Eval<T, P> ev;
                ev.at(T((px - bx.mx) * bx.cx), T((py - bx.my) * bx.cy));
                const T a = T(pd.a);
                const T wxx = T(W * bx.cx * bx.cx) * a, wyy = T(W * bx.cy * bx.cy) * a;
                const T wbx = T(W * pr.bx * bx.cx), wby = T(W * pr.by * bx.cy), wc = T(W * pr.c);
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const T h0 = wxx * ev.g0[j], h1 = wyy * ev.g1[j];
                    if (ADV) {
                        const T h2 = fmat(wbx, ev.g0[j], fmat(wby, ev.g1[j], wc * ev.v[j]));
#pragma unroll
                        for (int i = 0; i < NB; ++i)
                            D[i * NB + j] =
                                fmat(ev.g0[i], h0, fmat(ev.g1[i], h1, fmat(ev.v[i], h2, D[i * NB + j])));
                    } else {
#pragma unroll
                        for (int i = 0; i < NB; ++i)
                            D[i * NB + j] = fmat(ev.g0[i], h0, fmat(ev.g1[i], h1, D[i * NB + j]));
                    }
                }
                const T wf = T(W * pd.f);
#pragma unroll
                for (int i = 0; i < NB; ++i) R[i] = fmat(wf, ev.v[i], R[i]);
            }
        } else {
            // face f: edge (v_f, v_f+1) of the loop, points in canonical order
            const int f = lt - (nv - 2) * C::NCH;
            const int fslot = s_face[k] + f;
            const int va = m.cell_vtx[s + f], vb = m.cell_vtx[s + (f + 1 == nv ? 0 : f + 1)];
            const int o = s_fnb[fslot];
            const int ca = va < vb ? va : vb, cb = va < vb ? vb : va;
            const double xa = m.x[ca], ya = m.y[ca];
            const double tx = m.x[cb] - xa, ty = m.y[cb] - ya;
            const double len = sqrt(tx * tx + ty * ty);
            const double dir = va < vb ? 1.0 : -1.0;
            const double nx = dir * ty / len, ny = -dir * tx / len;  // outward for a CCW loop
            const double bn = pr.bx * nx + pr.by * ny;
            const double up = bn < 0.0 ? bn : 0.0;
            const T cnx = T(bx.cx * nx), cny = T(bx.cy * ny);
            const int goff = c_gl_off[C::NG - 1];
            if (o >= 0) {
                const CellGeo go = geo[o];
                const Box bo = box_of(go);
                const double s1 = gc.abar * P * P / gc.h, s2 = go.abar * P * P / go.h;
                const double sigma = pr.c_sigma * (s1 > s2 ? s1 : s2);
                const T conx = T(bo.cx * nx), cony = T(bo.cy * ny);
                if (!C::SPLIT) {
                    T X[NB2];
#pragma unroll
                    for (int e = 0; e < NB2; ++e) X[e] = T(0);
#pragma unroll
                    for (int q = 0; q < C::NG; ++q) {
                        const double tq = c_gl_t[goff + q], w = c_gl_w[goff + q] * len;
                        const double px = xa + tq * tx, py = ya + tq * ty;
                        const T a = Coef<T>::a(pr, px, py);
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
                    for (int e = 0; e < NB2; ++e) Xp[e * LDF + fslot] = X[e];
                } else {
                    // pass 1: self block
#pragma unroll 1
                    for (int q = 0; q < C::NG; ++q) {
                        const double tq = c_gl_t[goff + q], w = c_gl_w[goff + q] * len;
                        const double px = xa + tq * tx, py = ya + tq * ty;
                        const T a = Coef<T>::a(pr, px, py);
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
                    for (int e = 0; e < NB2; ++e) {
                        Dp[e * LD + t] = D[e];
                        D[e] = T(0);  // reused as the cross-block accumulator
                    }
                    // pass 2: cross block
#pragma unroll 1
                    for (int q = 0; q < C::NG; ++q) {
                        const double tq = c_gl_t[goff + q], w = c_gl_w[goff + q] * len;
                        const double px = xa + tq * tx, py = ya + tq * ty;
                        const T a = Coef<T>::a(pr, px, py);
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
                                D[i * NB + j] =
                                    fmat(e1.v[i], A2, fmat(fmat(cnx, e1.g0[i], cny * e1.g1[i]), B2, D[i * NB + j]));
                        }
                    }
#pragma unroll
                    for (int e = 0; e < NB2; ++e) Xp[e * LDF + fslot] = D[e];
                    // R is zero for interior faces; the partial D is already stored
#pragma unroll
                    for (int e = 0; e < NB; ++e) Rp[e * LD + t] = R[e];
                    continue;
                }

            } else if (m.face_bc[m.cell_face[s + f]] == 1) {
                // Dirichlet boundary face (carries the inflow term where b . n < 0)
                const double sigma = pr.c_sigma * gc.abar * P * P / gc.h;
#pragma unroll
                for (int q = 0; q < C::NG; ++q) {
                    const double tq = c_gl_t[goff + q], w = c_gl_w[goff + q] * len;
                    const double px = xa + tq * tx, py = ya + tq * ty;
                    const PointData pd = Coef<T>::data(pr, px, py, false);
                    Eval<T, P> e1;
                    e1.at(T((px - bx.mx) * bx.cx), T((py - bx.my) * bx.cy));
                    const T a = T(pd.a), g = T(pd.u);
                    const T ha = T(-w) * a, hs = T((sigma - up) * w);
                    const T ga = ha * g, gs = hs * g;
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
        for (int e = 0; e < NB2; ++e) Dp[e * LD + t] = D[e];
#pragma unroll
        for (int e = 0; e < NB; ++e) Rp[e * LD + t] = R[e];
    }
    __syncthreads();

    // ---- write the rows: consecutive lanes on consecutive entries
    const int64_t gbase = val_ptr[s_rp[0]];
    const int n_out = s_out[nc];
    for (int e = tid; e < n_out; e += C::WG) {
        const int k = find_owner(s_out, nc, e);
        const int o = e - s_out[k];
        const int r = o / NB2, ij = o - r * NB2;
        const int i = ij / NB, j = ij - i * NB;
        const int b = s_blk[k] + r;
        const int col = s_bcol[b];
        const double isq = s_isq[k];
        T sum = T(0);
        double scale;
        if (col == c0 + k) {
            for (int t = s_task[k]; t < s_task[k + 1]; ++t) sum += Dp[ij * LD + t];
            scale = norm_num(i) * norm_num(j) * isq * isq;
        } else {
            const int f0 = s_bface[b];  // always >= 0 for a pattern built from this mesh
            if (f0 >= 0) {
                sum = Xp[ij * LDF + f0];
                for (int f = f0 + 1; f < s_face[k + 1]; ++f)
                    if (s_fnb[f] == col) sum += Xp[ij * LDF + f];
            }
            scale = f0 >= 0 ? norm_num(i) * norm_num(j) * isq * s_fsqb[f0] : 0.0;
        }
        vals[gbase + e] = T(double(sum) * scale);
    }
    for (int e = tid; e < nc * NB; e += C::WG) {
        const int k = e / NB, i = e - k * NB;
        T sum = T(0);
        for (int t = s_task[k]; t < s_task[k + 1]; ++t) sum += Rp[i * LD + t];
        rhs[dof_ptr[c0 + k] + i] = T(double(sum) * norm_num(i) * s_isq[k]);
    }
}

template <typename T, int P>
static void launch_one(const DevMesh &m, const DevProblem &pr, const CellGeo *geo, const int64_t *row_ptr,
                       const int32_t *col_idx, const int64_t *val_ptr, const int64_t *dof_ptr, const int32_t *chunks,
                       int n_chunks, void *vals, void *rhs, hipStream_t st) {
    using C = AsmCfg<T, P>;
    const bool adv = pr.bx != 0.0 || pr.by != 0.0 || pr.c != 0.0;
    if (adv)
        hipLaunchKernelGGL((k_assemble2d<T, P, true>), dim3(n_chunks), dim3(C::WG), 0, st, m, pr, geo, row_ptr,
                           col_idx, val_ptr, dof_ptr, chunks, static_cast<T *>(vals), static_cast<T *>(rhs));
    else
        hipLaunchKernelGGL((k_assemble2d<T, P, false>), dim3(n_chunks), dim3(C::WG), 0, st, m, pr, geo, row_ptr,
                           col_idx, val_ptr, dof_ptr, chunks, static_cast<T *>(vals), static_cast<T *>(rhs));
}

bool launch_assemble2d(const DevMesh &m, const DevProblem &pr, const CellGeo *geo, const int64_t *row_ptr,
                       const int32_t *col_idx, const int64_t *val_ptr, const int64_t *dof_ptr, const int32_t *chunks,
                       int n_chunks, int precision, int p, void *vals, void *rhs, hipStream_t st) {
#define DGP_CASE(T, PP)                                                                                     \
    if (p == PP) {                                                                                          \
        launch_one<T, PP>(m, pr, geo, row_ptr, col_idx, val_ptr, dof_ptr, chunks, n_chunks, vals, rhs, st); \
        return true;                                                                                        \
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
