// 2D SIPG assembly, row-owner form (no floating-point atomics).
//
// Every block row r (element r's test functions) is produced by one group of
// 8 lanes.  Lane k of the group takes the fan sub-triangles t = k, k+8, ...
// (element term, first line of eq. dg-bilinear, and the load term of
// eq. dg-linear) and the faces f = k, k+8, ... of the element (interior-face
// consistency/symmetry/penalty/upwind couplings and boundary terms, the other
// lines of both equations), each written for the test functions of r:
//
//   element:  D_ij += w [a grad phi_j . grad phi_i + (b . grad phi_j) phi_i + c phi_j phi_i]
//   interior: D_ij += w [-a/2 dn_j phi_i - a/2 dn_i phi_j + sigma phi_j phi_i] - [bn<0] w bn phi_j phi_i
//             X_ij += w [-a/2 dn'_j phi_i + a/2 dn_i phi'_j - sigma phi'_j phi_i] + [bn<0] w bn phi'_j phi_i
//   boundary: D_ij += w [-a dn_j phi_i - a dn_i phi_j + sigma phi_j phi_i] - [bn<0] w bn phi_j phi_i
//             F_i  += w [-g a dn_i + sigma g phi_i] - [bn<0] w bn g phi_i
// (dn = grad phi . n_r, primes = the neighbour's basis, bn = b . n_r).
//
// Precision: positions, weights, coefficients, chain factors and the penalty
// are FP64; each per-point weight is formed in FP64 and rounded once to T.
// The basis is evaluated without its normalisation s_i = sqrt((2a+1)(2b+1)/|B|)
// (Legendre values are O(1) in T); every term is bilinear, so s_i s'_j is
// applied in FP64 to the finished block.  The 8 partial diagonal blocks of a
// row are summed by a fixed DPP tree (deterministic).  Rows are staged in LDS
// and written to HBM with 16-byte stores, contiguously in column order.
#include <type_traits>

#include "dgp_common.h"
#include "kernels.h"
#include "rules_data.h"

namespace dgp {

constexpr int kGroup = 8;  // lanes per element row

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Sum over the 8 lanes of an aligned group; every lane ends with the same bits.
template <typename T>
__device__ __forceinline__ T group_sum(T v) {
    v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);  // row_half_mirror
    return v;
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
    double mx, my, cx, cy;  // centre and chain factors 2/h
    __device__ __forceinline__ void from(const CellGeo &g) {
        mx = 0.5 * (g.lox + g.hix);
        my = 0.5 * (g.loy + g.hiy);
        cx = 2.0 / (g.hix - g.lox);
        cy = 2.0 / (g.hiy - g.loy);
    }
};

template <typename T, int P>
struct Cfg {
    static constexpr int NB = nb2d(P);
    static constexpr int NB2 = NB * NB;
    static constexpr int WG = sizeof(T) == 4 ? 256 : 128;
    static constexpr int CPB = WG / kGroup;  // element rows per work-group
    static constexpr int STAGE_BYTES_MAX = 48 * 1024;
    static constexpr int STAGE0 = CPB * 10 * NB2;
    static constexpr int STAGE = STAGE0 * (int)sizeof(T) > STAGE_BYTES_MAX ? STAGE_BYTES_MAX / (int)sizeof(T) : STAGE0;
    static constexpr int TDEG = P <= 2 ? 4 : 2 * P;
};

// normalisation numerator sqrt((2a+1)(2b+1)) of basis function i
__device__ __forceinline__ double norm_num(int i) {
    return sqrt((2.0 * exp_a(i) + 1.0) * (2.0 * exp_b(i) + 1.0));
}

template <typename T, int P>
__global__ void __launch_bounds__((Cfg<T, P>::WG))
    k_assemble2d(DevMesh m, DevProblem pr, const CellGeo *__restrict__ geo, const int64_t *__restrict__ row_ptr,
                 const int32_t *__restrict__ col_idx, const int64_t *__restrict__ val_ptr,
                 const int64_t *__restrict__ dof_ptr, T *__restrict__ vals, T *__restrict__ rhs) {
    using C = Cfg<T, P>;
    constexpr int NB = C::NB;
    constexpr int NB2 = C::NB2;
    __shared__ T stage[C::STAGE];

    const int lane = threadIdx.x % kGroup;
    const int c0 = blockIdx.x * C::CPB;
    const int c_end = min(c0 + C::CPB, m.n_cells);
    const int c = c0 + threadIdx.x / kGroup;
    const bool valid = c < m.n_cells;
    const int64_t gbase = val_ptr[row_ptr[c0]];
    const int64_t gend = val_ptr[row_ptr[c_end]];
    const bool staged = (gend - gbase) <= C::STAGE;

    T D[NB2], R[NB];
#pragma unroll
    for (int e = 0; e < NB2; ++e) D[e] = T(0);
#pragma unroll
    for (int e = 0; e < NB; ++e) R[e] = T(0);

    int64_t rp = 0;
    int rlen = 0;
    CellGeo gc;
    if (valid) {
        gc = geo[c];
        Box bx;
        bx.from(gc);
        const int64_t s = m.cell_ptr[c];
        const int nv = (int)(m.cell_ptr[c + 1] - s);
        rp = row_ptr[c];
        rlen = (int)(row_ptr[c + 1] - rp);
        const double bxv = pr.bx, byv = pr.by;

        // ---------------- element term on fan sub-triangles (v0, v_t+1, v_t+2)
        const int iv0 = m.cell_vtx[s];
        const double x0 = m.x[iv0], y0 = m.y[iv0];
        for (int t = lane; t < nv - 2; t += kGroup) {
            const int iv1 = m.cell_vtx[s + t + 1], iv2 = m.cell_vtx[s + t + 2];
            const double x1 = m.x[iv1], y1 = m.y[iv1], x2 = m.x[iv2], y2 = m.y[iv2];
            const double area = 0.5 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0));
            using R_ = Tri<C::TDEG>;
            for (int q = 0; q < R_::n; ++q) {
                const double l0 = R_::l(3 * q), l1 = R_::l(3 * q + 1), l2 = R_::l(3 * q + 2);
                const double px = l0 * x0 + l1 * x1 + l2 * x2;
                const double py = l0 * y0 + l1 * y1 + l2 * y2;
                const double W = R_::w(q) * area;
                const PointData pd = point_data(pr, px, py, true);
                Eval<T, P> ev;
                ev.at(T((px - bx.mx) * bx.cx), T((py - bx.my) * bx.cy));
                const T wxx = T(W * pd.a * bx.cx * bx.cx), wyy = T(W * pd.a * bx.cy * bx.cy);
                const T wbx = T(W * bxv * bx.cx), wby = T(W * byv * bx.cy), wc = T(W * pr.c), wf = T(W * pd.f);
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    const T h0 = wxx * ev.g0[j], h1 = wyy * ev.g1[j];
                    const T h2 = wbx * ev.g0[j] + wby * ev.g1[j] + wc * ev.v[j];
#pragma unroll
                    for (int i = 0; i < NB; ++i) D[i * NB + j] += ev.g0[i] * h0 + ev.g1[i] * h1 + ev.v[i] * h2;
                }
#pragma unroll
                for (int i = 0; i < NB; ++i) R[i] += wf * ev.v[i];
            }
        }

        // ---------------- faces of the element: edge (v_f, v_f+1) of its loop
        for (int f = lane; f < nv; f += kGroup) {
            const int va = m.cell_vtx[s + f], vb = m.cell_vtx[s + (f + 1 == nv ? 0 : f + 1)];
            const int F = m.cell_face[s + f];
            const int o = other_cell(m, F, c);
            // canonical point order (lower vertex id first) so both owners use the same points
            const int ca = va < vb ? va : vb, cb = va < vb ? vb : va;
            const double xa = m.x[ca], ya = m.y[ca];
            const double tx = m.x[cb] - xa, ty = m.y[cb] - ya;
            const double len = sqrt(tx * tx + ty * ty);
            const double dir = va < vb ? 1.0 : -1.0;  // loop direction vs canonical direction
            const double nx = dir * ty / len, ny = -dir * tx / len;  // outward for a CCW loop
            const double bn = bxv * nx + byv * ny;
            const double up = bn < 0.0 ? bn : 0.0;
            const T cnx = T(bx.cx * nx), cny = T(bx.cy * ny);
            const int ng = P + 1 > 3 ? P + 1 : 3;
            const int goff = c_gl_off[ng - 1];
            if (o >= 0) {
                const CellGeo go = geo[o];
                Box bo;
                bo.from(go);
                const double s1 = gc.abar * P * P / gc.h, s2 = go.abar * P * P / go.h;
                const double sigma = pr.c_sigma * (s1 > s2 ? s1 : s2);
                // the first face towards o owns the cross block and adds any later faces towards o
                bool owner = true;
                for (int j = 0; j < f; ++j)
                    if (other_cell(m, m.cell_face[s + j], c) == o) owner = false;
                T X[NB2];
#pragma unroll
                for (int e = 0; e < NB2; ++e) X[e] = T(0);
                const T conx = T(bo.cx * nx), cony = T(bo.cy * ny);
                for (int q = 0; q < ng; ++q) {
                    const double tq = c_gl_t[goff + q], w = c_gl_w[goff + q] * len;
                    const double px = xa + tq * tx, py = ya + tq * ty;
                    const double a = coef_a(pr, px, py);
                    Eval<T, P> e1, e2;
                    e1.at(T((px - bx.mx) * bx.cx), T((py - bx.my) * bx.cy));
                    e2.at(T((px - bo.mx) * bo.cx), T((py - bo.my) * bo.cy));
                    T dn[NB], dno[NB];
#pragma unroll
                    for (int i = 0; i < NB; ++i) {
                        dn[i] = cnx * e1.g0[i] + cny * e1.g1[i];
                        dno[i] = conx * e2.g0[i] + cony * e2.g1[i];
                    }
                    const T ha = T(-0.5 * a * w), hs = T((sigma - up) * w);
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        const T A1 = ha * dn[j] + hs * e1.v[j], B1 = ha * e1.v[j];
#pragma unroll
                        for (int i = 0; i < NB; ++i) D[i * NB + j] += e1.v[i] * A1 + dn[i] * B1;
                    }
                    if (owner) {
#pragma unroll
                        for (int j = 0; j < NB; ++j) {
                            const T A2 = ha * dno[j] - hs * e2.v[j], B2 = -ha * e2.v[j];
#pragma unroll
                            for (int i = 0; i < NB; ++i) X[i * NB + j] += e1.v[i] * A2 + dn[i] * B2;
                        }
                    }
                }
                if (owner) {
                    // later faces towards the same neighbour (agglomerates sharing several faces)
                    for (int f2 = f + 1; f2 < nv; ++f2) {
                        if (other_cell(m, m.cell_face[s + f2], c) != o) continue;
                        const int wa = m.cell_vtx[s + f2], wb = m.cell_vtx[s + (f2 + 1 == nv ? 0 : f2 + 1)];
                        const int da = wa < wb ? wa : wb, db = wa < wb ? wb : wa;
                        const double xa2 = m.x[da], ya2 = m.y[da];
                        const double tx2 = m.x[db] - xa2, ty2 = m.y[db] - ya2;
                        const double len2 = sqrt(tx2 * tx2 + ty2 * ty2);
                        const double dir2 = wa < wb ? 1.0 : -1.0;
                        const double nx2 = dir2 * ty2 / len2, ny2 = -dir2 * tx2 / len2;
                        const double bn2 = bxv * nx2 + byv * ny2;
                        const double up2 = bn2 < 0.0 ? bn2 : 0.0;
                        const T cnx2 = T(bx.cx * nx2), cny2 = T(bx.cy * ny2);
                        const T conx2 = T(bo.cx * nx2), cony2 = T(bo.cy * ny2);
                        for (int q = 0; q < ng; ++q) {
                            const double tq = c_gl_t[goff + q], w = c_gl_w[goff + q] * len2;
                            const double px = xa2 + tq * tx2, py = ya2 + tq * ty2;
                            const double a = coef_a(pr, px, py);
                            Eval<T, P> e1, e2;
                            e1.at(T((px - bx.mx) * bx.cx), T((py - bx.my) * bx.cy));
                            e2.at(T((px - bo.mx) * bo.cx), T((py - bo.my) * bo.cy));
                            const T ha = T(-0.5 * a * w), hs = T((sigma - up2) * w);
#pragma unroll
                            for (int j = 0; j < NB; ++j) {
                                const T dnoj = conx2 * e2.g0[j] + cony2 * e2.g1[j];
                                const T A2 = ha * dnoj - hs * e2.v[j], B2 = -ha * e2.v[j];
#pragma unroll
                                for (int i = 0; i < NB; ++i)
                                    X[i * NB + j] += e1.v[i] * A2 + (cnx2 * e1.g0[i] + cny2 * e1.g1[i]) * B2;
                            }
                        }
                    }
                    // scale by s_i s'_j in FP64 and place the block
                    int kc = 0;
                    while (kc < rlen && col_idx[rp + kc] != o) ++kc;
                    if (kc == rlen) continue;  // not in the pattern: the pattern is of another mesh
                    const int64_t off = val_ptr[rp + kc];
                    const double inv = 1.0 / (gc.sqrt_box * go.sqrt_box);
#pragma unroll
                    for (int i = 0; i < NB; ++i) {
#pragma unroll
                        for (int j = 0; j < NB; ++j) {
                            const T val = T(double(X[i * NB + j]) * norm_num(i) * norm_num(j) * inv);
                            if (staged)
                                stage[off - gbase + i * NB + j] = val;
                            else
                                vals[off + i * NB + j] = val;
                        }
                    }
                }
            } else if (m.face_bc[F] == 1) {
                // Dirichlet boundary face (also carries the inflow term where b . n < 0)
                const double sigma = pr.c_sigma * gc.abar * P * P / gc.h;
                for (int q = 0; q < ng; ++q) {
                    const double tq = c_gl_t[goff + q], w = c_gl_w[goff + q] * len;
                    const double px = xa + tq * tx, py = ya + tq * ty;
                    const PointData pd = point_data(pr, px, py, false);
                    Eval<T, P> e1;
                    e1.at(T((px - bx.mx) * bx.cx), T((py - bx.my) * bx.cy));
                    T dn[NB];
#pragma unroll
                    for (int i = 0; i < NB; ++i) dn[i] = cnx * e1.g0[i] + cny * e1.g1[i];
                    const T ha = T(-pd.a * w), hs = T((sigma - up) * w);
                    const T ga = T(-pd.a * w * pd.u), gs = T((sigma - up) * w * pd.u);
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        const T A1 = ha * dn[j] + hs * e1.v[j], B1 = ha * e1.v[j];
#pragma unroll
                        for (int i = 0; i < NB; ++i) D[i * NB + j] += e1.v[i] * A1 + dn[i] * B1;
                    }
#pragma unroll
                    for (int i = 0; i < NB; ++i) R[i] += dn[i] * ga + e1.v[i] * gs;
                }
            } else {
                // Neumann face: g_N = n . (a grad u) on the right-hand side only
                for (int q = 0; q < ng; ++q) {
                    const double tq = c_gl_t[goff + q], w = c_gl_w[goff + q] * len;
                    const double px = xa + tq * tx, py = ya + tq * ty;
                    const PointData pd = point_data(pr, px, py, false);
                    Eval<T, P> e1;
                    e1.at(T((px - bx.mx) * bx.cx), T((py - bx.my) * bx.cy));
                    const T gn = T(w * pd.a * (pd.ux * nx + pd.uy * ny));
#pragma unroll
                    for (int i = 0; i < NB; ++i) R[i] += gn * e1.v[i];
                }
            }
        }
    }

    // ---------------- diagonal block and load: fixed-order sum over the group
#pragma unroll
    for (int e = 0; e < NB2; ++e) D[e] = group_sum(D[e]);
#pragma unroll
    for (int e = 0; e < NB; ++e) R[e] = group_sum(R[e]);

    int kd = 0;
    while (kd < rlen && col_idx[rp + kd] != c) ++kd;
    if (valid && lane == 0 && kd < rlen) {
        const int64_t off = val_ptr[rp + kd];
        const double inv = 1.0 / (gc.sqrt_box * gc.sqrt_box);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
#pragma unroll
            for (int j = 0; j < NB; ++j) {
                const T val = T(double(D[i * NB + j]) * norm_num(i) * norm_num(j) * inv);
                if (staged)
                    stage[off - gbase + i * NB + j] = val;
                else
                    vals[off + i * NB + j] = val;
            }
        }
        const int64_t db = dof_ptr[c];
        const double invs = 1.0 / gc.sqrt_box;
#pragma unroll
        for (int i = 0; i < NB; ++i) rhs[db + i] = T(double(R[i]) * norm_num(i) * invs);
    }

    // ---------------- write the staged rows: contiguous, 16-byte stores
    __syncthreads();
    if (staged) {
        constexpr int VW = 16 / (int)sizeof(T);
        const int64_t n = gend - gbase;
        T *dst = vals + gbase;
        int64_t head = (int64_t)(((16 - ((uintptr_t)dst & 15)) & 15) / sizeof(T));
        if (head > n) head = n;
        for (int64_t e = threadIdx.x; e < head; e += C::WG) dst[e] = stage[e];
        const int64_t nvec = (n - head) / VW;
        using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
        for (int64_t v = threadIdx.x; v < nvec; v += C::WG) {
            V out;
            T *po = reinterpret_cast<T *>(&out);
#pragma unroll
            for (int u = 0; u < VW; ++u) po[u] = stage[head + v * VW + u];
            *reinterpret_cast<V *>(dst + head + v * VW) = out;
        }
        for (int64_t e = head + nvec * VW + threadIdx.x; e < n; e += C::WG) dst[e] = stage[e];
    }
}

template <typename T, int P>
static void launch_one(const DevMesh &m, const DevProblem &pr, const CellGeo *geo, const int64_t *row_ptr,
                       const int32_t *col_idx, const int64_t *val_ptr, const int64_t *dof_ptr, void *vals, void *rhs,
                       hipStream_t st) {
    using C = Cfg<T, P>;
    const int blocks = (m.n_cells + C::CPB - 1) / C::CPB;
    hipLaunchKernelGGL((k_assemble2d<T, P>), dim3(blocks), dim3(C::WG), 0, st, m, pr, geo, row_ptr, col_idx, val_ptr,
                       dof_ptr, static_cast<T *>(vals), static_cast<T *>(rhs));
}

bool launch_assemble2d(const DevMesh &m, const DevProblem &pr, const CellGeo *geo, const int64_t *row_ptr,
                       const int32_t *col_idx, const int64_t *val_ptr, const int64_t *dof_ptr, int precision,
                       int p, void *vals, void *rhs, hipStream_t st) {
#define DGP_CASE(T, PP)                                                                     \
    if (p == PP) {                                                                          \
        launch_one<T, PP>(m, pr, geo, row_ptr, col_idx, val_ptr, dof_ptr, vals, rhs, st); \
        return true;                                                                        \
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
