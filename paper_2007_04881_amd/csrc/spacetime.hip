// Space-time slabs (Section 2.3, equation spacetime_dg): the matrix and load of
// one time step I_n = (t0, t1] on prisms I_n x kappa over a 2D polygonal mesh,
// with the total-degree-p space-time basis on each prism's box
// [lo, hi] x [t0, t1] (n_b = (p+1)(p+2)(p+3)/6), row-owner form, one wave per
// prism.
//
// Per row the points are taken in passes of QP lanes, one point per lane:
//   * volume points: fan sub-triangle rule x (p + 1) Gauss points in time;
//     test terms u = (P, dP/dx, dP/dy), trial terms
//     t = w (dP/dt + b . grad P + c P, a dP/dx, a dP/dy): time derivative,
//     diffusion, advection and reaction of the prism;
//   * bottom points (t = t0): the time jump (U^+, W^+) as u = P, t = w P, and
//     the load w U_{n-1}^- P (U_{n-1}^- from the previous slab's coefficients or
//     the exact u(t0));
//   * face points: edge Gauss points x time Gauss points on I_n x F, grouped by
//     neighbour (or boundary edge); the self block takes u = (P, dn),
//     t = (alpha dn + beta P, gamma P) and the cross block the neighbour's
//     basis in the same form (the face lines of eq. dg-bilinear, the boundary
//     lines of eq. dg-linear).
// Each point stages its factors in LDS; then every lane sums its entries of the
// element block (and load) over the pass's points, and the lanes of each
// neighbour group's block sum over that group's points (a group never
// straddles a pass, so every cross block is written once).  The basis
// normalisation is applied to the finished sums in FP64; positions, weights,
// coefficients and the penalty are FP64, the factors and sums are T.
#include "asm_common.h"
#include "kernels.h"
#include "spacetime.h"
#include "wave.h"

namespace dgp {

namespace {

// basis index -> exponents (a, b, c) in the 3D hierarchical order (total degree,
// a descending, then b descending); c is the time exponent
struct StIdx {
    int a[35], b[35], c[35];
};
template <int P>
constexpr StIdx make_st_idx() {
    StIdx r{};
    int n = 0;
    for (int k = 0; k <= P; ++k)
        for (int a = k; a >= 0; --a)
            for (int b = k - a; b >= 0; --b) {
                r.a[n] = a;
                r.b[n] = b;
                r.c[n] = k - a - b;
                ++n;
            }
    return r;
}
// The index table of degree P as one object in device memory: a
// function-local constexpr copy indexed by a run-time basis number is built in
// private memory (scratch) on every call
template <int P>
__device__ constexpr StIdx kStIdx = make_st_idx<P>();

template <typename T, int P>
struct StCfg {
    static constexpr int NB = (P + 1) * (P + 2) * (P + 3) / 6;
    static constexpr int NB2 = NB * NB;
    static constexpr int E = NB2 + NB;               // element block and load
    static constexpr int EPL = (E + 63) / 64;
    static constexpr int QP = (sizeof(T) == 8 && P >= 3) ? 32 : 64;  // points per pass (LDS)
    static constexpr int TDEG = P <= 2 ? 4 : 2 * P;
    static constexpr int NQT = Tri<TDEG>::n;
    static constexpr int NT = P + 1;                 // Gauss points in time
    static constexpr int NGE = P + 1 > 3 ? P + 1 : 3;  // Gauss points per edge
    // LDS row per point: u0 u1 u2 t0 t1 t2 (self) s0 s1 (cross), then L0 L1 and the group
    static constexpr int W = 8 * NB + 3;
};

// unnormalised basis P_a(xi) P_b(eta) P_c(zeta) and its box-coordinate derivatives
template <typename T, int P>
struct StEval {
    static constexpr int NB = StCfg<T, P>::NB;
    T v[NB], dx[NB], dy[NB], dt[NB];
    __device__ __forceinline__ void at(T xi, T eta, T zeta) {
        const StIdx &I = kStIdx<P>;
        T Lx[P + 1], dLx[P + 1], Ly[P + 1], dLy[P + 1], Lt[P + 1], dLt[P + 1];
        legendre<T, P>(xi, Lx, dLx);
        legendre<T, P>(eta, Ly, dLy);
        legendre<T, P>(zeta, Lt, dLt);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            v[i] = Lx[I.a[i]] * Ly[I.b[i]] * Lt[I.c[i]];
            dx[i] = dLx[I.a[i]] * Ly[I.b[i]] * Lt[I.c[i]];
            dy[i] = Lx[I.a[i]] * dLy[I.b[i]] * Lt[I.c[i]];
            dt[i] = Lx[I.a[i]] * Ly[I.b[i]] * dLt[I.c[i]];
        }
    }
};

// sqrt((2a+1)(2b+1)(2c+1)) of basis function i
template <int P>
__device__ __forceinline__ double st_norm(int i) {
    const StIdx &I = kStIdx<P>;
    return sqrt(double((2 * I.a[i] + 1) * (2 * I.b[i] + 1) * (2 * I.c[i] + 1)));
}

__device__ __forceinline__ double st_exact_u(const StSlab &sl, const PointData &pd, double t) {
    return pd.u * (1.0 + sl.tau1 * t + sl.tau2 * t * t);
}

template <typename T, int P, bool ADV>
__global__ void __launch_bounds__(64) k_row_st(StArgs A) {
    using C = StCfg<T, P>;
    constexpr int NB = C::NB, NB2 = C::NB2, E = C::E, EPL = C::EPL, QP = C::QP, W = C::W;
    constexpr int NQT = C::NQT, NT = C::NT, NGE = C::NGE;
    using R_ = Tri<C::TDEG>;
    __shared__ T tab[QP * W];
    __shared__ int s_gleader[kMaxFaces2D], s_gsize[kMaxFaces2D], s_grank[kMaxFaces2D];

    const DevMesh &m = A.m;
    const DevProblem &pr = A.pr;
    const StSlab &sl = A.slab;
    const int lane = threadIdx.x;
    const int c = blockIdx.x;
    const int64_t s0 = m.cell_ptr[c];
    const int nv = (int)(m.cell_ptr[c + 1] - s0);
    const CellGeo g = A.geo[c];
    const Box bx = box_of(g);
    const TrigCentre tc = trig_centre_of(g);
    const double tau = sl.t1 - sl.t0, ct = 2.0 / tau;
    const double ihx = 1.0 / (g.hix - g.lox), ihy = 1.0 / (g.hiy - g.loy);
    const double hst = sqrt(g.h * g.h + tau * tau);
    const double pen_r = g.abar * P * P / hst;
    const int64_t blk0 = A.row_ptr[c];  // the row's first block (uniform degree: values at k NB^2)

    // loop edges, one per lane
    EdgeRec er{};
    if (lane < nv) er = A.erec[s0 + lane];
    const double ex = er.x, ey = er.y;
    const int vid = er.vid, o = lane < nv ? er.o : -3;
    const bool first = (er.rank & kEdgeFirst) != 0;
    // groups: one per neighbour (its edges in loop order), one per boundary edge;
    // the leader records the group's first edge, its point count and block rank
    const bool lead = lane < nv && (first || o < 0);
    const uint64_t gmask = __ballot(lead);
    const int ng = __popcll(gmask);
    if (lead) {
        const int gi = __popcll(gmask & ((1ull << lane) - 1ull));
        const int dup = o >= 0 ? (er.rank >> kEdgeDupShift) & 255 : 1;
        s_gleader[gi] = lane;
        s_gsize[gi] = dup * NGE * NT;
        s_grank[gi] = er.rank & 255;
    }
    __syncthreads();

    T acc[EPL];
#pragma unroll
    for (int k = 0; k < EPL; ++k) acc[k] = T(0);
    const double X0 = readlane_d(ex, 0), Y0 = readlane_d(ey, 0);

    // ---- volume and bottom points
    const int nsub = nv - 2;
    const int QV = nsub * NQT * NT, QB = nsub * NQT;
    for (int base = 0; base < QV + QB; base += QP) {
        const int q = base + lane;
        T *row = tab + lane * W;
        // the point's triangle (for the shuffles every lane takes part)
        int tri = 0, qi = 0, kt = 0;
        const bool vol = q < QV, bot = q >= QV && q < QV + QB;
        if (vol) {
            const int qs = q / NT;
            kt = q - qs * NT;
            tri = qs / NQT;
            qi = qs - tri * NQT;
        } else if (bot) {
            tri = (q - QV) / NQT;
            qi = (q - QV) - tri * NQT;
        }
        const double X1 = __shfl(ex, tri + 1, 64), Y1 = __shfl(ey, tri + 1, 64);
        const double X2 = __shfl(ex, tri + 2, 64), Y2 = __shfl(ey, tri + 2, 64);
        if (lane < QP) {
            for (int k = 0; k < W; ++k) row[k] = T(0);
            if (vol || bot) {
                const double area = 0.5 * ((X1 - X0) * (Y2 - Y0) - (X2 - X0) * (Y1 - Y0));
                // the point as the fan apex plus an offset, and t0 plus an offset in time:
                // box coordinates from the offsets
                const double l1 = R_::l(3 * qi + 1), l2 = R_::l(3 * qi + 2);
                const double dx = l1 * (X1 - X0) + l2 * (X2 - X0), dy = l1 * (Y1 - Y0) + l2 * (Y2 - Y0);
                const double px = X0 + dx, py = Y0 + dy;
                const double wx = R_::w(qi) * area;
                const PointData pd = point_data_near(pr, tc, px, py, vol);
                const int goff = c_gl_off[NT - 1];
                const double tr = vol ? c_gl_t[goff + kt] : 0.0;  // (t - t0) / tau
                const double t = sl.t0 + tr * tau;
                const double w = vol ? wx * c_gl_w[goff + kt] * tau : wx;
                StEval<T, P> ev;
                ev.at(T(((X0 - g.lox) - (g.hix - X0) + 2.0 * dx) * ihx),
                      T(((Y0 - g.loy) - (g.hiy - Y0) + 2.0 * dy) * ihy), T(2.0 * tr - 1.0));
                if (vol) {
                    const double Tt = 1.0 + sl.tau1 * t + sl.tau2 * t * t, dTt = sl.tau1 + 2.0 * sl.tau2 * t;
                    const T cxw = T(bx.cx), cyw = T(bx.cy);
                    const T wt = T(w * ct), wb0 = T(ADV ? w * pr.bx * bx.cx : 0.0),
                            wb1 = T(ADV ? w * pr.by * bx.cy : 0.0), wc = T(ADV ? w * pr.c : 0.0);
                    const T wa = T(w * pd.a);
#pragma unroll
                    for (int i = 0; i < NB; ++i) {
                        row[i] = ev.v[i];
                        row[NB + i] = cxw * ev.dx[i];
                        row[2 * NB + i] = cyw * ev.dy[i];
                        row[3 * NB + i] = wt * ev.dt[i] + wb0 * ev.dx[i] + wb1 * ev.dy[i] + wc * ev.v[i];
                        row[4 * NB + i] = wa * cxw * ev.dx[i];
                        row[5 * NB + i] = wa * cyw * ev.dy[i];
                    }
                    row[8 * NB] = T(w * (pd.u * dTt + Tt * pd.f));
                } else {
                    double uprev;
                    if (A.prev) {
                        // the previous slab's solution at its top (t0): P_c(1) = 1 in its box
                        const StIdx &I = kStIdx<P>;
                        T Lx[P + 1], dLx[P + 1], Ly[P + 1], dLy[P + 1];
                        legendre<T, P>(T(((X0 - g.lox) - (g.hix - X0) + 2.0 * dx) * ihx), Lx, dLx);
                        legendre<T, P>(T(((Y0 - g.loy) - (g.hiy - Y0) + 2.0 * dy) * ihy), Ly, dLy);
                        const double taup = sl.t0 - sl.tp0;
                        const double sp = 1.0 / (g.sqrt_box * sqrt(taup));
                        uprev = 0.0;
                        for (int j = 0; j < NB; ++j)
                            uprev += A.prev[(int64_t)c * NB + j] * st_norm<P>(j) * sp * double(Lx[I.a[j]] * Ly[I.b[j]]);
                    } else {
                        uprev = st_exact_u(sl, pd, sl.t0);
                    }
#pragma unroll
                    for (int i = 0; i < NB; ++i) {
                        row[i] = ev.v[i];
                        row[3 * NB + i] = T(w) * ev.v[i];
                    }
                    row[8 * NB] = T(w * uprev);
                }
            }
        }
        __syncthreads();
        const int nq = min(QP, QV + QB - base);
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            const int e = lane + 64 * k;
            if (e < E) {
                T sum = acc[k];
                if (e < NB2) {
                    const int i = e / NB, j = e - i * NB;
                    for (int qq = 0; qq < nq; ++qq) {
                        const T *r = tab + qq * W;
                        sum += r[i] * r[3 * NB + j] + r[NB + i] * r[4 * NB + j] + r[2 * NB + i] * r[5 * NB + j];
                    }
                } else {
                    const int i = e - NB2;
                    for (int qq = 0; qq < nq; ++qq) sum += tab[qq * W + 8 * NB] * tab[qq * W + i];
                }
                acc[k] = sum;
            }
        }
        __syncthreads();
    }

    // ---- face points, whole groups per pass
    const double isq_r = 1.0 / (g.sqrt_box * sqrt(tau));
    int gnext = 0;
    while (gnext < ng) {
        // groups gnext .. gend - 1 fill this pass
        int gend = gnext, npts = 0;
        while (gend < ng && npts + s_gsize[gend] <= QP) npts += s_gsize[gend++];
        if (gend == gnext) break;  // a group larger than a pass (refused on the host)
        // lane -> (group, edge of the group, edge point, time point)
        int gl = -1, kk = 0, pos = lane;
        for (int gg = gnext; gg < gend; ++gg) {
            if (gl < 0 && pos < s_gsize[gg]) {
                gl = gg;
                kk = pos;
            }
            if (gl < 0) pos -= s_gsize[gg];
        }
        const int ldr = gl >= 0 ? s_gleader[gl] : 0;
        const int og = __shfl(o, ldr, 64);
        // the kk-th point of the group: edge (kk / (NGE NT))-th of the row's edges towards og
        const int ke = kk / (NGE * NT), kp = kk - ke * (NGE * NT), kg = kp / NT, kt = kp - kg * NT;
        int fk = -1, seen = 0;
        for (int k = 0; k < nv; ++k) {
            const int ok = __shfl(o, k, 64);
            if (og >= 0 && ok == og) {
                if (seen == ke && fk < 0) fk = k;
                ++seen;
            }
        }
        if (og < 0) fk = ldr;  // a boundary group is its one edge
        const int f1 = fk >= 0 ? fk : 0, f2 = f1 + 1 == nv ? 0 : f1 + 1;
        const double Xa = __shfl(ex, f1, 64), Ya = __shfl(ey, f1, 64);
        const double Xb = __shfl(ex, f2, 64), Yb = __shfl(ey, f2, 64);
        const int Va = __shfl(vid, f1, 64), Vb = __shfl(vid, f2, 64);
        T *row = tab + lane * W;
        if (lane < QP) {
            for (int k = 0; k < W; ++k) row[k] = T(0);
            row[8 * NB + 2] = T(gl >= 0 ? gl - gnext : -1);
            if (gl >= 0 && fk >= 0 && lane < npts) {
                const bool fwd = Va < Vb;  // canonical order: lower vertex id first
                const double xa = fwd ? Xa : Xb, ya = fwd ? Ya : Yb;
                const double tx = (fwd ? Xb : Xa) - xa, ty = (fwd ? Yb : Ya) - ya;
                const double len = sqrt(tx * tx + ty * ty);
                const double dl = (fwd ? 1.0 : -1.0) / len;
                const double nx = ty * dl, ny = -tx * dl;  // outward for a counter-clockwise loop
                const double bn = pr.bx * nx + pr.by * ny;
                const double up = bn < 0.0 ? bn : 0.0;
                const int goe = c_gl_off[NGE - 1], got = c_gl_off[NT - 1];
                const double te = c_gl_t[goe + kg];
                const double dx = te * tx, dy = te * ty, px = xa + dx, py = ya + dy;
                const double tr = c_gl_t[got + kt];
                const double t = sl.t0 + tr * tau;
                const double w = c_gl_w[goe + kg] * len * c_gl_w[got + kt] * tau;
                StEval<T, P> ev;
                ev.at(T(((xa - g.lox) - (g.hix - xa) + 2.0 * dx) * ihx),
                      T(((ya - g.loy) - (g.hiy - ya) + 2.0 * dy) * ihy), T(2.0 * tr - 1.0));
                const T cnx = T(bx.cx * nx), cny = T(bx.cy * ny);
                T dn[NB];
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    dn[i] = cnx * ev.dx[i] + cny * ev.dy[i];
                    row[i] = ev.v[i];
                    row[NB + i] = dn[i];
                }
                if (og >= 0) {
                    const CellGeo go = A.geo[og];
                    const Box bo = box_of(go);
                    const double hso = sqrt(go.h * go.h + tau * tau);
                    const double sigma = pr.c_sigma * fmax(pen_r, go.abar * P * P / hso);
                    const double a = point_data_near(pr, tc, px, py, false).a;
                    const T al = T(-0.5 * a * w), be = T((sigma - up) * w), ga = T(-0.5 * a * w);
#pragma unroll
                    for (int i = 0; i < NB; ++i) {
                        row[3 * NB + i] = al * dn[i] + be * ev.v[i];
                        row[4 * NB + i] = ga * ev.v[i];
                    }
                    StEval<T, P> eo;
                    eo.at(T(((xa - go.lox) - (go.hix - xa) + 2.0 * dx) / (go.hix - go.lox)),
                          T(((ya - go.loy) - (go.hiy - ya) + 2.0 * dy) / (go.hiy - go.loy)), T(2.0 * tr - 1.0));
                    const T onx = T(bo.cx * nx), ony = T(bo.cy * ny);
                    const T bx_ = T((-sigma + up) * w), gx_ = T(0.5 * a * w);
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        const T dnj = onx * eo.dx[j] + ony * eo.dy[j];
                        row[6 * NB + j] = al * dnj + bx_ * eo.v[j];
                        row[7 * NB + j] = gx_ * eo.v[j];
                    }
                } else if (og == -1) {
                    const PointData pd = point_data(pr, px, py, false);
                    const double gD = st_exact_u(sl, pd, t);
                    const double sigma = pr.c_sigma * pen_r;
                    const T al = T(-pd.a * w), be = T((sigma - up) * w);
#pragma unroll
                    for (int i = 0; i < NB; ++i) {
                        row[3 * NB + i] = al * dn[i] + be * ev.v[i];
                        row[4 * NB + i] = al * ev.v[i];
                    }
                    row[8 * NB] = T((sigma - up) * w * gD);
                    row[8 * NB + 1] = T(-pd.a * w * gD);
                } else {
                    const PointData pd = point_data(pr, px, py, false);
                    const double Tt = 1.0 + sl.tau1 * t + sl.tau2 * t * t;
                    row[8 * NB] = T(w * pd.a * Tt * (pd.ux * nx + pd.uy * ny));
                }
            }
        }
        __syncthreads();
        // element block and load over the pass's points
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            const int e = lane + 64 * k;
            if (e < E) {
                T sum = acc[k];
                if (e < NB2) {
                    const int i = e / NB, j = e - i * NB;
                    for (int qq = 0; qq < npts; ++qq) {
                        const T *r = tab + qq * W;
                        sum += r[i] * r[3 * NB + j] + r[NB + i] * r[4 * NB + j];
                    }
                } else {
                    const int i = e - NB2;
                    for (int qq = 0; qq < npts; ++qq) {
                        const T *r = tab + qq * W;
                        sum += r[8 * NB] * r[i] + r[8 * NB + 1] * r[NB + i];
                    }
                }
                acc[k] = sum;
            }
        }
        // cross blocks of the interior groups of the pass: lane takes entries (group, i, j)
        int gfirst_pt = 0;
        for (int gg = gnext; gg < gend; ++gg) {
            const int ldr2 = s_gleader[gg];
            const int ogg = __shfl(o, ldr2, 64);
            const int sz = s_gsize[gg];
            if (ogg >= 0) {
                const int rank = s_grank[gg];
                const CellGeo go = A.geo[ogg];
                const double isq_o = 1.0 / (go.sqrt_box * sqrt(tau));
                T *vals = static_cast<T *>(A.vals);
                for (int e = lane; e < NB2; e += 64) {
                    const int i = e / NB, j = e - i * NB;
                    T sum = T(0);
                    for (int qq = gfirst_pt; qq < gfirst_pt + sz; ++qq) {
                        const T *r = tab + qq * W;
                        sum += r[i] * r[6 * NB + j] + r[NB + i] * r[7 * NB + j];
                    }
                    vals[(blk0 + rank) * NB2 + e] = T(double(sum) * st_norm<P>(i) * st_norm<P>(j) * isq_r * isq_o);
                }
            }
            gfirst_pt += sz;
        }
        __syncthreads();
        gnext = gend;
    }

    // ---- the element block and the load
    const int drank = A.cnt[4 * c + 3] & 255;
    T *vals = static_cast<T *>(A.vals);
    T *rhs = static_cast<T *>(A.rhs);
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
        const int e = lane + 64 * k;
        if (e < NB2) {
            const int i = e / NB, j = e - i * NB;
            vals[(blk0 + drank) * NB2 + e] = T(double(acc[k]) * st_norm<P>(i) * st_norm<P>(j) * isq_r * isq_r);
        } else if (e < E) {
            const int i = e - NB2;
            rhs[(int64_t)c * NB + i] = T(double(acc[k]) * st_norm<P>(i) * isq_r);
        }
    }
}

template <typename T, int P>
static void launch_st_t(const StArgs &a, hipStream_t st) {
    const bool adv = a.pr.bx != 0.0 || a.pr.by != 0.0 || a.pr.c != 0.0;
    if (adv)
        hipLaunchKernelGGL((k_row_st<T, P, true>), dim3(a.m.n_cells), dim3(64), 0, st, a);
    else
        hipLaunchKernelGGL((k_row_st<T, P, false>), dim3(a.m.n_cells), dim3(64), 0, st, a);
}

}  // namespace

int st_points_per_pass(int precision, int p) {
    return (precision == 0 && p >= 3) ? 32 : 64;
}

bool launch_spacetime(const StArgs &a, int precision, int p, hipStream_t st) {
#define DGP_ST(T, PP)         \
    if (p == PP) {            \
        launch_st_t<T, PP>(a, st); \
        return true;          \
    }
    if (precision == 0) {
        DGP_ST(double, 1) DGP_ST(double, 2) DGP_ST(double, 3)
    } else {
        DGP_ST(float, 1) DGP_ST(float, 2) DGP_ST(float, 3)
    }
#undef DGP_ST
    return false;
}

}  // namespace dgp
