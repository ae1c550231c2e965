// Reduced volume quadrature for polygonal elements.
//
// Every element is mapped to [-1, 1]^2 by its bounding box -- the box on which
// its Legendre basis lives (Section 3.1) -- so a rule found in those
// coordinates serves the basis directly.  A 16-node rule replaces the fan
// sub-triangulation for the volume matrix when it reproduces the element's
// Legendre moments of total degree <= 6, enough for every element integrand
// of p <= 3 with constant coefficients (the sub-triangulation rule of
// Section 3.3 needs (n_v - 2) x 12 points for the same degree).
//
// Kernels:
//   k_cell_poly   element -> normalised polygon, network features, moments
//   k_train_poly  the same for seeded random polygons (training data)
//   k_rule_init   initial rule from the network output, or the 4 x 4 Gauss
//                 tensor rule scaled to the polygon's area
//   k_refine      FP64 damped minimum-norm Gauss-Newton (Levenberg-Marquardt)
//                 on the 28 moment equations, one wave per element
//                 (Gauss-Jordan in registers), and the acceptance test
#include "dgp_common.h"
#include "kernels.h"
#include "rules_data.h"

namespace dgp {

namespace {

constexpr int WG_POLY = 128;
constexpr int NM = kQrMoments;

// exponents (a, b) of moment m: total degree 0..6, a descending
__constant__ signed char c_ma[NM] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0, 4, 3, 2, 1, 0, 5, 4, 3, 2, 1, 0, 6, 5, 4, 3, 2, 1, 0};
__constant__ signed char c_mb[NM] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4, 0, 1, 2, 3, 4, 5, 0, 1, 2, 3, 4, 5, 6};

// Legendre values P_0..P_6 (three-term recurrence)
__device__ __forceinline__ void leg6(double x, double *P) {
    P[0] = 1.0;
    P[1] = x;
#pragma unroll
    for (int n = 1; n < 6; ++n) P[n + 1] = ((2.0 * n + 1.0) * x * P[n] - n * P[n - 1]) / (n + 1.0);
}

// Moments int_P P_a(xi) P_b(eta), a + b <= 6, of the polygon held in
// s_x/s_y[v * WG_POLY + lane] (m vertices, counter-clockwise), by the
// degree-6 rule on the fan from vertex 0 (signed areas: exact for every
// simple polygon whose fan triangles are oriented consistently).
__device__ void poly_moments(const double *s_x, const double *s_y, int lane, int m, double *M) {
#pragma unroll
    for (int i = 0; i < NM; ++i) M[i] = 0.0;
    const double x0 = s_x[lane], y0 = s_y[lane];
    for (int t = 1; t + 1 < m; ++t) {
        const double x1 = s_x[t * WG_POLY + lane], y1 = s_y[t * WG_POLY + lane];
        const double x2 = s_x[(t + 1) * WG_POLY + lane], y2 = s_y[(t + 1) * WG_POLY + lane];
        const double A = 0.5 * ((x1 - x0) * (y2 - y0) - (x2 - x0) * (y1 - y0));
        for (int q = 0; q < DGP_TRI6_N; ++q) {
            const double l0 = c_tri6_l[3 * q], l1 = c_tri6_l[3 * q + 1], l2 = c_tri6_l[3 * q + 2];
            const double px = l0 * x0 + l1 * x1 + l2 * x2, py = l0 * y0 + l1 * y1 + l2 * y2;
            const double W = c_tri6_w[q] * A;
            double Lx[7], Ly[7];
            leg6(px, Lx);
            leg6(py, Ly);
#pragma unroll
            for (int i = 0; i < NM; ++i) M[i] += W * Lx[c_ma[i]] * Ly[c_mb[i]];
        }
    }
}

// Shared tail of both polygon kernels: rotate the normalised loop so that it
// starts at its smallest xi (then smallest eta), fix the orientation, and
// write features, moments and area.  On entry s_x/s_y hold the m normalised
// vertices in loop order.
__device__ void finish_polygon(double *s_x, double *s_y, int lane, int m, int64_t idx, float *feat, double *feat64,
                               double *mom, double *parea) {
    double a2 = 0.0;
    for (int i = 0; i < m; ++i) {
        const int j = i + 1 == m ? 0 : i + 1;
        a2 += s_x[i * WG_POLY + lane] * s_y[j * WG_POLY + lane] - s_x[j * WG_POLY + lane] * s_y[i * WG_POLY + lane];
    }
    if (a2 < 0.0) {  // clockwise input: reverse the loop
        for (int i = 0, j = m - 1; i < j; ++i, --j) {
            const double tx = s_x[i * WG_POLY + lane], ty = s_y[i * WG_POLY + lane];
            s_x[i * WG_POLY + lane] = s_x[j * WG_POLY + lane];
            s_y[i * WG_POLY + lane] = s_y[j * WG_POLY + lane];
            s_x[j * WG_POLY + lane] = tx;
            s_y[j * WG_POLY + lane] = ty;
        }
        a2 = -a2;
    }
    int st = 0;
    for (int i = 1; i < m; ++i) {
        const double xi = s_x[i * WG_POLY + lane], yi = s_y[i * WG_POLY + lane];
        const double xs = s_x[st * WG_POLY + lane], ys = s_y[st * WG_POLY + lane];
        if (xi < xs || (xi == xs && yi < ys)) st = i;
    }
    // rotate in place by st (three reversals)
    auto rev = [&](int i, int j) {
        for (; i < j; ++i, --j) {
            const double tx = s_x[i * WG_POLY + lane], ty = s_y[i * WG_POLY + lane];
            s_x[i * WG_POLY + lane] = s_x[j * WG_POLY + lane];
            s_y[i * WG_POLY + lane] = s_y[j * WG_POLY + lane];
            s_x[j * WG_POLY + lane] = tx;
            s_y[j * WG_POLY + lane] = ty;
        }
    };
    if (st > 0) {
        rev(0, st - 1);
        rev(st, m - 1);
        rev(0, m - 1);
    }
    float *f = feat + idx * kQrIn;
    for (int i = 0; i < kQrMaxV; ++i) {
        const double xi = i < m ? s_x[i * WG_POLY + lane] : 0.0, yi = i < m ? s_y[i * WG_POLY + lane] : 0.0;
        f[2 * i] = (float)xi;
        f[2 * i + 1] = (float)yi;
        f[2 * kQrMaxV + i] = i < m ? 1.0f : 0.0f;
        if (feat64) {
            feat64[idx * kQrIn + 2 * i] = xi;
            feat64[idx * kQrIn + 2 * i + 1] = yi;
            feat64[idx * kQrIn + 2 * kQrMaxV + i] = i < m ? 1.0 : 0.0;
        }
    }
    double M[NM];
    poly_moments(s_x, s_y, lane, m, M);
#pragma unroll
    for (int i = 0; i < NM; ++i) mom[idx * NM + i] = M[i];
    parea[idx] = 0.5 * a2;
}

__device__ __forceinline__ double clip1(double v) { return v < -1.0 ? -1.0 : v > 1.0 ? 1.0 : v; }

// ----------------------------------------------------------------- Philox
// Philox-4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11).
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// [0, 1) from the top 24 bits (exact in FP32 and FP64)
__device__ __forceinline__ double unit24(uint32_t u) { return (double)(u >> 8) * (1.0 / 16777216.0); }

}  // namespace

__global__ void __launch_bounds__(WG_POLY) k_cell_poly(DevMesh m, const CellGeo *__restrict__ geo, float *feat,
                                                       double *mom, double *parea, uint8_t *eligible) {
    __shared__ double s_x[kQrMaxV * WG_POLY], s_y[kQrMaxV * WG_POLY];
    const int lane = threadIdx.x;
    const int c = blockIdx.x * WG_POLY + lane;
    if (c >= m.n_cells) return;
    const int64_t s = m.cell_ptr[c];
    const int nv = (int)(m.cell_ptr[c + 1] - s);
    if (nv > kQrMaxV) {
        eligible[c] = 0;
        for (int i = 0; i < kQrIn; ++i) feat[(int64_t)c * kQrIn + i] = 0.0f;
        for (int i = 0; i < NM; ++i) mom[(int64_t)c * NM + i] = 0.0;
        parea[c] = 0.0;
        return;
    }
    const CellGeo g = geo[c];
    for (int i = 0; i < nv; ++i) {
        const int v = m.cell_vtx[s + i];
        const double x = m.x[v], y = m.y[v];
        // ((x - lo) - (hi - x)) / (hi - lo): the box's extreme vertices map to -1 and 1 exactly
        s_x[i * WG_POLY + lane] = clip1(((x - g.lox) - (g.hix - x)) / (g.hix - g.lox));
        s_y[i * WG_POLY + lane] = clip1(((y - g.loy) - (g.hiy - y)) / (g.hiy - g.loy));
    }
    eligible[c] = 1;
    finish_polygon(s_x, s_y, lane, nv, c, feat, nullptr, mom, parea);
}

// Training polygon `first + i`: Philox-4x32-10 under the key (seed low word,
// seed high word), counter (index, j, 0, 0) for draw j.  Draw 0: vertex count
// 3..12, convex or star-shaped, ellipse aspect, rotation; draw j >= 1: angle
// jitter and radius of vertex j - 1.  Angles are stratified, so the vertices
// come out in counter-clockwise order and nothing is rejected.
__global__ void __launch_bounds__(WG_POLY) k_train_poly(uint64_t seed, int64_t first, int64_t n, float *feat,
                                                        double *feat64, double *mom, double *parea) {
    __shared__ double s_x[kQrMaxV * WG_POLY], s_y[kQrMaxV * WG_POLY];
    const int lane = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * WG_POLY + lane;
    if (i >= n) return;
    const uint32_t k0 = (uint32_t)(seed & 0xFFFFFFFFu), k1 = (uint32_t)(seed >> 32);
    const uint32_t index = (uint32_t)(first + i);
    uint32_t u[4] = {index, 0u, 0u, 0u};
    philox4x32_10(u, k0, k1);
    const int mv = 3 + (int)(unit24(u[0]) * 10.0);
    const bool convex = unit24(u[1]) < 0.5;
    const double aspect = __dadd_rn(0.3, __dmul_rn(0.7, unit24(u[2])));
    const double rot = 2.0 * kPi * unit24(u[3]);
    double lox = 1e300, loy = 1e300, hix = -1e300, hiy = -1e300;
    for (int k = 0; k < mv; ++k) {
        uint32_t d[4] = {index, (uint32_t)(k + 1), 0u, 0u};
        philox4x32_10(d, k0, k1);
        const double th = __dadd_rn(__ddiv_rn(__dmul_rn(2.0 * kPi, __dadd_rn(k + 0.1, __dmul_rn(0.8, unit24(d[0])))), mv),
                                    rot);
        double sn, cs;
        sincos(th, &sn, &cs);
        double x, y;
        if (convex) {
            x = cs;
            y = __dmul_rn(aspect, sn);
        } else {
            const double r = __dadd_rn(0.35, __dmul_rn(0.65, unit24(d[1])));
            x = __dmul_rn(r, cs);
            y = __dmul_rn(r, sn);
        }
        s_x[k * WG_POLY + lane] = x;
        s_y[k * WG_POLY + lane] = y;
        lox = fmin(lox, x);
        loy = fmin(loy, y);
        hix = fmax(hix, x);
        hiy = fmax(hiy, y);
    }
    for (int k = 0; k < mv; ++k) {
        const double x = s_x[k * WG_POLY + lane], y = s_y[k * WG_POLY + lane];
        s_x[k * WG_POLY + lane] = clip1(__ddiv_rn(__dsub_rn(__dsub_rn(x, lox), __dsub_rn(hix, x)), __dsub_rn(hix, lox)));
        s_y[k * WG_POLY + lane] = clip1(__ddiv_rn(__dsub_rn(__dsub_rn(y, loy), __dsub_rn(hiy, y)), __dsub_rn(hiy, loy)));
    }
    finish_polygon(s_x, s_y, lane, mv, i, feat, feat64, mom, parea);
}

// Initial rules: from the network output z [n][48] (nodes tanh(z_0..31) as
// (xi, eta) pairs, weights |P| softmax(z_32..47)), or, with z == nullptr, the
// 4 x 4 Gauss tensor rule on [-1, 1]^2 with weights scaled to |P| / 4.
__global__ void k_rule_init(int n, const float *__restrict__ z, const double *__restrict__ parea, double *nodes,
                            double *weights) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const double A = parea[c];
    if (z) {
        const float *zc = z + (int64_t)c * kQrOut;
        for (int i = 0; i < 2 * kQrNodes; ++i) nodes[(int64_t)c * 2 * kQrNodes + i] = tanh((double)zc[i]);
        double smax = -1e300;
        for (int k = 0; k < kQrNodes; ++k) smax = fmax(smax, (double)zc[2 * kQrNodes + k]);
        double e[kQrNodes], sum = 0.0;
#pragma unroll
        for (int k = 0; k < kQrNodes; ++k) {
            e[k] = exp((double)zc[2 * kQrNodes + k] - smax);
            sum += e[k];
        }
#pragma unroll
        for (int k = 0; k < kQrNodes; ++k) weights[(int64_t)c * kQrNodes + k] = A * (e[k] / sum);
    } else {
        // Gauss-Legendre, 4 points on [-1, 1]
        const double t[4] = {-0.8611363115940526, -0.3399810435848563, 0.3399810435848563, 0.8611363115940526};
        const double w[4] = {0.3478548451374538, 0.6521451548625461, 0.6521451548625461, 0.3478548451374538};
        for (int i = 0; i < 4; ++i)
            for (int j = 0; j < 4; ++j) {
                const int k = 4 * i + j;
                nodes[(int64_t)c * 2 * kQrNodes + 2 * k] = t[i];
                nodes[(int64_t)c * 2 * kQrNodes + 2 * k + 1] = t[j];
                weights[(int64_t)c * kQrNodes + k] = A * 0.25 * w[i] * w[j];
            }
    }
}

// Damped minimum-norm Gauss-Newton (Levenberg-Marquardt) on Q(u) = M,
// u = (nodes, weights) in R^48, Q_ab(u) = sum_k w_k P_a(xi_k) P_b(eta_k):
//     du = -J^T (J J^T + mu g I)^{-1} (Q(u) - M),   g = max diag(J J^T);
// a step is taken only if it lowers ||Q - M||_2 (then mu /= 10), otherwise mu
// grows tenfold and the step is recomputed.  Stops as soon as
// max_ab |Q_ab - M_ab| / |P| <= tol (accepted) or after max_it steps
// (rejected: the element keeps the sub-triangulation rule).
//
// One wave per element, each wave with its own LDS, no work-group barriers:
// lanes k < 16 tabulate the Legendre polynomials at node k; J J^T (28 x 28,
// lower triangle) is formed entry-parallel from the tables; lane i < 28 then holds
// row i of J J^T + mu g I and Gauss-Jordan elimination broadcasts each pivot
// row through scalar registers; lane c < 48 forms component c of J^T z.
namespace {

constexpr int RWAVES = 2;  // elements (waves) per work-group

struct RefineLds {
    double T[2][4][kQrNodes][8];  // per rule slot: P(xi), P'(xi), P(eta), P'(eta) at each node, degrees 0..6
    double G[32][33];
    double u[2][3 * kQrNodes];    // per rule slot: (xi_k, eta_k) interleaved, then w_k
};

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// exponents of moment m (total degree order, a descending)
__host__ __device__ constexpr int mom_a(int m) {
    int d = 0;
    while ((d + 1) * (d + 2) / 2 <= m) ++d;
    return d - (m - d * (d + 1) / 2);
}
__host__ __device__ constexpr int mom_b(int m) {
    int d = 0;
    while ((d + 1) * (d + 2) / 2 <= m) ++d;
    return m - d * (d + 1) / 2;
}

// tables of rule slot s (lanes < 32), then the residual of moment lane m < 28 (0 on other lanes)
__device__ double tables_residual(RefineLds &L, int s, int lane, int am, int bm, double Mm) {
    if (lane < 2 * kQrNodes) {
        const int k = lane & (kQrNodes - 1), eta = lane >= kQrNodes;
        double P[7], dP[7];
        legendre<double, 6>(L.u[s][2 * k + eta], P, dP);
#pragma unroll
        for (int d = 0; d < 7; ++d) {
            L.T[s][2 * eta][k][d] = P[d];
            L.T[s][2 * eta + 1][k][d] = dP[d];
        }
    }
    wave_sync();
    double r = 0.0;
    if (lane < NM) {
        double Q = 0.0;
        for (int k = 0; k < kQrNodes; ++k) Q += L.u[s][2 * kQrNodes + k] * L.T[s][0][k][am] * L.T[s][2][k][bm];
        r = Q - Mm;
    }
    return r;
}

// entry (m, c) of J at rule slot s (m < 28 real rows; rows 28..31 are zero)
__device__ __forceinline__ double jac(const RefineLds &L, int s, int m, int c) {
    if (m >= NM) return 0.0;
    const int a = mom_a(m), b = mom_b(m);
    if (c >= 2 * kQrNodes) {
        const int k = c - 2 * kQrNodes;
        return L.T[s][0][k][a] * L.T[s][2][k][b];
    }
    const int k = c >> 1;
    const double w = L.u[s][2 * kQrNodes + k];
    return (c & 1) ? w * L.T[s][0][k][a] * L.T[s][3][k][b] : w * L.T[s][1][k][a] * L.T[s][2][k][b];
}

}  // namespace

__global__ void __launch_bounds__(64 * RWAVES) k_refine(int n, const double *__restrict__ mom,
                                                        const double *__restrict__ parea,
                                                        const uint8_t *__restrict__ eligible, double *nodes,
                                                        double *weights, uint8_t *accepted, double *residual,
                                                        int32_t *iters, int max_it, double tol, double mu0) {
    __shared__ RefineLds Lw[RWAVES];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = blockIdx.x * RWAVES + wv;
    if (c >= n) return;
    RefineLds &L = Lw[wv];
    if (!eligible[c]) {
        if (lane == 0) {
            accepted[c] = 0;
            residual[c] = INFINITY;
            iters[c] = 0;
        }
        return;
    }
    const double A = parea[c];
    if (lane < 2 * kQrNodes) L.u[0][lane] = nodes[(int64_t)c * 2 * kQrNodes + lane];
    if (lane < kQrNodes) L.u[0][2 * kQrNodes + lane] = weights[(int64_t)c * kQrNodes + lane];
    const int am = lane < NM ? mom_a(lane) : 0, bm = lane < NM ? mom_b(lane) : 0;
    const double Mm = lane < NM ? mom[(int64_t)c * NM + lane] : 0.0;
    wave_sync();
    int cur = 0, it = 0;
    bool ok = false;
    double mu = mu0;
    double rm = tables_residual(L, cur, lane, am, bm, Mm);
    double rn2 = wave_sum(rm * rm);
    double res = wave_max(fabs(rm)) / A;
    for (;;) {
        if (res <= tol) {
            ok = true;
            break;
        }
        if (it >= max_it || !(res < 1e300)) break;
        // G0 = J J^T: lanes over the 406 entries of the lower triangle (mirrored)
        for (int idx = lane; idx < NM * (NM + 1) / 2; idx += 64) {
            int m_ = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
            if ((m_ + 1) * (m_ + 2) / 2 <= idx) ++m_;
            if (m_ * (m_ + 1) / 2 > idx) --m_;
            const int n_ = idx - m_ * (m_ + 1) / 2;
            const int a1 = mom_a(m_), b1 = mom_b(m_), a2 = mom_a(n_), b2 = mom_b(n_);
            const double(*T)[kQrNodes][8] = L.T[cur];
            double gv = 0.0;
            for (int k = 0; k < kQrNodes; ++k) {
                const double wk = L.u[cur][2 * kQrNodes + k];
                const double vm = T[0][k][a1] * T[2][k][b1], vn = T[0][k][a2] * T[2][k][b2];
                const double xm = T[1][k][a1] * T[2][k][b1], xn = T[1][k][a2] * T[2][k][b2];
                const double ym = T[0][k][a1] * T[3][k][b1], yn = T[0][k][a2] * T[3][k][b2];
                gv += wk * wk * (xm * xn + ym * yn) + vm * vn;
            }
            L.G[m_][n_] = gv;
            L.G[n_][m_] = gv;
        }
        wave_sync();
        double grow[NM];
#pragma unroll
        for (int k = 0; k < NM; ++k) grow[k] = lane < NM ? L.G[lane][k] : 0.0;
        const double gmax = wave_max(lane < NM ? L.G[lane][lane] : 0.0);
        bool taken = false;
        while (mu <= 1e6) {
            const double lam = mu * gmax;
            // Gauss-Jordan on (G0 + lam I) z = r, lane i owns row i
            double g[NM];
#pragma unroll
            for (int k = 0; k < NM; ++k) g[k] = grow[k] + (k == lane ? lam : 0.0);
            double z = rm, diag = 1.0;
            bool spd = true;
#pragma unroll
            for (int j = 0; j < NM; ++j) {
                const double piv = readlane_d(g[j], j);
                if (!(piv > 0.0)) spd = false;
                const double inv = 1.0 / piv;
                const double zj = readlane_d(z, j);
                const double f = (lane == j || lane >= NM) ? 0.0 : g[j] * inv;
#pragma unroll
                for (int k = j + 1; k < NM; ++k) g[k] -= f * readlane_d(g[k], j);
                z -= f * zj;
                if (lane == j) diag = piv;
            }
            if (!spd) {
                mu *= 10.0;
                continue;
            }
            z = lane < NM ? z / diag : 0.0;
            // trial rule u - J^T z (lane c < 48 owns component c)
            const int nx = 1 - cur;
            if (lane < 3 * kQrNodes) {
                double du = 0.0;
#pragma unroll
                for (int m_ = 0; m_ < NM; ++m_) du += jac(L, cur, m_, lane) * readlane_d(z, m_);
                L.u[nx][lane] = L.u[cur][lane] - du;
            }
            wave_sync();
            const double rt = tables_residual(L, nx, lane, am, bm, Mm);
            const double rtn2 = wave_sum(rt * rt);
            if (rtn2 < rn2) {
                cur = nx;
                rm = rt;
                rn2 = rtn2;
                res = wave_max(fabs(rt)) / A;
                mu = fmax(mu * 0.1, 1e-15);
                taken = true;
                break;
            }
            mu *= 10.0;
        }
        if (!taken) break;
        ++it;
    }
    wave_sync();
    if (lane < 2 * kQrNodes) nodes[(int64_t)c * 2 * kQrNodes + lane] = L.u[cur][lane];
    if (lane < kQrNodes) weights[(int64_t)c * kQrNodes + lane] = L.u[cur][2 * kQrNodes + lane];
    if (lane == 0) {
        accepted[c] = ok ? 1 : 0;
        residual[c] = res;
        iters[c] = it;
    }
}

void launch_cell_poly(const DevMesh &m, const CellGeo *geo, float *feat, double *mom, double *parea, uint8_t *eligible,
                      hipStream_t st) {
    const int nb = (m.n_cells + WG_POLY - 1) / WG_POLY;
    hipLaunchKernelGGL(k_cell_poly, dim3(nb), dim3(WG_POLY), 0, st, m, geo, feat, mom, parea, eligible);
}

void launch_train_poly(uint64_t seed, int64_t first, int64_t n, float *feat, double *feat64, double *mom,
                       double *parea, hipStream_t st) {
    if (n <= 0) return;
    const int nb = (int)((n + WG_POLY - 1) / WG_POLY);
    hipLaunchKernelGGL(k_train_poly, dim3(nb), dim3(WG_POLY), 0, st, seed, first, n, feat, feat64, mom, parea);
}

void launch_rule_init(int n, const float *z, const double *parea, double *nodes, double *weights, hipStream_t st) {
    hipLaunchKernelGGL(k_rule_init, dim3((n + 255) / 256), dim3(256), 0, st, n, z, parea, nodes, weights);
}

// Keep, per element, the start with the smaller initial moment residual:
// the network's (in nodes / weights) or the template's (nodes_t / w_t);
// start_tmpl[c] = 1 where the template's was kept.
__global__ void k_rule_pick(int n, const double *__restrict__ res_net, const double *__restrict__ res_tmpl,
                            double *nodes, double *weights, const double *__restrict__ nodes_t,
                            const double *__restrict__ w_t, uint8_t *start_tmpl) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const bool tmpl = res_tmpl[c] < res_net[c];
    start_tmpl[c] = tmpl;
    if (tmpl) {
        for (int i = 0; i < 2 * kQrNodes; ++i) nodes[(int64_t)c * 2 * kQrNodes + i] = nodes_t[(int64_t)c * 2 * kQrNodes + i];
        for (int k = 0; k < kQrNodes; ++k) weights[(int64_t)c * kQrNodes + k] = w_t[(int64_t)c * kQrNodes + k];
    }
}

// Elements to start again from the template: eligible, not accepted, started from the network.
__global__ void k_rule_retry_mask(int n, const uint8_t *__restrict__ elig, const uint8_t *__restrict__ acc,
                                  const uint8_t *__restrict__ start_tmpl, uint8_t *mask) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n) mask[c] = elig[c] && !acc[c];  // either start (start_tmpl kept for the statistics)
}

// Take the retried rules that were accepted (their steps add to the first attempt's).
__global__ void k_rule_merge(int n, const uint8_t *__restrict__ mask, const uint8_t *__restrict__ acc2,
                             const double *__restrict__ res2, const int32_t *__restrict__ it2,
                             const double *__restrict__ nodes2, const double *__restrict__ w2, double *nodes,
                             double *weights, uint8_t *acc, double *res, int32_t *it) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n || !mask[c]) return;
    it[c] += it2[c];
    if (!acc2[c]) return;
    for (int i = 0; i < 2 * kQrNodes; ++i) nodes[(int64_t)c * 2 * kQrNodes + i] = nodes2[(int64_t)c * 2 * kQrNodes + i];
    for (int k = 0; k < kQrNodes; ++k) weights[(int64_t)c * kQrNodes + k] = w2[(int64_t)c * kQrNodes + k];
    acc[c] = 1;
    res[c] = res2[c];
}

void launch_rule_pick(int n, const double *res_net, const double *res_tmpl, double *nodes, double *weights,
                      const double *nodes_t, const double *w_t, uint8_t *start_tmpl, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_rule_pick, dim3((n + 255) / 256), dim3(256), 0, st, n, res_net, res_tmpl, nodes, weights,
                       nodes_t, w_t, start_tmpl);
}

void launch_rule_retry_mask(int n, const uint8_t *elig, const uint8_t *acc, const uint8_t *start_tmpl, uint8_t *mask,
                            hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_rule_retry_mask, dim3((n + 255) / 256), dim3(256), 0, st, n, elig, acc, start_tmpl, mask);
}

void launch_rule_merge(int n, const uint8_t *mask, const uint8_t *acc2, const double *res2, const int32_t *it2,
                       const double *nodes2, const double *w2, double *nodes, double *weights, uint8_t *acc,
                       double *res, int32_t *it, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_rule_merge, dim3((n + 255) / 256), dim3(256), 0, st, n, mask, acc2, res2, it2, nodes2, w2,
                       nodes, weights, acc, res, it);
}

void launch_refine(int n, const double *mom, const double *parea, const uint8_t *eligible, double *nodes,
                   double *weights, uint8_t *accepted, double *residual, int32_t *iters, int max_it, double tol,
                   double mu0, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_refine, dim3((n + RWAVES - 1) / RWAVES), dim3(64 * RWAVES), 0, st, n, mom, parea, eligible,
                       nodes, weights, accepted, residual, iters, max_it, tol, mu0);
}

}  // namespace dgp
