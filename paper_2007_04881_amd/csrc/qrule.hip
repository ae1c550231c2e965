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
//                 on the 28 moment equations, one wave per element, and the
//                 acceptance test
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
// (rejected: the element keeps the sub-triangulation rule).  One wave per
// element; J J^T is formed from the node tables without storing J, then
// factored by Cholesky in LDS.
namespace {

struct RefineLds {
    double u[2][3 * kQrNodes];       // current and trial (nodes interleaved xi, eta; then weights)
    double T[2][4][kQrNodes][8];     // P(xi), P'(xi), P(eta), P'(eta) at each node, degrees 0..6
    double G0[NM][NM + 1], G[NM][NM + 1];
    double r[2][NM], z[NM], Mm[NM];
};

// node tables and residual of rule `s` (all 64 lanes; ends with the wave in sync)
__device__ double tables_and_residual(RefineLds &L, int s, int lane) {
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
    __syncthreads();
    double rm = 0.0;
    if (lane < NM) {
        const int a = c_ma[lane], b = c_mb[lane];
        double Q = 0.0;
        for (int k = 0; k < kQrNodes; ++k) Q += L.u[s][2 * kQrNodes + k] * L.T[s][0][k][a] * L.T[s][2][k][b];
        rm = Q - L.Mm[lane];
        L.r[s][lane] = rm;
    }
    __syncthreads();
    return rm;
}

__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

}  // namespace

__global__ void __launch_bounds__(64) k_refine(int n, const double *__restrict__ mom, const double *__restrict__ parea,
                                               const uint8_t *__restrict__ eligible, double *nodes, double *weights,
                                               uint8_t *accepted, double *residual, int32_t *iters, int max_it,
                                               double tol, double mu0) {
    __shared__ RefineLds L;
    const int c = blockIdx.x;
    const int lane = threadIdx.x;
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
    if (lane < NM) L.Mm[lane] = mom[(int64_t)c * NM + lane];
    __syncthreads();
    int cur = 0, it = 0;
    bool ok = false;
    double mu = mu0;
    double rm = tables_and_residual(L, cur, lane);
    double rn2 = wave_sum(rm * rm);
    double res = wave_max(fabs(rm)) / A;
    for (;;) {
        if (res <= tol) {
            ok = true;
            break;
        }
        if (it >= max_it || !(res < 1e300)) break;
        // G0 = J J^T (lower triangle) at the current rule
        for (int idx = lane; idx < NM * (NM + 1) / 2; idx += 64) {
            int m_ = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
            if ((m_ + 1) * (m_ + 2) / 2 <= idx) ++m_;
            if (m_ * (m_ + 1) / 2 > idx) --m_;
            const int n_ = idx - m_ * (m_ + 1) / 2;
            const int am = c_ma[m_], bm = c_mb[m_], an = c_ma[n_], bn = c_mb[n_];
            double g = 0.0;
            for (int k = 0; k < kQrNodes; ++k) {
                const double wk = L.u[cur][2 * kQrNodes + k];
                const double(*T)[kQrNodes][8] = L.T[cur];
                const double vm = T[0][k][am] * T[2][k][bm], vn = T[0][k][an] * T[2][k][bn];
                const double xm = T[1][k][am] * T[2][k][bm], xn = T[1][k][an] * T[2][k][bn];
                const double ym = T[0][k][am] * T[3][k][bm], yn = T[0][k][an] * T[3][k][bn];
                g += wk * wk * (xm * xn + ym * yn) + vm * vn;
            }
            L.G0[m_][n_] = g;
        }
        __syncthreads();
        const double gmax = wave_max(lane < NM ? L.G0[lane][lane] : 0.0);
        bool taken = false;
        while (mu <= 1e6) {
            const double lam = mu * gmax;
            for (int idx = lane; idx < NM * (NM + 1); idx += 64) {
                const int i = idx / (NM + 1), j = idx - i * (NM + 1);
                if (j <= i) L.G[i][j] = L.G0[i][j] + (i == j ? lam : 0.0);
            }
            if (lane < NM) L.z[lane] = L.r[cur][lane];
            __syncthreads();
            // Cholesky, right-looking
            bool spd = true;
            for (int j = 0; j < NM; ++j) {
                const double d = L.G[j][j];
                if (!(d > 0.0)) {
                    spd = false;
                    break;
                }
                const double piv = sqrt(d);
                __syncthreads();
                if (lane == 0) L.G[j][j] = piv;
                if (lane > j && lane < NM) L.G[lane][j] /= piv;
                __syncthreads();
                if (lane > j && lane < NM) {
                    const double lij = L.G[lane][j];
                    for (int k = j + 1; k <= lane; ++k) L.G[lane][k] -= lij * L.G[k][j];
                }
                __syncthreads();
            }
            if (!spd) {
                __syncthreads();
                mu *= 10.0;
                continue;
            }
            // L y = r, then L^T z = y
            for (int j = 0; j < NM; ++j) {
                const double yj = L.z[j] / L.G[j][j];
                __syncthreads();
                if (lane == j) L.z[j] = yj;
                if (lane > j && lane < NM) L.z[lane] -= L.G[lane][j] * yj;
                __syncthreads();
            }
            for (int j = NM - 1; j >= 0; --j) {
                const double zj = L.z[j] / L.G[j][j];
                __syncthreads();
                if (lane == j) L.z[j] = zj;
                if (lane < j) L.z[lane] -= L.G[j][lane] * zj;
                __syncthreads();
            }
            // trial rule u - J^T z
            const int nx = 1 - cur;
            if (lane < 2 * kQrNodes) {
                const int k = lane >> 1, eta = lane & 1;
                double du = 0.0;
                for (int m_ = 0; m_ < NM; ++m_) {
                    const int a = c_ma[m_], b = c_mb[m_];
                    du += L.z[m_] * (eta ? L.T[cur][0][k][a] * L.T[cur][3][k][b] : L.T[cur][1][k][a] * L.T[cur][2][k][b]);
                }
                L.u[nx][lane] = L.u[cur][lane] - du * L.u[cur][2 * kQrNodes + k];
            } else if (lane < 3 * kQrNodes) {
                const int k = lane - 2 * kQrNodes;
                double du = 0.0;
                for (int m_ = 0; m_ < NM; ++m_) du += L.z[m_] * L.T[cur][0][k][c_ma[m_]] * L.T[cur][2][k][c_mb[m_]];
                L.u[nx][lane] = L.u[cur][lane] - du;
            }
            __syncthreads();
            const double rt = tables_and_residual(L, nx, lane);
            const double rtn2 = wave_sum(rt * rt);
            if (rtn2 < rn2) {
                cur = nx;
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
    __syncthreads();
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

void launch_refine(int n, const double *mom, const double *parea, const uint8_t *eligible, double *nodes,
                   double *weights, uint8_t *accepted, double *residual, int32_t *iters, int max_it, double tol,
                   double mu0, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_refine, dim3(n), dim3(64), 0, st, n, mom, parea, eligible, nodes, weights, accepted, residual,
                       iters, max_it, tol, mu0);
}

}  // namespace dgp
