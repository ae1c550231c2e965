// Per-cell geometry in FP64 (kept FP64 in every precision mode):
// bounding box (Section 3.1: the basis lives on it), h_kappa = diam(kappa)
// (Section 2.2), |kappa| by the shoelace formula, and
// abar_kappa = max of a over the cell's volume quadrature points, the discrete
// ||a||_{L_inf(kappa)} of the penalty (Appendix A).  One lane per cell.
#include "dgp_common.h"
#include "kernels.h"
#include "rules_data.h"

namespace dgp {

template <int DEG>
struct TriRule;
template <>
struct TriRule<4> {
    static constexpr int n = DGP_TRI4_N;
    __device__ static const double *l() { return c_tri4_l; }
    __device__ static const double *w() { return c_tri4_w; }
};
template <>
struct TriRule<6> {
    static constexpr int n = DGP_TRI6_N;
    __device__ static const double *l() { return c_tri6_l; }
    __device__ static const double *w() { return c_tri6_w; }
};
template <>
struct TriRule<8> {
    static constexpr int n = DGP_TRI8_N;
    __device__ static const double *l() { return c_tri8_l; }
    __device__ static const double *w() { return c_tri8_w; }
};

template <int DEG>
__device__ double max_a_over_fan(const DevMesh &m, const DevProblem &pr, int64_t s, int nv) {
    using R = TriRule<DEG>;
    const double *L = R::l();
    double x0 = m.x[m.cell_vtx[s]], y0 = m.y[m.cell_vtx[s]];
    double amax = -1e300;
    for (int t = 0; t + 2 < nv; ++t) {
        int v1 = m.cell_vtx[s + t + 1], v2 = m.cell_vtx[s + t + 2];
        double x1 = m.x[v1], y1 = m.y[v1], x2 = m.x[v2], y2 = m.y[v2];
        for (int q = 0; q < R::n; ++q) {
            double px = L[3 * q] * x0 + L[3 * q + 1] * x1 + L[3 * q + 2] * x2;
            double py = L[3 * q] * y0 + L[3 * q + 1] * y1 + L[3 * q + 2] * y2;
            amax = fmax(amax, coef_a(pr, px, py));
        }
    }
    return amax;
}

__global__ void __launch_bounds__(256) k_geometry(DevMesh m, DevProblem pr, CellGeo *geo) {
    int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= m.n_cells) return;
    int64_t s = m.cell_ptr[c];
    int nv = (int)(m.cell_ptr[c + 1] - s);
    double lox = 1e300, loy = 1e300, hix = -1e300, hiy = -1e300, a2 = 0.0, d2 = 0.0;
    for (int i = 0; i < nv; ++i) {
        int vi = m.cell_vtx[s + i];
        double xi = m.x[vi], yi = m.y[vi];
        lox = fmin(lox, xi);
        loy = fmin(loy, yi);
        hix = fmax(hix, xi);
        hiy = fmax(hiy, yi);
        int vn = m.cell_vtx[s + (i + 1 == nv ? 0 : i + 1)];
        a2 += xi * m.y[vn] - m.x[vn] * yi;
        for (int j = i + 1; j < nv; ++j) {
            int vj = m.cell_vtx[s + j];
            double dx = xi - m.x[vj], dy = yi - m.y[vj];
            d2 = fmax(d2, dx * dx + dy * dy);
        }
    }
    CellGeo g;
    g.lox = lox;
    g.loy = loy;
    g.hix = hix;
    g.hiy = hiy;
    g.h = sqrt(d2);
    g.area = 0.5 * a2;
    g.sqrt_box = sqrt((hix - lox) * (hiy - loy));
    if (pr.a1 == 0.0) {
        g.abar = pr.a0;
    } else {
        int p = m.cell_p[c];
        g.abar = p <= 2 ? max_a_over_fan<4>(m, pr, s, nv) : p == 3 ? max_a_over_fan<6>(m, pr, s, nv)
                                                                   : max_a_over_fan<8>(m, pr, s, nv);
    }
    geo[c] = g;
}

void launch_geometry(const DevMesh &m, const DevProblem &pr, CellGeo *geo, hipStream_t st) {
    hipLaunchKernelGGL(k_geometry, dim3((m.n_cells + 255) / 256), dim3(256), 0, st, m, pr, geo);
}

}  // namespace dgp
