// Shared device-side definitions of the dgpoly kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgp {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxP = 4;          // 2D kernels are built for p = 1..4
constexpr int kTile = 256;        // cells per work-group in the pattern kernels
constexpr int kMaxFaces2D = 24;   // faces per polygon handled by the preparation kernel

// State of the single-pass (decoupled look-back) scan over tiles of elements.
struct Lookback {
    unsigned long long *counter;  // tickets, never reset while the mesh lives
    unsigned long long *status;   // per tile: (epoch << 2) | 1 aggregate, | 2 inclusive prefix
    int64_t *agg;                 // per tile: blocks, values, dofs
    int64_t *incl;                // per tile: inclusive prefix of the same
    int *error;                   // set if a look-back ever gives up
};

// Device copy of the mesh (structure of arrays, as uploaded).
struct DevMesh {
    int32_t n_cells;
    int32_t n_faces;
    int32_t n_vertices;
    const double *x, *y;
    const int64_t *cell_ptr;
    const int32_t *cell_vtx;
    const int8_t *cell_p;
    const int64_t *cell_face_ptr;
    const int32_t *cell_face;
    const int32_t *face_vtx;
    const int32_t *face_cell;
    const int8_t *face_bc;
};

// Per-cell geometry written by the geometry kernel, one 64-byte record per
// cell so that a neighbour's data is two 32-byte loads from one cache line.
struct alignas(64) CellGeo {
    double lox, loy, hix, hiy;  // bounding box
    double h;                   // diameter (largest vertex distance)
    double abar;                // max of a over the volume quadrature points
    double sqrt_box;            // sqrt(|bounding box|), basis normalisation
    double area;                // |kappa|
};

// Problem data as the kernels see it.
struct DevProblem {
    double a0, a1, bx, by, c, c_sigma;
    int32_t u_kind;  // 0 sines, 1 polynomial
    double u[10];
};

__host__ __device__ constexpr int nb2d(int p) { return (p + 1) * (p + 2) / 2; }

// Basis exponents in hierarchical order (total degree, x-exponent descending).
__host__ __device__ constexpr int exp_a(int i) {
    return i == 0 ? 0 : i == 1 ? 1 : i == 2 ? 0 : i == 3 ? 2 : i == 4 ? 1 : i == 5 ? 0 : i == 6 ? 3 : i == 7 ? 2
         : i == 8 ? 1 : i == 9 ? 0 : i == 10 ? 4 : i == 11 ? 3 : i == 12 ? 2 : i == 13 ? 1 : 0;
}
__host__ __device__ constexpr int exp_b(int i) {
    return i == 0 ? 0 : i == 1 ? 0 : i == 2 ? 1 : i == 3 ? 0 : i == 4 ? 1 : i == 5 ? 2 : i == 6 ? 0 : i == 7 ? 1
         : i == 8 ? 2 : i == 9 ? 3 : i == 10 ? 0 : i == 11 ? 1 : i == 12 ? 2 : i == 13 ? 3 : 4;
}

// other element of face f as seen from cell c (-1 on the boundary)
__device__ __forceinline__ int other_cell(const DevMesh &m, int f, int c) {
    int l = m.face_cell[2 * f], r = m.face_cell[2 * f + 1];
    return l == c ? r : l;
}

// ------------------------------------------------------------ coefficients
// a(x) = a0 + a1 sin(2 pi x) cos(2 pi y)
__device__ __forceinline__ double coef_a(const DevProblem &pr, double x, double y) {
    if (pr.a1 == 0.0) return pr.a0;
    double s2x, c2x, s2y, c2y;
    sincospi(2.0 * x, &s2x, &c2x);
    sincospi(2.0 * y, &s2y, &c2y);
    return pr.a0 + pr.a1 * s2x * c2y;
}

struct PointData {
    double a;  // diffusion coefficient
    double u;  // manufactured solution (boundary data)
    double f;  // load -div(a grad u) + b.grad u + c u
    double ux, uy;
};

// Manufactured data at (x, y); the load uses the closed-form derivatives of a and u.
__device__ __forceinline__ PointData point_data(const DevProblem &pr, double x, double y, bool need_f) {
    PointData d;
    double ax = 0.0, ay = 0.0, lap;
    double sx = 0.0, cx = 0.0, sy = 0.0, cy = 0.0;
    bool trig = pr.u_kind == 0 || pr.a1 != 0.0;
    if (trig) {
        sincospi(x, &sx, &cx);
        sincospi(y, &sy, &cy);
    }
    if (pr.a1 != 0.0) {
        double s2x = 2.0 * sx * cx, c2x = cx * cx - sx * sx;
        double s2y = 2.0 * sy * cy, c2y = cy * cy - sy * sy;
        d.a = pr.a0 + pr.a1 * s2x * c2y;
        ax = 2.0 * kPi * pr.a1 * c2x * c2y;
        ay = -2.0 * kPi * pr.a1 * s2x * s2y;
    } else {
        d.a = pr.a0;
    }
    if (pr.u_kind == 0) {
        d.u = sx * sy;
        d.ux = kPi * cx * sy;
        d.uy = kPi * sx * cy;
        lap = -2.0 * kPi * kPi * d.u;
    } else {
        const double *c = pr.u;
        d.u = c[0] + c[1] * x + c[2] * y + c[4] * x * x + c[5] * y * y + c[7] * x * y;
        d.ux = c[1] + 2.0 * c[4] * x + c[7] * y;
        d.uy = c[2] + 2.0 * c[5] * y + c[7] * x;
        lap = 2.0 * c[4] + 2.0 * c[5];
    }
    d.f = need_f ? (-(ax * d.ux + ay * d.uy) - d.a * lap + pr.bx * d.ux + pr.by * d.uy + pr.c * d.u) : 0.0;
    return d;
}

// Legendre P_0..P_n and derivatives by the three-term recurrence.
template <typename T, int N>
__device__ __forceinline__ void legendre(T x, T *P, T *dP) {
    P[0] = T(1);
    dP[0] = T(0);
    if (N >= 1) {
        P[1] = x;
        dP[1] = T(1);
    }
#pragma unroll
    for (int n = 1; n < N; ++n) {
        P[n + 1] = T((2.0 * n + 1.0) / (n + 1.0)) * x * P[n] - T(n / (n + 1.0)) * P[n - 1];
        dP[n + 1] = dP[n - 1] + T(2 * n + 1) * P[n];
    }
}

}  // namespace dgp
