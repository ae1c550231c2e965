// Shared device-side definitions of the dgpoly kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dgp {

constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxP = 4;
constexpr int kLaunchCfgs = 4;  // 2D row-kernel launch configurations (register budget x row order)
constexpr size_t kAltSpillMax = 32;  // bytes per lane of extra spill the larger-occupancy budget may have
constexpr int kInlineTiles = 1024;  // 2D steps on at most this many tiles launch no scan kernel          // 2D kernels are built for p = 1..4
constexpr int kMaxFaces2D = 24;   // faces per polygon handled by the preparation kernel
constexpr int kPrepTile = 32;     // elements per preparation work-group (a tile)

// reduced volume rules: network and moment sizes
constexpr int kQrMaxV = 12;                    // polygons with at most 12 vertices get a reduced rule
constexpr int kQrNodes = 16;                   // nodes per reduced rule
constexpr int kQrIn = 3 * kQrMaxV;             // 24 coordinates + 12 validity flags
constexpr int kQrHidden = 128;
constexpr int kQrOut = 3 * kQrNodes;           // 32 node coordinates + 16 weight logits
constexpr int kQrMoments = 28;                 // Legendre moments of total degree <= 6
// parameter blob: W1[36][128] b1 W2[128][128] b2 W3[128][128] b3 W4[128][48] b4 (FP32, [in][out])
constexpr int kMlpW1 = 0, kMlpB1 = kMlpW1 + kQrIn * kQrHidden;
constexpr int kMlpW2 = kMlpB1 + kQrHidden, kMlpB2 = kMlpW2 + kQrHidden * kQrHidden;
constexpr int kMlpW3 = kMlpB2 + kQrHidden, kMlpB3 = kMlpW3 + kQrHidden * kQrHidden;
constexpr int kMlpW4 = kMlpB3 + kQrHidden, kMlpB4 = kMlpW4 + kQrHidden * kQrOut;
constexpr int kMlpParams = kMlpB4 + kQrOut;    // 43,952

// Device copy of the mesh (structure of arrays, as uploaded).
struct DevMesh {
    int32_t n_cells;
    int32_t n_faces;
    int32_t n_vertices;
    const double *x, *y, *z;  // z: 3D only
    const int64_t *cell_ptr;
    const int32_t *cell_vtx;
    const int8_t *cell_p;
    const int64_t *cell_face_ptr;
    const int32_t *cell_face;
    const int32_t *face_vtx;
    const int32_t *face_cell;
    const int8_t *face_bc;
    const int32_t *face_opp;  // 3D only: vertex of the left cell's tetrahedron opposite the face
};

// Per-cell geometry written by the preparation kernel, one 128-byte record per
// cell (two cache lines).  The reciprocals and the penalty factor are stored
// so that the rows reading a neighbour's record need no division.
struct alignas(64) CellGeo {
    double lox, loy, hix, hiy;  // bounding box
    double h;                   // diameter (largest vertex distance)
    double abar;                // max of a over the volume quadrature points
    double sqrt_box;            // sqrt(|bounding box|), basis normalisation
    double area;                // |kappa|
    double sx, cx, sy, cy;      // sin / cos (pi x), (pi y) at the box centre (0, 1, 0, 1 if unused)
    double ihx, ihy;            // 1 / (hix - lox), 1 / (hiy - loy)
    double isq;                 // 1 / sqrt_box
    double pen;                 // abar p^2 / h at the element's own degree (diameter penalty)
};
static_assert(sizeof(CellGeo) == 128, "two cache lines per element");

// One loop edge of an element as the assembly needs it (32 bytes).
struct alignas(16) EdgeRec {
    double x, y;   // start vertex of the edge
    int32_t vid;   // its global id (orders the edge's points canonically)
    int32_t o;     // neighbour across the edge, or minus the boundary code
    int32_t rank;  // interior edge: position of the neighbour's block in the row (bits 0-7), number of the
                   // row's edges towards that neighbour (bits 8-15), | kEdgeFirst on its first edge
    int32_t voff;  // interior edge: value offset of that block inside the row
};
constexpr int32_t kEdgeFirst = 1 << 30;
constexpr int kEdgeDupShift = 8;

// Outputs of the preparation kernel.
struct PrepOut {
    CellGeo *geo;        // [n_cells]
    int32_t *nbr;        // [loop entries] neighbour across each edge, or -boundary code
    EdgeRec *erec;       // [loop entries]
    int32_t *cnt;        // [n_cells][4] blocks, values, dofs before the element in its tile; diagonal rank | offset << 8
    int32_t *tile_sum;   // [n_tiles][4]: blocks, values and dofs of the tile, then 0
    int64_t *tile_off;   // [n_tiles + 1][3] exclusive prefix of the tile sums (totals last)
    // covering penalty only: [2 n_faces] abar p^2 min(1 / |K^F|, p^2 / |kappa|) of the
    // face's left (2 f) and right (2 f + 1) element; sigma_F = C_sigma |F| max of the two
    double *pen_face;
};

// Problem data as the kernels see it.
struct DevProblem {
    double a0, a1, bx, by, c, c_sigma;
    double bz;  // 3D only
    int32_t u_kind;  // 0 sines, 1 polynomial
    double u[10];
    int32_t penalty;  // 0: C abar p^2 / h; 1: the covering form (pen_face)
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

// Manufactured data at (x, y) from sin/cos(pi x), sin/cos(pi y); the load uses
// the closed-form derivatives of a and u.
// SINES: the caller handles the sine solution only (u_kind 0), so the
// polynomial branch and its coefficients are left out of its code.
template <bool SINES = false>
__device__ __forceinline__ PointData point_data_sc(const DevProblem &pr, double x, double y, double sx, double cx,
                                                   double sy, double cy, bool need_f) {
    PointData d;
    double ax = 0.0, ay = 0.0, lap;
    if (pr.a1 != 0.0) {
        const double s2x = 2.0 * sx * cx, c2x = cx * cx - sx * sx;
        const double s2y = 2.0 * sy * cy, c2y = cy * cy - sy * sy;
        d.a = pr.a0 + pr.a1 * s2x * c2y;
        ax = 2.0 * kPi * pr.a1 * c2x * c2y;
        ay = -2.0 * kPi * pr.a1 * s2x * s2y;
    } else {
        d.a = pr.a0;
    }
    if (SINES || pr.u_kind == 0) {
        d.u = sx * sy;
        d.ux = kPi * cx * sy;
        d.uy = kPi * sx * cy;
        lap = -2.0 * kPi * kPi * d.u;
    } else {
        // the coefficients are read here, at an offset (zero) that an empty
        // scalar move hides from the compiler: plain reads of the kernel
        // argument would be hoisted to the kernel's start, and the six values
        // would hold twelve scalar registers through every loop of the caller
        int z;
        asm volatile("s_mov_b32 %0, 0" : "=s"(z));
        const double *c = pr.u + z;
        d.u = c[0] + c[1] * x + c[2] * y + c[4] * x * x + c[5] * y * y + c[7] * x * y;
        d.ux = c[1] + 2.0 * c[4] * x + c[7] * y;
        d.uy = c[2] + 2.0 * c[5] * y + c[7] * x;
        lap = 2.0 * c[4] + 2.0 * c[5];
    }
    d.f = need_f ? (-(ax * d.ux + ay * d.uy) - d.a * lap + pr.bx * d.ux + pr.by * d.uy + pr.c * d.u) : 0.0;
    return d;
}

__device__ __forceinline__ bool needs_trig(const DevProblem &pr) { return pr.u_kind == 0 || pr.a1 != 0.0; }

// Manufactured data at (x, y) with sin/cos evaluated directly (exact at integer points).
template <bool SINES = false>
__device__ __forceinline__ PointData point_data(const DevProblem &pr, double x, double y, bool need_f) {
    double sx = 0.0, cx = 1.0, sy = 0.0, cy = 1.0;
    if (SINES || needs_trig(pr)) {
        sincospi(x, &sx, &cx);
        sincospi(y, &sy, &cy);
    }
    return point_data_sc<SINES>(pr, x, y, sx, cx, sy, cy, need_f);
}

// sin/cos(pi (x0 + d)) from s0 = sin(pi x0), c0 = cos(pi x0) by angle addition,
// with sin/cos(pi d) from their Taylor series through t^11 / t^10 (t = pi d);
// the truncation error is below 1e-18 for |t| <= kNearT.
constexpr double kNearT = 0.2;
__device__ __forceinline__ void sincospi_near(double s0, double c0, double d, double *s, double *c) {
    const double t = kPi * d, t2 = t * t;
    const double st =
        t * (1.0 + t2 * (-1.0 / 6 + t2 * (1.0 / 120 + t2 * (-1.0 / 5040 + t2 * (1.0 / 362880 + t2 * (-1.0 / 39916800))))));
    const double ct =
        1.0 + t2 * (-0.5 + t2 * (1.0 / 24 + t2 * (-1.0 / 720 + t2 * (1.0 / 40320 + t2 * (-1.0 / 3628800)))));
    *s = s0 * ct + c0 * st;
    *c = c0 * ct - s0 * st;
}

// sin/cos(pi x), sin/cos(pi y) at an element centre, for evaluation at nearby points
struct TrigCentre {
    double x0, y0, sx, cx, sy, cy;
    int near;  // the element fits within |pi d| <= kNearT of the centre
};

__device__ __forceinline__ TrigCentre trig_centre(const DevProblem &pr, double x0, double y0, double half_diam) {
    TrigCentre t;
    t.x0 = x0;
    t.y0 = y0;
    t.sx = 0.0;
    t.cx = 1.0;
    t.sy = 0.0;
    t.cy = 1.0;
    t.near = kPi * half_diam <= kNearT;
    if (needs_trig(pr)) {
        sincospi(x0, &t.sx, &t.cx);
        sincospi(y0, &t.sy, &t.cy);
    }
    return t;
}

// The same from the values stored with the element's geometry.
__device__ __forceinline__ TrigCentre trig_centre_of(const CellGeo &g) {
    TrigCentre t;
    t.x0 = 0.5 * (g.lox + g.hix);
    t.y0 = 0.5 * (g.loy + g.hiy);
    t.sx = g.sx;
    t.cx = g.cx;
    t.sy = g.sy;
    t.cy = g.cy;
    const double hx = g.hix - g.lox, hy = g.hiy - g.loy;
    t.near = kPi * 0.5 * sqrt(hx * hx + hy * hy) <= kNearT;
    return t;
}

// Manufactured data at a point inside the element of centre t.
__device__ __forceinline__ PointData point_data_near(const DevProblem &pr, const TrigCentre &t, double x, double y,
                                                     bool need_f) {
    if (!needs_trig(pr)) return point_data_sc(pr, x, y, 0.0, 1.0, 0.0, 1.0, need_f);
    if (!t.near) return point_data(pr, x, y, need_f);
    double sx, cx, sy, cy;
    sincospi_near(t.sx, t.cx, x - t.x0, &sx, &cx);
    sincospi_near(t.sy, t.cy, y - t.y0, &sy, &cy);
    return point_data_sc(pr, x, y, sx, cx, sy, cy, need_f);
}

// Diffusion coefficient at a point inside the element of centre t.
__device__ __forceinline__ double coef_a_near(const DevProblem &pr, const TrigCentre &t, double x, double y) {
    if (pr.a1 == 0.0) return pr.a0;
    if (!t.near) return coef_a(pr, x, y);
    double sx, cx, sy, cy;
    sincospi_near(t.sx, t.cx, x - t.x0, &sx, &cx);
    sincospi_near(t.sy, t.cy, y - t.y0, &sy, &cy);
    return pr.a0 + pr.a1 * (2.0 * sx * cx) * (cy * cy - sy * sy);
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

// Arguments of the assembly kernel.
struct AsmArgs {
    DevMesh m;
    DevProblem pr;
    const CellGeo *geo;
    const int32_t *nbr;
    const int32_t *cnt;
    const int64_t *tile_off;
    // non-null: no scan was launched; each row sums the tile sums before its
    // own tile (2D meshes of at most kInlineTiles tiles)
    const int4 *tile_sum = nullptr;
    int32_t n_tiles = 0;
    const EdgeRec *erec;
    const double *pen_face;  // covering penalty (PrepOut::pen_face)
    int64_t *row_ptr;
    int32_t *col_idx;
    int64_t *val_ptr;
    int64_t *dof_ptr;
    void *vals;
    void *rhs;
    int values;         // 0: pattern only
    int write_pattern;  // write row_ptr, col_idx, val_ptr, dof_ptr
    int reduced;        // volume matrix of accepted elements with their reduced rule
    const double *qr_nodes;  // [n_cells][16][2] (xi, eta) in box coordinates
    const double *qr_w;      // [n_cells][16] weights in box coordinates
    const uint8_t *qr_ok;    // [n_cells]
    const int32_t *rows;     // rows to assemble (null: all, in order)
    int32_t n_rows;
};

}  // namespace dgp
