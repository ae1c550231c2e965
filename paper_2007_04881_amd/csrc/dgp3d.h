// Polyhedral (3D) meshes: per-cell records of the preparation kernel and the
// arguments of the 3D assembly kernel.
//
// A 3D cell is a union of tetrahedra (four vertex ids each in cell_vtx); its
// faces are the boundary triangles of that union (face_vtx, three ids each),
// interface triangles towards another cell or triangles on the domain
// boundary.  The outward normal of a face follows from face_opp, the vertex of
// the left cell's tetrahedron opposite the triangle.  Volume integrals use the
// 11-point degree-4 rule on every tetrahedron, face integrals the 6-point
// degree-4 rule on every triangle (Section 3: standard rules on the simplices
// of a sub-tessellation), which integrate the mass and penalty terms exactly
// for p <= 2.
#pragma once
#include "dgp_common.h"

namespace dgp {

constexpr int kMaxP3D = 2;         // 3D kernels are built for p = 1, 2
constexpr int kMaxFaces3D = 1024;  // boundary triangles of one polyhedron handled by the preparation kernel
constexpr int kVtxHash3D = 1024;   // LDS hash slots per polyhedron for its distinct surface vertices
constexpr int kMaxVtx3D = 384;     // distinct surface vertices of one polyhedron handled by the preparation kernel
constexpr int kMaxGroups3D = 64;  // face groups (neighbours and boundary codes) of one polyhedron
constexpr int kPrepTile3D = 4;     // cells per tile of the 3D row offsets (one preparation work-group)

__host__ __device__ constexpr int nb3d(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }

// Exponents (a, b, c) of x, y, z of basis function i in hierarchical order
// (total degree, then a descending, then b descending), two bits each.
constexpr unsigned long long kExp3Pack = 0x814211142404040ULL;
__host__ __device__ constexpr int exp3(int i, int d) { return (int)((kExp3Pack >> (6 * i + 2 * d)) & 3); }

// Per-cell geometry (FP64 in every precision mode).
struct alignas(16) CellGeo3 {
    double lo[3], hi[3];  // bounding box
    double h;             // diameter: largest distance between two vertices
    double abar;          // max of a over the element (a is constant in 3D)
    double sqrt_box;      // sqrt(|bounding box|), basis normalisation
    double vol;           // |kappa| (written by the assembly kernel)
    double s[3], c[3];    // sin / cos (pi x_d) at the box centre (0 / 1 when unused)
    int32_t n_groups;     // face groups of the cell (one per neighbour and boundary code)
    int32_t pad[3];
};

// Face group of a cell: `count` consecutive entries from `start` of the cell's
// grouped face list, all towards neighbour `code` (>= 0) or on the boundary
// with code -1 (Dirichlet) / -2 (Neumann); rank_voff = rank of the
// neighbour's block among the row's columns | (value offset inside the row << 8).
struct FaceGroup {
    int32_t start, count, code, rank_voff;
};

struct Prep3Out {
    CellGeo3 *geo;
    int32_t *forder;    // [cell-face entries] face ids grouped by neighbour, same ranges as cell_face
    FaceGroup *grp;     // [cell-face entries] the cell's groups, from the start of its range
    int32_t *cnt;       // [4 n_cells] prefix of blocks / values / dofs in the cell's tile, diagonal rank | offset << 8
    int64_t *tile_sum;  // [3 n_tiles]
    int64_t *tile_off;  // [3 (n_tiles + 1)] exclusive scan, totals last
    int32_t *err;       // set when a cell exceeds the preparation kernel's limits
};

struct Asm3Args {
    DevMesh m;
    DevProblem pr;
    const CellGeo3 *geo;
    const int32_t *forder;
    const FaceGroup *grp;
    const int32_t *cnt;
    const int64_t *tile_off;
    int64_t *row_ptr;
    int32_t *col_idx;
    int64_t *val_ptr;
    int64_t *dof_ptr;
    void *vals;
    void *rhs;
    int32_t values;         // 0: write the pattern only
    int32_t write_pattern;  // 1: write row_ptr / col_idx / val_ptr / dof_ptr
    const int32_t *rows;    // rows of one degree (mixed degrees), or null for all cells
    int32_t n_rows;
};

}  // namespace dgp
