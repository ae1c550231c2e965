// Host-side context behind the C ABI (private to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <vector>

#include "../../include/dgpoly.h"
#include "dgp_common.h"
#include "dgp3d.h"

struct dgp_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    hipStream_t cap_stream = nullptr;  // used while capturing a graph
    char err[512] = {0};

    // mesh
    bool has_mesh = false;
    int dim = 2;
    int64_t n_cells = 0, n_faces = 0, n_vertices = 0, n_cell_vtx = 0;
    int p_uniform = -1;                // common degree, or -1 when degrees differ
    int p_max = 0;
    int32_t *rows_by_p = nullptr;      // mixed degrees: element ids grouped by degree (stable)
    int64_t rows_off[dgp::kMaxP + 2] = {};  // group of degree p: rows_by_p[rows_off[p] .. rows_off[p + 1])
    int32_t *rows_sub = nullptr;  // 2D: element ids by degree, then per XCD range most fan sub-triangles first; same rows_off
    int32_t *rows_lpt = nullptr;  // 2D mixed degrees: all element ids by (degree, sub-triangles) descending
    int32_t *rows_3d = nullptr;   // 3D, one degree: element ids along a Morton curve of their first vertex
    int64_t n_boundary_faces = 0;
    int max_dup2d = 1;            // 2D: most edges one cell shares with one neighbour
    std::vector<void *> mesh_bufs;
    dgp::DevMesh dm{};

    // pattern (col_idx / val_ptr sized by the upper bound n_cells + n_cell_vtx)
    bool has_pattern = false;
    int64_t nnzb = 0, n_vals = 0, n_dofs = 0;
    int64_t *row_ptr = nullptr, *val_ptr = nullptr, *dof_ptr = nullptr;
    int32_t *col_idx = nullptr;
    // preparation outputs and the assembly's bookkeeping (one allocation)
    void *work = nullptr;
    dgp::PrepOut prep{};
    dgp::Prep3Out prep3{};  // 3D meshes
    int64_t n_cell_face = 0;
    int n_tiles = 0;


    void *static_scratch = nullptr;  // device address of the library's static scratch array on this device

    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    // reduced volume rules (element data, network, fitted rules)
    float *mlp = nullptr;          // parameters on the device
    bool has_mlp = false;
    bool has_qrule = false;
    void *qr_buf = nullptr;        // one allocation, carved below
    float *qr_feat = nullptr;      // [n_cells][36]
    double *qr_mom = nullptr;      // [n_cells][28]
    double *qr_area = nullptr;     // [n_cells]  |P| in box coordinates
    double *qr_nodes = nullptr;    // [n_cells][32]
    double *qr_w = nullptr;        // [n_cells][16]
    double *qr_res = nullptr;      // [n_cells]
    int32_t *qr_iters = nullptr;   // [n_cells]
    uint8_t *qr_elig = nullptr;    // [n_cells]
    uint8_t *qr_ok = nullptr;      // [n_cells]

    // the last step's arguments (re-launched by dgp_time_kernels)
    bool has_last = false;
    dgp::DevProblem last_pr{};
    int last_precision = 0, last_rule = 0;
    void *last_vals = nullptr, *last_rhs = nullptr;

    // register-budget variant of the 2D row kernel per [precision][degree] (dgp_autotune)
    // 2D launch configuration per [FP64, FP32][degree]: bit 0 = the row kernel's
    // register budget (one more wave per SIMD), bit 1 = rows in rows_sub order;
    // until dgp_autotune or dgp_set_launch, 2 (the default budget, rows_sub
    // order: the faster order on every workload measured)
    int8_t row_cfg[2][dgp::kMaxP + 1] = {{2, 2, 2, 2, 2}, {2, 2, 2, 2, 2}};
    static_assert(dgp::kMaxP == 4, "one initial entry per degree");
    // mixed-degree 2D meshes: one persistent launch over every degree bin (1) or
    // one launch per degree (0), per [FP64, FP32]
    int8_t fused[2] = {0, 0};

    // Approach-1 workspace (COO records, sort buffers), allocated on first use
    void *a1_buf = nullptr;
    size_t a1_bytes = 0;

    bool timing = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool ev_pattern = false, ev_assemble = false;
};

dgp_status dgp_fail(dgp_ctx *ctx, dgp_status st, const char *fmt, ...);
void dgp_free_qrule(dgp_ctx *c);
void dgp_free_approach1(dgp_ctx *c);

#define HIPCHK(ctx, call)                                                                                    \
    do {                                                                                                     \
        hipError_t e_ = (call);                                                                              \
        if (e_ != hipSuccess) return dgp_fail(ctx, DGP_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)
