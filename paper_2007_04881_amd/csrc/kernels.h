// Launchers of the dgpoly kernels (host side, called by the runtime).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dgp_common.h"
#include "dgp3d.h"

namespace dgp {

// Geometry, edge neighbours and row sizes, then the scan of the tile sums (two launches).
// scan = false: the tile sums are left for the assembly kernel to sum (see AsmArgs::tile_sum);
// p_uniform > 0: the common degree of all cells (or -1)
void launch_prep(const DevMesh &m, const DevProblem &pr, const PrepOut &out, hipStream_t st, bool scan, int p_uniform);

// One wave per element row: pattern (if a.write_pattern) and values of rows
// a.rows[0 .. n_rows) (all rows in order if a.rows is null), all of degree p;
// mixed: neighbours may have any degree up to kMaxP (else all have degree p).
// alt: 0 = the default register budget, 1 = one more wave per SIMD (see dgp_autotune)
bool launch_row2d(const AsmArgs &a, int precision, int p, bool mixed, int alt, hipStream_t st);
// One persistent launch over the rows a.rows[0 .. n_rows) of every degree (mixed-degree
// meshes), dispatching per row to the same body as launch_row2d(.., mixed = true, ..).
void launch_row2d_fused(const AsmArgs &a, int precision, hipStream_t st);
// per-lane scratch bytes (register spills) of the row kernel instantiation that
// launch_row2d(a, precision, p, mixed, alt, ..) runs
size_t row2d_spill_bytes(const AsmArgs &a, int precision, int p, bool mixed, int alt);
// The FP32 row kernel for rows of degree p <= 2 with the plain rules and the
// sine manufactured solution, on meshes of one degree or (mixed) among
// neighbours of any degree (launch_row2d takes it whenever row2d_f32_applies);
// same outputs within FP32 rounding.
bool row2d_f32_applies(const AsmArgs &a, int precision, int p);
void launch_row2d_f32(const AsmArgs &a, int p, bool mixed, int alt, hipStream_t st);
size_t row2d_f32_spill_bytes(int p, bool mixed, int alt, bool adv);

// ---- polyhedral (3D) meshes
// Geometry, face groups and row counts of every cell, then the tile scan.
void launch_prep3d(const DevMesh &m, const DevProblem &pr, const Prep3Out &out, hipStream_t st);
// One wave per element row of degree p (1 or 2), as launch_row2d.
bool launch_row3d(const Asm3Args &a, int precision, int p, hipStream_t st);

// ---- reduced volume rules
void launch_cell_poly(const DevMesh &m, const CellGeo *geo, float *feat, double *mom, double *parea, uint8_t *eligible,
                      hipStream_t st);
void launch_train_poly(uint64_t seed, int64_t first, int64_t n, float *feat, double *feat64, double *mom,
                       double *parea, hipStream_t st);
void launch_rule_init(int n, const float *z, const double *parea, double *nodes, double *weights, hipStream_t st);
void launch_refine(int n, const double *mom, const double *parea, const uint8_t *eligible, double *nodes,
                   double *weights, uint8_t *accepted, double *residual, int32_t *iters, int max_it, double tol,
                   double mu0, hipStream_t st);

// per element the start (network or template) of smaller initial residual; retry and merge
void launch_rule_pick(int n, const double *res_net, const double *res_tmpl, double *nodes, double *weights,
                      const double *nodes_t, const double *w_t, uint8_t *start_tmpl, hipStream_t st);
void launch_rule_retry_mask(int n, const uint8_t *elig, const uint8_t *acc, const uint8_t *start_tmpl, uint8_t *mask,
                            hipStream_t st);
void launch_rule_merge(int n, const uint8_t *mask, const uint8_t *acc2, const double *res2, const int32_t *it2,
                       const double *nodes2, const double *w2, double *nodes, double *weights, uint8_t *acc,
                       double *res, int32_t *it, hipStream_t st);

// ---- the rule network (FP32 on the matrix cores)
// C = epi(A B): A(m, k) = A[m sam + k sak], B(k, n) = B[k sbk + n sbn], C row-major.
struct GemmArgs {
    const float *A;
    int64_t sam, sak;
    const float *B;
    int64_t sbk, sbn;
    float *C;
    int64_t ldc;
    int M, N, K;
    const float *bias;  // [N] or null
    int act;            // 0 identity, 1 SiLU (pre-activation to Zout if set), 2 times SiLU'(Z)
    const float *Z;     // act 2: pre-activation, leading dimension ldc
    float *Zout;
    float *work;        // split-K partial sums, at least ksplit * M * N floats (ksplit > 1)
    int ksplit;         // K ranges summed separately, then added in a fixed order
};
void launch_gemm(const GemmArgs &g, hipStream_t st);
// forward pass of the network over n rows of x [n][36]; h1, h2 [n][128] scratch; out [n][48]
void mlp_forward(const float *params, const float *x, int64_t n, float *h1, float *h2, float *out, hipStream_t st);
// loss and gradient with respect to the 48 outputs: mean over the n rows of sum_ab (Q_ab - M_ab)^2 / |P|^2
void launch_loss_grad(const float *out, const double *mom, const double *parea, int64_t n, int64_t n_mean, float *dout,
                      float *loss_rows, hipStream_t st);
// column sums of a [rows][cols] matrix into dst (deterministic)
void launch_colsum(const float *a, int64_t rows, int cols, float *dst, hipStream_t st);
void launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t st);

}  // namespace dgp
