// Host runtime of the Approach-1 ablation (COO records, radix sort,
// segmented reduction; Section 3.3): its workspace and entry point.
#include <hip/hip_runtime.h>

#include <cstring>

#include "approach1.h"
#include "ctx.h"
#include "kernels.h"

using namespace dgp;

void dgp_free_approach1(dgp_ctx *c) {
    if (c->a1_buf) (void)hipFree(c->a1_buf);
    c->a1_buf = nullptr;
    c->a1_bytes = 0;
}

extern "C" dgp_status dgp_assemble_coo(dgp_ctx *ctx, const dgp_problem *prob, int precision, void *vals, void *rhs,
                                       int64_t *row_ptr, int32_t *col_idx, int64_t *val_ptr, int64_t *dof_ptr) {
    if (!ctx || !prob || !vals || !rhs || !row_ptr || !col_idx || !val_ptr || !dof_ptr)
        return dgp_fail(ctx, DGP_EINVAL, "null argument");
    if (!ctx->has_pattern) return dgp_fail(ctx, DGP_ESTATE, "dgp_assemble_coo before dgp_pattern (output sizes)");
    if (precision != DGP_F64 && precision != DGP_F32) return dgp_fail(ctx, DGP_EINVAL, "precision %d", precision);
    if (prob->u_kind != DGP_U_SIN && prob->u_kind != DGP_U_POLY) return dgp_fail(ctx, DGP_EINVAL, "u_kind");
    if (!(prob->c_sigma >= 0.0)) return dgp_fail(ctx, DGP_EINVAL, "c_sigma must be >= 0");
    if (prob->penalty != DGP_PEN_DIAMETER && prob->penalty != DGP_PEN_COVERING)
        return dgp_fail(ctx, DGP_EINVAL, "penalty %d", prob->penalty);
    if (ctx->dim != 2 || ctx->p_uniform <= 0)
        return dgp_fail(ctx, DGP_EUNSUPPORTED, "Approach 1 is built for 2D meshes of one degree");
    const int p = ctx->p_uniform;
    const int64_t N = ctx->n_cells, F = ctx->n_faces;
    const int64_t R = N + 4 * F;
    if (R > INT32_MAX / 2) return dgp_fail(ctx, DGP_EUNSUPPORTED, "too many records");
    const int tiles = (int)((R + 2047) / 2048);
    // workspace: record values (sized for FP64), keys x 3, record numbers x 3,
    // digit histograms, heads, unique numbers, segment starts, two counters
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t S = approach1_record_values(p);
    const size_t o_vals = 0;
    const size_t o_keys = o_vals + al(sizeof(double) * S * (size_t)R);
    const size_t o_perm = o_keys + 3 * al(sizeof(uint64_t) * (size_t)R);
    const size_t o_hist = o_perm + 3 * al(sizeof(int32_t) * (size_t)R);
    const size_t o_heads = o_hist + al(sizeof(int32_t) * 256 * (size_t)tiles);
    const size_t o_uidx = o_heads + al(sizeof(int32_t) * (size_t)R);
    const size_t o_seg = o_uidx + al(sizeof(int32_t) * (size_t)R);
    const size_t o_cnt = o_seg + al(sizeof(int32_t) * (size_t)(R + 1));
    const size_t bytes = o_cnt + 256;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if (ctx->a1_bytes < bytes) {
        dgp_free_approach1(ctx);
        if (hipMalloc(&ctx->a1_buf, bytes) != hipSuccess) return dgp_fail(ctx, DGP_ENOMEM, "Approach-1 workspace");
        ctx->a1_bytes = bytes;
    }
    char *b = static_cast<char *>(ctx->a1_buf);
    // records actually used: every element, one per boundary face, four per interior face
    const int32_t n_valid = (int32_t)(N + ctx->n_boundary_faces + 4 * (F - ctx->n_boundary_faces));
    HIPCHK(ctx, hipMemcpyAsync(b + o_cnt + 4, &n_valid, sizeof(n_valid), hipMemcpyHostToDevice, ctx->stream));

    A1Args a;
    a.m = ctx->dm;
    dgp_problem pc = *prob;
    DevProblem dp{};
    dp.a0 = pc.a0;
    dp.a1 = pc.a1;
    dp.bx = pc.b[0];
    dp.by = pc.b[1];
    dp.bz = pc.b[2];
    dp.c = pc.c;
    dp.c_sigma = pc.c_sigma;
    dp.u_kind = pc.u_kind;
    for (int i = 0; i < 10; ++i) dp.u[i] = pc.u_poly[i];
    dp.penalty = pc.penalty;
    a.pr = dp;
    a.geo = ctx->prep.geo;
    a.pen_face = ctx->prep.pen_face;
    a.n_records = (int32_t)R;
    a.n_valid_records = reinterpret_cast<const int32_t *>(b + o_cnt + 4);
    a.nnzb_bound = (int32_t)ctx->nnzb;
    a.rec_vals = b + o_vals;
    a.keys = reinterpret_cast<uint64_t *>(b + o_keys);
    a.keys_alt[0] = reinterpret_cast<uint64_t *>(b + o_keys + al(sizeof(uint64_t) * (size_t)R));
    a.keys_alt[1] = reinterpret_cast<uint64_t *>(b + o_keys + 2 * al(sizeof(uint64_t) * (size_t)R));
    for (int k = 0; k < 3; ++k) a.perm[k] = reinterpret_cast<int32_t *>(b + o_perm + k * al(sizeof(int32_t) * (size_t)R));
    a.hist = reinterpret_cast<int32_t *>(b + o_hist);
    a.heads = reinterpret_cast<int32_t *>(b + o_heads);
    a.uidx = reinterpret_cast<int32_t *>(b + o_uidx);
    a.seg = reinterpret_cast<int32_t *>(b + o_seg);
    a.total = reinterpret_cast<int32_t *>(b + o_cnt);
    a.row_ptr = row_ptr;
    a.col_idx = col_idx;
    a.val_ptr = val_ptr;
    a.dof_ptr = dof_ptr;
    a.vals = vals;
    a.rhs = rhs;
    // geometry (boxes, diameters, abar, penalty sides) from the preparation kernel
    launch_prep(ctx->dm, dp, ctx->prep, ctx->stream, false, ctx->p_uniform);
    if (!launch_approach1(a, precision, p, ctx->stream))
        return dgp_fail(ctx, DGP_EUNSUPPORTED, "no Approach-1 kernels for p = %d", p);
    HIPCHK(ctx, hipGetLastError());
    return DGP_OK;
}
