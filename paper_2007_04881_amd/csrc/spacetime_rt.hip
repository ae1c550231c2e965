// Host entry of the space-time slab assembly (Section 2.3): checks, the
// preparation kernel (spatial geometry and neighbour ranks), the prism kernel.
#include <hip/hip_runtime.h>

#include "ctx.h"
#include "kernels.h"
#include "spacetime.h"

using namespace dgp;

extern "C" dgp_status dgp_assemble_st(dgp_ctx *ctx, const dgp_problem *prob, int precision, const dgp_slab *slab,
                                      void *vals, void *rhs) {
    if (!ctx || !prob || !slab || !vals || !rhs) return dgp_fail(ctx, DGP_EINVAL, "null argument");
    if (!ctx->has_pattern) return dgp_fail(ctx, DGP_ESTATE, "dgp_assemble_st before dgp_pattern");
    if (precision != DGP_F64 && precision != DGP_F32) return dgp_fail(ctx, DGP_EINVAL, "precision %d", precision);
    if (prob->u_kind != DGP_U_SIN && prob->u_kind != DGP_U_POLY) return dgp_fail(ctx, DGP_EINVAL, "u_kind");
    if (!(prob->c_sigma >= 0.0)) return dgp_fail(ctx, DGP_EINVAL, "c_sigma must be >= 0");
    if (!(slab->t1 > slab->t0)) return dgp_fail(ctx, DGP_EINVAL, "empty slab (t1 <= t0)");
    if (slab->prev && !(slab->t0 > slab->tp0)) return dgp_fail(ctx, DGP_EINVAL, "previous slab: tp0 >= t0");
    if (prob->penalty != DGP_PEN_DIAMETER)
        return dgp_fail(ctx, DGP_EUNSUPPORTED, "space-time slabs take the diameter penalty");
    if (ctx->dim != 2 || ctx->p_uniform < 1 || ctx->p_uniform > 3)
        return dgp_fail(ctx, DGP_EUNSUPPORTED, "space-time slabs are built for 2D meshes of one degree 1..3");
    const int p = ctx->p_uniform;
    const int ngt = (p + 1 > 3 ? p + 1 : 3) * (p + 1);  // face points per edge
    if (ctx->max_dup2d * ngt > st_points_per_pass(precision, p))
        return dgp_fail(ctx, DGP_EUNSUPPORTED, "a cell shares %d edges with one neighbour (at most %d here)",
                        ctx->max_dup2d, st_points_per_pass(precision, p) / ngt);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    DevProblem dp{};
    dp.a0 = prob->a0;
    dp.a1 = prob->a1;
    dp.bx = prob->b[0];
    dp.by = prob->b[1];
    dp.bz = prob->b[2];
    dp.c = prob->c;
    dp.c_sigma = prob->c_sigma;
    dp.u_kind = prob->u_kind;
    for (int i = 0; i < 10; ++i) dp.u[i] = prob->u_poly[i];
    dp.penalty = prob->penalty;
    // spatial geometry, edge records with the neighbours' block ranks, diagonal ranks
    launch_prep(ctx->dm, dp, ctx->prep, ctx->stream, false, ctx->p_uniform);
    StArgs a;
    a.m = ctx->dm;
    a.pr = dp;
    a.slab.t0 = slab->t0;
    a.slab.t1 = slab->t1;
    a.slab.tp0 = slab->tp0;
    a.slab.tau1 = slab->tau1;
    a.slab.tau2 = slab->tau2;
    a.geo = ctx->prep.geo;
    a.erec = ctx->prep.erec;
    a.cnt = ctx->prep.cnt;
    a.row_ptr = ctx->row_ptr;
    a.prev = slab->prev;
    a.vals = vals;
    a.rhs = rhs;
    if (!launch_spacetime(a, precision, p, ctx->stream))
        return dgp_fail(ctx, DGP_EUNSUPPORTED, "no space-time kernel for p = %d", p);
    HIPCHK(ctx, hipGetLastError());
    return DGP_OK;
}
