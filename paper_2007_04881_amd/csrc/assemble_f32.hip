// The FP32 row kernels of rows of degree p <= 2 with the plain rules (the
// device code is in row_f32.h): meshes of one degree, and (MX) the p <= 2 rows
// of mixed-degree meshes.
#include "kernels.h"
#include "row_f32.h"

namespace dgp {

namespace {

template <int P, bool ADV, int ALT, bool MX>
__global__ void __launch_bounds__(256, 3 + ALT) k_row2d_f32(AsmArgs A) {
    using C = F32Cfg<P, MX>;
    __shared__ float xlds[4 * C::LW];
    // the row index is uniform across the wave: keep it (and what derives from it) in scalar registers
    const int wid = xcd_block(blockIdx.x, gridDim.x) * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (wid >= A.n_rows) return;
    const int c = A.rows ? __builtin_amdgcn_readfirstlane(A.rows[wid]) : wid;
    row_f32<P, ADV, MX>(A, c, xlds + (threadIdx.x >> 6) * C::LW);
}

template <int P, bool MX>
const void *kernel_of(bool adv, int alt) {
    return adv ? (alt ? (const void *)k_row2d_f32<P, true, 1, MX> : (const void *)k_row2d_f32<P, true, 0, MX>)
               : (alt ? (const void *)k_row2d_f32<P, false, 1, MX> : (const void *)k_row2d_f32<P, false, 0, MX>);
}

template <int P, bool MX>
void launch_p(const AsmArgs &a, int alt, hipStream_t st) {
    const bool adv = a.pr.bx != 0.0 || a.pr.by != 0.0 || a.pr.c != 0.0;
    const int nb = (a.n_rows + 3) / 4;
    if (nb <= 0) return;
    if (adv) {
        if (alt)
            hipLaunchKernelGGL((k_row2d_f32<P, true, 1, MX>), dim3(nb), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_row2d_f32<P, true, 0, MX>), dim3(nb), dim3(256), 0, st, a);
    } else {
        if (alt)
            hipLaunchKernelGGL((k_row2d_f32<P, false, 1, MX>), dim3(nb), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_row2d_f32<P, false, 0, MX>), dim3(nb), dim3(256), 0, st, a);
    }
}

template <int P, bool MX>
size_t spill_p(int alt, bool adv) {
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, kernel_of<P, MX>(adv, alt)) != hipSuccess) return 0;
    return fa.localSizeBytes;
}

}  // namespace

bool row2d_f32_applies(const AsmArgs &a, int precision, int p) {
    return precision == 1 && !a.reduced && a.pr.u_kind == 0 && (p == 1 || p == 2);
}

void launch_row2d_f32(const AsmArgs &a, int p, bool mixed, int alt, hipStream_t st) {
    if (mixed) {
        if (p == 1)
            launch_p<1, true>(a, alt, st);
        else
            launch_p<2, true>(a, alt, st);
    } else {
        if (p == 1)
            launch_p<1, false>(a, alt, st);
        else
            launch_p<2, false>(a, alt, st);
    }
}

size_t row2d_f32_spill_bytes(int p, bool mixed, int alt, bool adv) {
    if (mixed) return p == 1 ? spill_p<1, true>(alt, adv) : spill_p<2, true>(alt, adv);
    return p == 1 ? spill_p<1, false>(alt, adv) : spill_p<2, false>(alt, adv);
}

}  // namespace dgp
