// Space-time slabs over 2D meshes: arguments and launcher.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dgp_common.h"

namespace dgp {

struct StSlab {
    double t0, t1;      // the slab I_n = (t0, t1]
    double tp0;         // the previous slab's start (its box in time is [tp0, t0])
    double tau1, tau2;  // manufactured u = u_s(x, y) (1 + tau1 t + tau2 t^2)
};

struct StArgs {
    DevMesh m;
    DevProblem pr;
    StSlab slab;
    const CellGeo *geo;    // preparation kernel (spatial boxes, diameters, abar)
    const EdgeRec *erec;   // loop edges with neighbour block ranks
    const int32_t *cnt;    // diagonal rank per row (bits 0-7 of cnt[4 c + 3])
    const int64_t *row_ptr;  // the pattern's row offsets (blocks; uniform degree)
    const double *prev;    // previous slab's coefficients [n_cells][n_b] or null (exact u(t0))
    void *vals, *rhs;      // [nnzb][n_b^2], [n_cells][n_b]
};

// One wave per prism row (uniform degree p = 1..3); false for other p.
bool launch_spacetime(const StArgs &a, int precision, int p, hipStream_t st);
// points per pass of the kernel for this precision and degree (a neighbour's
// face points must fit in one pass)
int st_points_per_pass(int precision, int p);

}  // namespace dgp
