// Launchers of the dgpoly kernels (host side, called by the runtime).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dgp_common.h"

namespace dgp {

// Geometry (always) and, with do_pattern, the block pattern, in one kernel.
int prep_tiles(int n_cells);
void launch_prep(const DevMesh &m, const DevProblem &pr, CellGeo *geo, bool do_pattern, const Lookback &lb,
                 int64_t *row_ptr, int32_t *col_idx, int64_t *val_ptr, int64_t *dof_ptr, hipStream_t st);

// Capacities of one assembly work-group for (precision, p): the runtime cuts
// the element rows into chunks of consecutive rows that respect them.
struct AsmLimits {
    int slots;               // quadrature tasks
    int fslots;              // face tasks
    int maxc;                // elements
    int maxb;                // blocks
    int tasks_per_triangle;  // element-term tasks per fan sub-triangle
};
void assemble_limits(int precision, int p, AsmLimits *lim);

// Assembly of every block row; p is the common degree of all cells; chunks
// holds n_chunks + 1 element offsets.  Returns false if no kernel is built
// for (precision, p).
bool launch_assemble2d(const DevMesh &m, const DevProblem &pr, const CellGeo *geo, const int64_t *row_ptr,
                       const int32_t *col_idx, const int64_t *val_ptr, const int64_t *dof_ptr, const int32_t *chunks,
                       int n_chunks, int precision, int p, void *vals, void *rhs, hipStream_t st);

}  // namespace dgp
