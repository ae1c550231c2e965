// Launchers of the dgpoly kernels (host side, called by the runtime).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dgp_common.h"

namespace dgp {

// Pattern: tile_sums [3 * n_tiles] scratch, totals [3] (blocks, values, dofs).
// With row_ptr == nullptr only the counts and totals are produced.
void launch_pattern(const DevMesh &m, int64_t *tile_sums, int64_t *totals, int64_t *row_ptr, int32_t *col_idx,
                    int64_t *val_ptr, int64_t *dof_ptr, hipStream_t st);

void launch_geometry(const DevMesh &m, const DevProblem &pr, CellGeo *geo, hipStream_t st);

// Assembly of every block row; p_uniform is the common degree of all cells.
// Returns false if no kernel is built for (precision, p).
bool launch_assemble2d(const DevMesh &m, const DevProblem &pr, const CellGeo *geo, const int64_t *row_ptr,
                       const int32_t *col_idx, const int64_t *val_ptr, const int64_t *dof_ptr, int precision,
                       int p_uniform, void *vals, void *rhs, hipStream_t st);

}  // namespace dgp
