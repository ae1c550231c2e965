// Approach 1 (COO records with duplicates, sorted and reduced): arguments and launcher.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dgp_common.h"

namespace dgp {

struct A1Args {
    DevMesh m;
    DevProblem pr;
    const CellGeo *geo;       // from the preparation kernel
    const double *pen_face;   // covering penalty sides (PrepOut::pen_face)
    int32_t n_records;        // n_cells + 4 n_faces
    const int32_t *n_valid_records;  // device: n_cells + boundary faces + 4 interior faces
    int32_t nnzb_bound;       // grid of the reduction (the pattern's block count)
    void *rec_vals;           // [n_records][n_b^2 + n_b]
    uint64_t *keys;           // [n_records] row * n_cells + column (n_cells^2: unused)
    uint64_t *keys_alt[2];    // sort buffers
    int32_t *perm[3];         // record numbers: initial, then the two sort buffers
    int32_t *hist;            // [256 * tiles of 2048 keys]
    int32_t *heads, *uidx, *seg;  // [n_records], [n_records], [n_records + 1]
    int32_t *total;           // device: number of distinct blocks
    int64_t *row_ptr;         // outputs: the pattern (as dgp_pattern's) and the values
    int32_t *col_idx;
    int64_t *val_ptr;
    int64_t *dof_ptr;
    void *vals, *rhs;
};

// Element and face records, the sort and the reduction on stream st (uniform degree p).
bool launch_approach1(const A1Args &a, int precision, int p, hipStream_t st);
// values per record for degree p
size_t approach1_record_values(int p);

}  // namespace dgp
