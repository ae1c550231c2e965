// Block sparsity pattern (Section 3.4, Approach 2): block row r holds the
// sorted unique set {r} U {elements sharing at least one face with r}, so the
// faces of one interface (possibly many) map to a single block.
//
// Three kernels, all integer and deterministic:
//   k_row_count    per cell: blocks, values and dofs of its row; per-tile sums
//   k_tile_scan    one work-group: exclusive scan of the tile sums (+ totals)
//   k_pattern_fill per cell: in-tile scan + tile offset -> row_ptr, dof_ptr,
//                  sorted col_idx and val_ptr of the row
#include "dgp_common.h"
#include "kernels.h"

namespace dgp {

struct RowCount {
    int64_t blocks, vals, dofs;
};

// Count the row of cell c: neighbours are the other cells of its faces,
// duplicates (several faces to one neighbour) counted once.
__device__ __forceinline__ RowCount row_count(const DevMesh &m, int c) {
    RowCount rc;
    int nb = nb2d(m.cell_p[c]);
    int64_t s = m.cell_face_ptr[c], e = m.cell_face_ptr[c + 1];
    rc.blocks = 1;
    rc.vals = (int64_t)nb * nb;
    rc.dofs = nb;
    for (int64_t k = s; k < e; ++k) {
        int o = other_cell(m, m.cell_face[k], c);
        if (o < 0 || o == c) continue;
        bool dup = false;
        for (int64_t j = s; j < k; ++j)
            if (other_cell(m, m.cell_face[j], c) == o) {
                dup = true;
                break;
            }
        if (!dup) {
            rc.blocks += 1;
            rc.vals += (int64_t)nb * nb2d(m.cell_p[o]);
        }
    }
    return rc;
}

// Exclusive scan of three int64 values over a 256-thread block (Hillis-Steele in LDS).
__device__ __forceinline__ RowCount block_exclusive_scan(RowCount v, RowCount *total) {
    __shared__ int64_t sh[3][kTile];
    int t = threadIdx.x;
    sh[0][t] = v.blocks;
    sh[1][t] = v.vals;
    sh[2][t] = v.dofs;
    __syncthreads();
    for (int off = 1; off < kTile; off <<= 1) {
        int64_t a = 0, b = 0, c = 0;
        if (t >= off) {
            a = sh[0][t - off];
            b = sh[1][t - off];
            c = sh[2][t - off];
        }
        __syncthreads();
        sh[0][t] += a;
        sh[1][t] += b;
        sh[2][t] += c;
        __syncthreads();
    }
    RowCount ex;
    ex.blocks = sh[0][t] - v.blocks;
    ex.vals = sh[1][t] - v.vals;
    ex.dofs = sh[2][t] - v.dofs;
    total->blocks = sh[0][kTile - 1];
    total->vals = sh[1][kTile - 1];
    total->dofs = sh[2][kTile - 1];
    __syncthreads();
    return ex;
}

__global__ void __launch_bounds__(kTile) k_row_count(DevMesh m, int64_t *tile_sums) {
    int c = blockIdx.x * kTile + threadIdx.x;
    RowCount rc = {0, 0, 0};
    if (c < m.n_cells) rc = row_count(m, c);
    RowCount tot;
    block_exclusive_scan(rc, &tot);
    if (threadIdx.x == 0) {
        tile_sums[3 * blockIdx.x + 0] = tot.blocks;
        tile_sums[3 * blockIdx.x + 1] = tot.vals;
        tile_sums[3 * blockIdx.x + 2] = tot.dofs;
    }
}

// One work-group of 1024 threads scans the tile sums in chunks; writes the
// exclusive offsets in place and the totals to totals[0..2].
__global__ void __launch_bounds__(1024) k_tile_scan(int64_t *tile_sums, int n_tiles, int64_t *totals) {
    __shared__ int64_t sh[3][1024];
    int t = threadIdx.x;
    int64_t carry[3] = {0, 0, 0};
    for (int base = 0; base < n_tiles; base += 1024) {
        int i = base + t;
        int64_t v[3];
        for (int q = 0; q < 3; ++q) {
            v[q] = i < n_tiles ? tile_sums[3 * i + q] : 0;
            sh[q][t] = v[q];
        }
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int64_t a[3] = {0, 0, 0};
            if (t >= off)
                for (int q = 0; q < 3; ++q) a[q] = sh[q][t - off];
            __syncthreads();
            for (int q = 0; q < 3; ++q) sh[q][t] += a[q];
            __syncthreads();
        }
        if (i < n_tiles)
            for (int q = 0; q < 3; ++q) tile_sums[3 * i + q] = carry[q] + sh[q][t] - v[q];
        int64_t last[3] = {sh[0][1023], sh[1][1023], sh[2][1023]};
        __syncthreads();
        for (int q = 0; q < 3; ++q) carry[q] += last[q];
    }
    if (t == 0)
        for (int q = 0; q < 3; ++q) totals[q] = carry[q];
}

__global__ void __launch_bounds__(kTile) k_pattern_fill(DevMesh m, const int64_t *tile_offs, int64_t *row_ptr,
                                                        int32_t *col_idx, int64_t *val_ptr, int64_t *dof_ptr) {
    int c = blockIdx.x * kTile + threadIdx.x;
    RowCount rc = {0, 0, 0};
    if (c < m.n_cells) rc = row_count(m, c);
    RowCount tot;
    RowCount ex = block_exclusive_scan(rc, &tot);
    if (c >= m.n_cells) return;
    int64_t rb = tile_offs[3 * blockIdx.x + 0] + ex.blocks;
    int64_t vb = tile_offs[3 * blockIdx.x + 1] + ex.vals;
    int64_t db = tile_offs[3 * blockIdx.x + 2] + ex.dofs;
    row_ptr[c] = rb;
    dof_ptr[c] = db;
    if (c == m.n_cells - 1) {
        row_ptr[c + 1] = rb + rc.blocks;
        dof_ptr[c + 1] = db + rc.dofs;
        val_ptr[rb + rc.blocks] = vb + rc.vals;
    }
    // emit the columns in ascending order: repeatedly take the smallest id above the last one
    int nb = nb2d(m.cell_p[c]);
    int64_t s = m.cell_face_ptr[c], e = m.cell_face_ptr[c + 1];
    int prev = -1;
    for (int64_t t = 0; t < rc.blocks; ++t) {
        int next = c > prev ? c : 0x7fffffff;
        for (int64_t k = s; k < e; ++k) {
            int o = other_cell(m, m.cell_face[k], c);
            if (o > prev && o < next) next = o;
        }
        col_idx[rb + t] = next;
        val_ptr[rb + t] = vb;
        vb += (int64_t)nb * nb2d(m.cell_p[next]);
        prev = next;
    }
}

void launch_pattern(const DevMesh &m, int64_t *tile_sums, int64_t *totals, int64_t *row_ptr, int32_t *col_idx,
                    int64_t *val_ptr, int64_t *dof_ptr, hipStream_t st) {
    int n_tiles = (m.n_cells + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_row_count, dim3(n_tiles), dim3(kTile), 0, st, m, tile_sums);
    hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, st, tile_sums, n_tiles, totals);
    if (row_ptr)
        hipLaunchKernelGGL(k_pattern_fill, dim3(n_tiles), dim3(kTile), 0, st, m, tile_sums, row_ptr, col_idx,
                           val_ptr, dof_ptr);
}

}  // namespace dgp
