// The part of a 2D element row that every row kernel shares: where the row's
// blocks go, its row of the block pattern (Section 3.4, Approach 2: one block
// per distinct neighbour, columns ascending), and its loop edges spread over
// the wave's lanes with the neighbour / boundary groups the face terms use.
#pragma once

#include "dgp_common.h"
#include "wave.h"

namespace dgp {
namespace {

struct RowHead {
    int64_t pre_b, pre_v, pre_d;  // the row's first block, value and degree of freedom
    int drank, dvoff;             // rank and value offset of the diagonal block
    int nv;                       // loop vertices (= edges)
    int64_t s0;                   // the row's first loop entry (cell_ptr)
    // lane k < nv: loop edge k (from vertex k to vertex k + 1)
    double ex, ey;  // its start vertex
    int vid, o, rank, voff, dupc;
    bool first;     // first edge towards its neighbour
    // groups: one per neighbour (led by its first edge) and one per boundary edge
    uint64_t gmask;
    int ng;
    int maxdup;  // most edges shared with one neighbour (at least 1)
    int gtab;    // lane g < ng: loop index of the g-th group's leading edge
};

// Offsets of element row c (scanned tile sums, or the sums of the tiles before
// its own when no scan ran, plus the element's prefix inside its tile), its loop
// edges, and, if requested, its row of the pattern.  NB: the row's block size.
// Returns false if only the pattern was asked for.
__device__ __forceinline__ bool row_head(const AsmArgs &A, const int c, const int NB, RowHead &h) {
    const DevMesh &m = A.m;
    const int lane = threadIdx.x & 63;
    const int64_t s = m.cell_ptr[c];
    const int nv = (int)(m.cell_ptr[c + 1] - s);
    h.s0 = s;
    h.nv = nv;
    const int t0 = c / kPrepTile;
    const int4 cr = reinterpret_cast<const int4 *>(A.cnt)[c];
    int64_t tb, tv, td;  // the tile's offsets
    if (A.tile_sum) {
        // no scan kernel ran: sum the sums of the tiles before this one (at most
        // kInlineTiles of them; with at most 24 edges per polygon every prefix
        // stays far below 2^31)
        int sb = 0, sv = 0, sd = 0;
        for (int t = lane; t < t0; t += 64) {
            const int4 v = A.tile_sum[t];
            sb += v.x;
            sv += v.y;
            sd += v.z;
        }
        tb = __builtin_amdgcn_readfirstlane(wave_sum_i(sb));
        tv = __builtin_amdgcn_readfirstlane(wave_sum_i(sv));
        td = __builtin_amdgcn_readfirstlane(wave_sum_i(sd));
    } else {
        tb = A.tile_off[3 * t0];
        tv = A.tile_off[3 * t0 + 1];
        td = A.tile_off[3 * t0 + 2];
    }
    h.pre_b = tb + cr.x;
    h.pre_v = tv + cr.y;
    h.pre_d = td + cr.z;
    h.drank = cr.w & 255;
    h.dvoff = cr.w >> 8;

    h.vid = 0;
    h.o = -3;
    h.rank = 0;
    h.voff = 0;
    h.dupc = 0;
    h.first = false;
    h.ex = 0.0;
    h.ey = 0.0;
    if (lane < nv) {
        const EdgeRec er = A.erec[s + lane];
        h.ex = er.x;
        h.ey = er.y;
        h.vid = er.vid;
        h.o = er.o;
        h.first = (er.rank & kEdgeFirst) != 0;
        h.rank = er.rank & 255;
        h.dupc = (er.rank >> kEdgeDupShift) & 255;
        h.voff = er.voff;
    }
    const uint64_t fm = __ballot(h.first);
    if (A.write_pattern) {
        if (h.first) {
            A.col_idx[h.pre_b + h.rank] = h.o;
            A.val_ptr[h.pre_b + h.rank] = h.pre_v + h.voff;
        }
        if (lane == 0) {
            A.col_idx[h.pre_b + h.drank] = c;
            A.val_ptr[h.pre_b + h.drank] = h.pre_v + h.dvoff;
            A.row_ptr[c] = h.pre_b;
            A.dof_ptr[c] = h.pre_d;
            if (c == m.n_cells - 1) {
                const int n_tiles = (m.n_cells + kPrepTile - 1) / kPrepTile;
                const int nblk = 1 + __popcll(fm);
                A.row_ptr[c + 1] = h.pre_b + nblk;
                A.dof_ptr[c + 1] = h.pre_d + NB;
                A.val_ptr[h.pre_b + nblk] = A.tile_sum ? tv + A.tile_sum[t0].y : A.tile_off[3 * n_tiles + 1];
            }
        }
    }
    if (!A.values) return false;

    h.gmask = __ballot(h.first || (lane < nv && h.o < 0));
    h.ng = __popcll(h.gmask);
    h.maxdup = max(__builtin_amdgcn_readfirstlane(wave_max_i(h.dupc)), 1);
    {
        // lane g gets the position of the g-th set bit of gmask: a forward
        // permutation sends group leaders to lanes 0 .. ng - 1 in order and the
        // other lanes, in order, to ng .. 63
        const bool lead = (h.gmask >> lane) & 1ull;
        const int gidx = __popcll(h.gmask & ((1ull << lane) - 1ull));
        const int dst = lead ? gidx : h.ng + (lane - gidx);
        h.gtab = __builtin_amdgcn_ds_permute(dst << 2, lane);
    }
    return true;
}

}  // namespace
}  // namespace dgp
