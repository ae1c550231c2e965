// Preparation of polyhedral cells, one wave per cell:
//
// * geometry in FP64: bounding box and h = diam(kappa), the largest distance
//   between two vertices (Section 2.2).  Both are taken over the vertices of
//   the cell's boundary triangles, which include every extreme point of the
//   polyhedron, so they equal the values over all of its vertices.  The
//   distinct vertices are collected in an LDS hash set first, so the
//   distance loop is quadratic in the distinct vertices only;
// * the block row (Section 3.4, Approach 2: one block per element and per
//   distinct neighbour): the cell's faces are grouped by neighbour in
//   ascending order (boundary faces last, one group per boundary code) by
//   repeated wave minima over the neighbour ids, with each group's rank among
//   the row's columns and the offset of its block inside the row;
// * the row's counts (blocks, values, dofs) as prefixes inside the
//   work-group's tile of 4 cells, and the tile sums, which a one-work-group
//   kernel scans.
#include "dgp3d.h"
#include "kernels.h"
#include "wave.h"

namespace dgp {

namespace {

constexpr int WG3 = 256;
constexpr int CPW = WG3 / 64;             // cells per work-group (one tile)
static_assert(CPW == kPrepTile3D, "tile size");
constexpr int HSL = kVtxHash3D / 64;      // hash slots per lane in the compaction
constexpr int OWN = kMaxVtx3D / 64;       // distinct vertices per lane
constexpr int kBoundaryKey = 0x7fffff00;  // group key of boundary faces: this | boundary code

// wavefront reductions of the ROCm device library (declared by HIP's headers
// only under HIP_ENABLE_EXTRA_WARP_SYNC_TYPES for the 64-bit types)
extern "C" __device__ __attribute__((const)) double __ockl_wfred_min_f64(double);
extern "C" __device__ __attribute__((const)) double __ockl_wfred_max_f64(double);

__device__ __forceinline__ int wave_min_i(int v) { return __ockl_wfred_min_i32(v); }
__device__ __forceinline__ double wave_min_d(double v) { return __ockl_wfred_min_f64(v); }
__device__ __forceinline__ double wave_max_d(double v) { return __ockl_wfred_max_f64(v); }
__device__ __forceinline__ double readlane_dbl(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

}  // namespace

__global__ void __launch_bounds__(WG3) k_prep3d(DevMesh m, DevProblem pr, Prep3Out out) {
    // per wave: the hash set of distinct vertices, then (reused) the face keys;
    // the compacted vertex list, then (reused) the face ids with the neighbour sizes
    __shared__ int s_a[CPW][kVtxHash3D];
    __shared__ int s_b[CPW][kVtxHash3D];
    __shared__ int s_cnt[CPW][3];

    const int lane = threadIdx.x & 63;
    // the cell, its face count and its distinct-vertex count are wave-uniform:
    // keep them in scalar registers so loops over them are uniform
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int c = blockIdx.x * CPW + w;
    const bool valid = c < m.n_cells;
    int64_t fs = 0;
    int nf = 0, p = 1;
    if (valid) {
        fs = m.cell_face_ptr[c];
        nf = (int)(m.cell_face_ptr[c + 1] - fs);
        p = m.cell_p[c];
    }
    int err = 0;
    if (nf > kMaxFaces3D) {
        err = 1;
        nf = 0;
    }
    int *hash = s_a[w], *list = s_b[w];
    for (int k = lane; k < kVtxHash3D; k += 64) hash[k] = -1;
    __syncthreads();

    // ---- the vertices of the cell's faces into the hash set
    for (int k = lane; k < nf; k += 64) {
        const int F = m.cell_face[fs + k];
        for (int t = 0; t < 3; ++t) {
            const int v = m.face_vtx[3 * F + t];
            int slot = (int)(((unsigned)v * 2654435761u) >> 22) & (kVtxHash3D - 1);
            bool placed = false;
            for (int probe = 0; probe < kVtxHash3D; ++probe) {
                const int old = atomicCAS(&hash[slot], -1, v);
                if (old == -1 || old == v) {
                    placed = true;
                    break;
                }
                slot = (slot + 1) & (kVtxHash3D - 1);
            }
            if (!placed) err = 2;
        }
    }
    __syncthreads();

    // ---- compact the distinct vertices into list[0 .. nu)
    int nmine = 0;
    for (int k = 0; k < HSL; ++k) nmine += hash[lane * HSL + k] >= 0;
    int incl = nmine;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(incl, off, 64);
        if (lane >= off) incl += t;
    }
    const int nu = __builtin_amdgcn_readfirstlane(__shfl(incl, 63, 64));
    int pos = incl - nmine;
    for (int k = 0; k < HSL; ++k) {
        const int v = hash[lane * HSL + k];
        if (v >= 0) list[pos++] = v;
    }
    if (nu > 64 * OWN) err = 3;
    __syncthreads();

    // ---- bounding box and diameter over the distinct vertices (FP64).  Lanes
    // hold vertices lane, lane + 64, ...; empty slots repeat vertex 0, which
    // changes neither the box nor the largest distance.
    const int nk = min((nu + 63) / 64, OWN);  // uniform
    double ox[OWN], oy[OWN], oz[OWN];
    double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
    {
        const int v0 = nu > 0 ? list[0] : 0;
#pragma unroll
        for (int k = 0; k < OWN; ++k) {
            ox[k] = oy[k] = oz[k] = 0.0;
            if (k < nk) {
                const int i = lane + 64 * k;
                const int v = i < nu ? list[i] : v0;
                ox[k] = m.x[v];
                oy[k] = m.y[v];
                oz[k] = m.z[v];
                lo[0] = fmin(lo[0], ox[k]);
                lo[1] = fmin(lo[1], oy[k]);
                lo[2] = fmin(lo[2], oz[k]);
                hi[0] = fmax(hi[0], ox[k]);
                hi[1] = fmax(hi[1], oy[k]);
                hi[2] = fmax(hi[2], oz[k]);
            }
        }
    }
    for (int d = 0; d < 3; ++d) {
        lo[d] = wave_min_d(lo[d]);
        hi[d] = wave_max_d(hi[d]);
    }
    // Diameter.  With c the box centre and R the largest |v - c|, a pair can
    // only be longer than a known pair (length L) if both ends satisfy
    // |v - c| >= L - R (|v_i - v_j| <= |v_i - c| + |v_j - c|).  L starts as the
    // distance from the vertex farthest from c to the vertex farthest from it;
    // only the vertices passing the test are then compared with all others, so
    // the longest pair, whose ends both pass, is among the compared ones.
    const double cc[3] = {0.5 * (lo[0] + hi[0]), 0.5 * (lo[1] + hi[1]), 0.5 * (lo[2] + hi[2])};
    double r2[OWN];
    double r2max = 0.0;
#pragma unroll
    for (int k = 0; k < OWN; ++k) {
        r2[k] = 0.0;
        if (k < nk) {
            const double dx = ox[k] - cc[0], dy = oy[k] - cc[1], dz = oz[k] - cc[2];
            r2[k] = dx * dx + dy * dy + dz * dz;
            r2max = fmax(r2max, r2[k]);
        }
    }
    r2max = wave_max_d(r2max);
    double ax = 0.0, ay = 0.0, az = 0.0;
#pragma unroll
    for (int k = OWN - 1; k >= 0; --k) {
        if (k < nk) {
            const uint64_t hit = __ballot(r2[k] == r2max);
            if (hit) {
                const int l = __builtin_ctzll(hit);
                ax = readlane_dbl(ox[k], l);
                ay = readlane_dbl(oy[k], l);
                az = readlane_dbl(oz[k], l);
            }
        }
    }
    double d2 = 0.0;
#pragma unroll
    for (int k = 0; k < OWN; ++k) {
        if (k < nk) {
            const double dx = ox[k] - ax, dy = oy[k] - ay, dz = oz[k] - az;
            d2 = fmax(d2, dx * dx + dy * dy + dz * dz);
        }
    }
    d2 = wave_max_d(d2);
    // candidates: |v - c| >= L - R, with a relative margin for rounding
    const double thr = sqrt(d2) - sqrt(r2max);
    const double thr2 = thr > 0.0 ? thr * thr * (1.0 - 1e-9) : 0.0;
    double d2c = d2;
#pragma unroll
    for (int k2 = 0; k2 < OWN; ++k2) {
        if (k2 < nk) {
            uint64_t cand = __ballot(r2[k2] >= thr2);
            while (cand) {
                const int l = __builtin_ctzll(cand);
                cand &= cand - 1;
                const double xj = readlane_dbl(ox[k2], l), yj = readlane_dbl(oy[k2], l), zj = readlane_dbl(oz[k2], l);
#pragma unroll
                for (int k = 0; k < OWN; ++k) {
                    if (k < nk) {
                        const double dx = ox[k] - xj, dy = oy[k] - yj, dz = oz[k] - zj;
                        d2c = fmax(d2c, dx * dx + dy * dy + dz * dz);
                    }
                }
            }
        }
    }
    d2 = wave_max_d(d2c);
    err = wave_max_i(err);
    __syncthreads();  // the hash set and the vertex list are free from here on

    // ---- face groups: neighbours ascending, then boundary codes.  Keys in
    // hash[], face ids with the neighbour's basis size (bits 27..30) in list[].
    int *key = hash, *fid = list;
    for (int k = lane; k < nf; k += 64) {
        const int F = m.cell_face[fs + k];
        const int o = other_cell(m, F, c);
        key[k] = o >= 0 ? o : (kBoundaryKey | (int)m.face_bc[F]);
        fid[k] = F | ((o >= 0 ? nb3d(m.cell_p[o]) : 0) << 27);
    }
    wave_sync();
    const int nbc = nb3d(p);
    int prev = -1, start = 0, ng = 0, nbrs = 0, vsum = 0, below = 0, vbelow = 0;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    while (true) {
        int kmin = INT_MAX;
        for (int k = lane; k < nf; k += 64) {
            const int kk = key[k];
            if (kk > prev && kk < kmin) kmin = kk;
        }
        kmin = wave_min_i(kmin);
        if (kmin == INT_MAX) break;
        int cg = 0, nbo = 0;
        for (int k0 = 0; k0 < nf; k0 += 64) {
            const int k = k0 + lane;
            const bool hit = k < nf && key[k] == kmin;
            const uint64_t bal = __ballot(hit);
            if (hit) {
                const int f = fid[k];
                out.forder[fs + start + cg + __popcll(bal & lt)] = f & 0x07ffffff;
                nbo = f >> 27;
            }
            cg += __popcll(bal);
        }
        FaceGroup g;
        g.start = start;
        g.count = cg;
        if (kmin < kBoundaryKey) {
            const int o = kmin;
            nbo = wave_max_i(nbo);
            const int rank = nbrs + (o > c ? 1 : 0);
            const int voff = nbc * vsum + (o > c ? nbc * nbc : 0);
            g.code = o;
            g.rank_voff = rank | (voff << 8);
            nbrs += 1;
            vsum += nbo;
            if (o < c) {
                below += 1;
                vbelow += nbo;
            }
        } else {
            g.code = -(kmin & 0xff);
            g.rank_voff = 0;
        }
        if (lane == 0) out.grp[fs + ng] = g;
        ng += 1;
        if (ng > kMaxGroups3D) err = 4;
        start += cg;
        prev = kmin;
    }

    if (valid && lane == 0) {
        CellGeo3 g;
        double box = 1.0;
        for (int d = 0; d < 3; ++d) {
            g.lo[d] = lo[d];
            g.hi[d] = hi[d];
            box *= hi[d] - lo[d];
            g.s[d] = 0.0;
            g.c[d] = 1.0;
            if (needs_trig(pr)) sincospi(0.5 * (lo[d] + hi[d]), &g.s[d], &g.c[d]);
        }
        g.h = sqrt(d2);
        g.abar = pr.a0;
        g.sqrt_box = sqrt(box);
        g.vol = 0.0;
        g.n_groups = ng;
        g.pad[0] = g.pad[1] = g.pad[2] = 0;
        out.geo[c] = g;
        if (err) atomicOr(out.err, err);  // 1 faces, 2 or 3 distinct vertices, 4 face groups
    }
    // the row's counts; prefixes inside the work-group's tile of CPW cells
    if (lane == 0) {
        s_cnt[w][0] = valid ? 1 + nbrs : 0;
        s_cnt[w][1] = valid ? nbc * (nbc + vsum) : 0;
        s_cnt[w][2] = valid ? nbc : 0;
    }
    __syncthreads();
    if (valid && lane == 0) {
        int pb = 0, pv = 0, pd = 0;
        for (int k = 0; k < w; ++k) {
            pb += s_cnt[k][0];
            pv += s_cnt[k][1];
            pd += s_cnt[k][2];
        }
        out.cnt[4 * c + 0] = pb;
        out.cnt[4 * c + 1] = pv;
        out.cnt[4 * c + 2] = pd;
        out.cnt[4 * c + 3] = below | ((nbc * vbelow) << 8);
    }
    if (threadIdx.x < 3) {
        int64_t sum = 0;
        for (int k = 0; k < CPW; ++k) sum += s_cnt[k][threadIdx.x];
        out.tile_sum[3 * blockIdx.x + threadIdx.x] = sum;
    }
}

// Exclusive scan of the tile sums (blocks, values, dofs) into tile_off, totals
// after the last tile.  One work-group; each thread sums a run of tiles.
__global__ void __launch_bounds__(1024) k_scan3d(int n_tiles, const int64_t *__restrict__ tile_sum,
                                                 int64_t *__restrict__ tile_off) {
    __shared__ int64_t sh[3][1024];
    const int t = threadIdx.x;
    const int per = (n_tiles + 1023) / 1024;
    const int a = t * per, b = min(a + per, n_tiles);
    // the run's first KC tile sums are loaded together and kept for the
    // write-back; longer runs read the rest twice
    constexpr int KC = 8;
    int64_t keep[KC][3];
#pragma unroll
    for (int k = 0; k < KC; ++k)
#pragma unroll
        for (int q = 0; q < 3; ++q) keep[k][q] = a + k < b ? tile_sum[3 * (a + k) + q] : 0;
    int64_t run[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < KC; ++k)
#pragma unroll
        for (int q = 0; q < 3; ++q) run[q] += keep[k][q];
    for (int i = a + KC; i < b; ++i)
        for (int q = 0; q < 3; ++q) run[q] += tile_sum[3 * i + q];
    for (int q = 0; q < 3; ++q) sh[q][t] = run[q];
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v[3] = {0, 0, 0};
        if (t >= off)
            for (int q = 0; q < 3; ++q) v[q] = sh[q][t - off];
        __syncthreads();
        for (int q = 0; q < 3; ++q) sh[q][t] += v[q];
        __syncthreads();
    }
    int64_t acc[3];
    for (int q = 0; q < 3; ++q) acc[q] = sh[q][t] - run[q];
#pragma unroll
    for (int k = 0; k < KC; ++k)
        if (a + k < b)
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                tile_off[3 * (a + k) + q] = acc[q];
                acc[q] += keep[k][q];
            }
    for (int i = a + KC; i < b; ++i)
        for (int q = 0; q < 3; ++q) {
            tile_off[3 * i + q] = acc[q];
            acc[q] += tile_sum[3 * i + q];
        }
    if (t == 1023)
        for (int q = 0; q < 3; ++q) tile_off[3 * n_tiles + q] = sh[q][1023];
}

void launch_prep3d(const DevMesh &m, const DevProblem &pr, const Prep3Out &out, hipStream_t st) {
    const int n_tiles = (m.n_cells + kPrepTile3D - 1) / kPrepTile3D;
    hipLaunchKernelGGL(k_prep3d, dim3(n_tiles), dim3(WG3), 0, st, m, pr, out);
    hipLaunchKernelGGL(k_scan3d, dim3(1), dim3(1024), 0, st, n_tiles, out.tile_sum, out.tile_off);
}

}  // namespace dgp
