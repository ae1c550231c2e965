// Element preparation: geometry (FP64) and the block sparsity pattern in one
// pass over the mesh.
//
// Geometry (every precision mode keeps it FP64): bounding box (the basis lives
// on it, Section 3.1), h = diam(kappa) (Section 2.2), |kappa|, and
// abar = max of a over the element's volume quadrature points (the discrete
// ||a||_{L_inf(kappa)} of the penalty, Appendix A).
//
// Pattern (Section 3.4, Approach 2): row r = sorted unique {r} U {elements
// sharing a face with r}; all faces of one interface map to one block.
//
// Eight lanes per element: lane k owns faces k, k+8, k+16 and the fan
// sub-triangles and vertices with the same stride.  Neighbour ranks come from
// comparisons across the group (lane shuffles), not from sorting in memory.
// Row, value and dof offsets use a single-pass scan with decoupled look-back:
// each work-group takes a ticket (its tile), publishes its aggregate, then
// walks back over the tiles before it until it finds an inclusive prefix.
// Tickets are taken in launch order, so every tile waited on belongs to a
// work-group that is already running and publishes without waiting.
#include "dgp_common.h"
#include "kernels.h"
#include "rules_data.h"

namespace dgp {

namespace {

constexpr int G = 8;
constexpr int SLOTS = kMaxFaces2D / G;  // faces per lane
constexpr int WG = 256;
constexpr int CPB = WG / G;             // elements per tile

template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ int gsum_i(int v) {
    v += dpp_i<0xB1>(v);
    v += dpp_i<0x4E>(v);
    v += dpp_i<0x141>(v);
    return v;
}
__device__ __forceinline__ double gsum_d(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    return v;
}
__device__ __forceinline__ double gmax_d(double v) {
    v = fmax(v, dpp_d<0xB1>(v));
    v = fmax(v, dpp_d<0x4E>(v));
    v = fmax(v, dpp_d<0x141>(v));
    return v;
}
__device__ __forceinline__ double gmin_d(double v) {
    v = fmin(v, dpp_d<0xB1>(v));
    v = fmin(v, dpp_d<0x4E>(v));
    v = fmin(v, dpp_d<0x141>(v));
    return v;
}

template <int DEG>
__device__ double max_a_on_triangle(const DevProblem &pr, double x0, double y0, double x1, double y1, double x2,
                                    double y2) {
    const double *L = DEG == 4 ? c_tri4_l : DEG == 6 ? c_tri6_l : c_tri8_l;
    const int n = DEG == 4 ? DGP_TRI4_N : DEG == 6 ? DGP_TRI6_N : DGP_TRI8_N;
    double amax = -1e300;
    for (int q = 0; q < n; ++q) {
        double px = L[3 * q] * x0 + L[3 * q + 1] * x1 + L[3 * q + 2] * x2;
        double py = L[3 * q] * y0 + L[3 * q + 1] * y1 + L[3 * q + 2] * y2;
        amax = fmax(amax, coef_a(pr, px, py));
    }
    return amax;
}

}  // namespace

__global__ void __launch_bounds__(WG)
    k_prep(DevMesh m, DevProblem pr, CellGeo *__restrict__ geo, int do_pattern, int n_tiles, Lookback lb,
           int64_t *__restrict__ row_ptr, int32_t *__restrict__ col_idx, int64_t *__restrict__ val_ptr,
           int64_t *__restrict__ dof_ptr) {
    __shared__ int64_t s_ex[CPB][3];
    __shared__ int64_t s_prefix[3];
    __shared__ unsigned long long s_ticket;

    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    int tile = blockIdx.x;
    unsigned long long epoch = 0;
    if (do_pattern) {
        if (threadIdx.x == 0) s_ticket = atomicAdd(lb.counter, 1ULL);
        __syncthreads();
        tile = (int)(s_ticket % (unsigned long long)n_tiles);
        epoch = s_ticket / (unsigned long long)n_tiles + 1;
    }
    const int c = tile * CPB + grp;
    const bool valid = c < m.n_cells;
    int64_t s = 0;
    int nv = 0, p = 1;
    if (valid) {
        s = m.cell_ptr[c];
        nv = (int)(m.cell_ptr[c + 1] - s);
        p = m.cell_p[c];
    }

    // ------------------------------------------------------------ geometry
    double lox = 1e300, loy = 1e300, hix = -1e300, hiy = -1e300, a2 = 0.0, d2 = 0.0, amax = -1e300;
    for (int i = lane; i < nv; i += G) {
        const int vi = m.cell_vtx[s + i];
        const double xi = m.x[vi], yi = m.y[vi];
        lox = fmin(lox, xi);
        loy = fmin(loy, yi);
        hix = fmax(hix, xi);
        hiy = fmax(hiy, yi);
        const int vn = m.cell_vtx[s + (i + 1 == nv ? 0 : i + 1)];
        a2 += xi * m.y[vn] - m.x[vn] * yi;
        for (int j = i + 1; j < nv; ++j) {
            const int vj = m.cell_vtx[s + j];
            const double dx = xi - m.x[vj], dy = yi - m.y[vj];
            d2 = fmax(d2, dx * dx + dy * dy);
        }
    }
    if (valid && pr.a1 != 0.0) {
        const int v0 = m.cell_vtx[s];
        const double x0 = m.x[v0], y0 = m.y[v0];
        for (int t = lane; t + 2 < nv; t += G) {
            const int v1 = m.cell_vtx[s + t + 1], v2 = m.cell_vtx[s + t + 2];
            const double x1 = m.x[v1], y1 = m.y[v1], x2 = m.x[v2], y2 = m.y[v2];
            double am = p <= 2 ? max_a_on_triangle<4>(pr, x0, y0, x1, y1, x2, y2)
                      : p == 3 ? max_a_on_triangle<6>(pr, x0, y0, x1, y1, x2, y2)
                               : max_a_on_triangle<8>(pr, x0, y0, x1, y1, x2, y2);
            amax = fmax(amax, am);
        }
    }
    lox = gmin_d(lox);
    loy = gmin_d(loy);
    hix = gmax_d(hix);
    hiy = gmax_d(hiy);
    a2 = gsum_d(a2);
    d2 = gmax_d(d2);
    amax = gmax_d(amax);
    if (valid && lane == 0) {
        CellGeo g;
        g.lox = lox;
        g.loy = loy;
        g.hix = hix;
        g.hiy = hiy;
        g.h = sqrt(d2);
        g.abar = pr.a1 != 0.0 ? amax : pr.a0;
        g.sqrt_box = sqrt((hix - lox) * (hiy - loy));
        g.area = 0.5 * a2;
        geo[c] = g;
    }
    if (!do_pattern) return;

    // ------------------------------------------------------------- pattern
    // neighbours of this lane's faces (-1: none or boundary)
    int nb[SLOTS], nbsz[SLOTS];
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
        const int f = lane + G * q;
        nb[q] = -1;
        nbsz[q] = 0;
        if (f < nv) {
            const int o = other_cell(m, m.cell_face[s + f], c);
            if (o >= 0 && o != c) {
                nb[q] = o;
                nbsz[q] = nb2d(m.cell_p[o]);
            }
        }
    }
    // a neighbour counts once: at its first face; rank = unique neighbours below it
    bool first[SLOTS];
    int rank[SLOTS], valoff[SLOTS];
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
        first[q] = nb[q] >= 0;
        rank[q] = c < nb[q] ? 1 : 0;
        valoff[q] = c < nb[q] ? nb2d(p) : 0;
    }
    int self_rank = 0, self_valoff = 0;
    const int base = threadIdx.x & ~(G - 1);
    // pass 1: first occurrence
#pragma unroll
    for (int q2 = 0; q2 < SLOTS; ++q2) {
        for (int l2 = 0; l2 < G; ++l2) {
            const int v = __shfl(nb[q2], base + l2, 64);
            const int j = l2 + G * q2;
#pragma unroll
            for (int q = 0; q < SLOTS; ++q)
                if (v == nb[q] && j < lane + G * q) first[q] = false;
        }
    }
    // pass 2: ranks and value offsets among unique neighbours
#pragma unroll
    for (int q2 = 0; q2 < SLOTS; ++q2) {
        for (int l2 = 0; l2 < G; ++l2) {
            const int v = __shfl(nb[q2], base + l2, 64);
            const int u = __shfl((int)first[q2], base + l2, 64);
            const int sz = __shfl(nbsz[q2], base + l2, 64);
            if (u) {
#pragma unroll
                for (int q = 0; q < SLOTS; ++q)
                    if (v < nb[q]) {
                        rank[q] += 1;
                        valoff[q] += sz;
                    }
                if (v < c) {
                    self_rank += 1;
                    self_valoff += sz;
                }
            }
        }
    }
    int cnt = 0, szsum = 0;
#pragma unroll
    for (int q = 0; q < SLOTS; ++q)
        if (first[q]) {
            cnt += 1;
            szsum += nbsz[q];
        }
    cnt = gsum_i(cnt);
    szsum = gsum_i(szsum);
    const int nbc = nb2d(p);
    const int64_t my_blocks = valid ? 1 + cnt : 0;
    const int64_t my_vals = valid ? (int64_t)nbc * (nbc + szsum) : 0;
    const int64_t my_dofs = valid ? nbc : 0;

    // tile scan over the 32 elements (wave 0, lanes 0..31)
    if (lane == 0) {
        s_ex[grp][0] = my_blocks;
        s_ex[grp][1] = my_vals;
        s_ex[grp][2] = my_dofs;
    }
    __syncthreads();
    if (threadIdx.x < 64) {
        // exclusive scan of the tile's rows (lanes 0..31), aggregate in lane 31
        const int t = threadIdx.x;
        int64_t v[3] = {0, 0, 0};
        if (t < CPB)
            for (int q = 0; q < 3; ++q) v[q] = s_ex[t][q];
        int64_t incl[3] = {v[0], v[1], v[2]};
        for (int off = 1; off < CPB; off <<= 1) {
            for (int q = 0; q < 3; ++q) {
                const int64_t o = __shfl_up(incl[q], off, 64);
                if (t >= off) incl[q] += o;
            }
        }
        int64_t agg[3];
        for (int q = 0; q < 3; ++q) {
            if (t < CPB) s_ex[t][q] = incl[q] - v[q];
            agg[q] = __shfl(incl[q], CPB - 1, 64);
        }
        // publish the aggregate
        if (t == 0) {
            for (int q = 0; q < 3; ++q) lb.agg[3 * tile + q] = agg[q];
            __hip_atomic_store(&lb.status[tile], (epoch << 2) | 1ULL, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        // decoupled look-back over windows of 64 preceding tiles: stop at the
        // nearest tile that has published its inclusive prefix
        int64_t pre[3] = {0, 0, 0};
        int end = tile;
        long spins = 0;
        while (end > 0) {
            const int j = end - 64 + t;
            const unsigned long long st =
                j >= 0 ? __hip_atomic_load(&lb.status[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                       : ((epoch << 2) | 2ULL);
            if (!__all((st >> 2) == epoch)) {
                if (++spins > (1L << 20)) {  // safety net: never expected; flags the result as invalid
                    if (t == 0) lb.error[0] = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const unsigned long long incl_mask = __ballot((st & 3ULL) == 2ULL);
            const int hi = incl_mask ? 63 - __clzll(incl_mask) : -1;
            int64_t w[3] = {0, 0, 0};
            if (j >= 0 && t > hi)
                for (int q = 0; q < 3; ++q) w[q] = lb.agg[3 * j + q];
            if (j >= 0 && t == hi)
                for (int q = 0; q < 3; ++q) w[q] = lb.incl[3 * j + q];
            for (int q = 0; q < 3; ++q) {
                for (int off = 32; off >= 1; off >>= 1) w[q] += __shfl_xor(w[q], off, 64);
                pre[q] += w[q];
            }
            if (hi >= 0) break;
            end -= 64;
        }
        if (t == 0) {
            for (int q = 0; q < 3; ++q) {
                lb.incl[3 * tile + q] = pre[q] + agg[q];
                s_prefix[q] = pre[q];
            }
            __hip_atomic_store(&lb.status[tile], (epoch << 2) | 2ULL, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    if (!valid) return;
    const int64_t rb = s_prefix[0] + s_ex[grp][0];
    const int64_t vb = s_prefix[1] + s_ex[grp][1];
    const int64_t db = s_prefix[2] + s_ex[grp][2];
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
        if (first[q]) {
            col_idx[rb + rank[q]] = nb[q];
            val_ptr[rb + rank[q]] = vb + (int64_t)nbc * valoff[q];
        }
    }
    if (lane == 0) {
        col_idx[rb + self_rank] = c;
        val_ptr[rb + self_rank] = vb + (int64_t)nbc * self_valoff;
        row_ptr[c] = rb;
        dof_ptr[c] = db;
        if (c == m.n_cells - 1) {
            row_ptr[c + 1] = rb + my_blocks;
            dof_ptr[c + 1] = db + my_dofs;
            val_ptr[rb + my_blocks] = vb + my_vals;
        }
    }
}

int prep_tiles(int n_cells) { return (n_cells + CPB - 1) / CPB; }

void launch_prep(const DevMesh &m, const DevProblem &pr, CellGeo *geo, bool do_pattern, const Lookback &lb,
                 int64_t *row_ptr, int32_t *col_idx, int64_t *val_ptr, int64_t *dof_ptr, hipStream_t st) {
    const int n_tiles = prep_tiles(m.n_cells);
    hipLaunchKernelGGL(k_prep, dim3(n_tiles), dim3(WG), 0, st, m, pr, geo, do_pattern ? 1 : 0, n_tiles, lb, row_ptr,
                       col_idx, val_ptr, dof_ptr);
}

}  // namespace dgp
