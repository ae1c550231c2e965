// Element preparation, one pass over the mesh with eight lanes per element:
//
// * geometry in FP64 (kept FP64 in every precision mode): bounding box (the
//   basis lives on it, Section 3.1), h = diam(kappa) (Section 2.2), |kappa|,
//   and abar = max of a over the element's volume quadrature points (the
//   discrete ||a||_{L_inf(kappa)} of the penalty, Appendix A);
// * the neighbour across each edge of the loop (nbr; on the boundary minus the
//   boundary code: -1 Dirichlet, -2 Neumann);
// * the element's block row (Section 3.4, Approach 2: one block per element
//   and per distinct neighbour, however many faces they share): for every loop
//   edge a record with its start vertex, the neighbour, the rank of the
//   neighbour's block among the row's columns and the block's value offset
//   inside the row; per element the prefix of blocks, values and dofs inside
//   its tile of 32 elements and the position of the diagonal block; per tile
//   the sums.
// A second, one-work-group kernel scans the tile sums; work-groups never wait
// on one another (kernel boundaries order the three launches of a step).
#include "dgp_common.h"
#include "kernels.h"
#include "rules_data.h"
#include "wave.h"

namespace dgp {

namespace {

constexpr int G = 8;
constexpr int SLOTS = kMaxFaces2D / G;  // faces per lane
constexpr int WG = 256;
constexpr int CPB = WG / G;             // elements per tile
static_assert(CPB == kPrepTile, "tile size");

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
// reductions over the 8 lanes of a group (quad_perm xor 1, xor 2, half-row mirror)
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

// max of a over this lane's share of the volume points (fan triangles of the
// degree-DEG rule), the element's G lanes taking the points in turn
template <int DEG>
__device__ double max_a_points(const DevProblem &pr, const TrigCentre &tc, const double2 *loop, int nv, int lane) {
    const double *L = DEG == 4 ? c_tri4_l : DEG == 6 ? c_tri6_l : c_tri8_l;
    constexpr int n = DEG == 4 ? DGP_TRI4_N : DEG == 6 ? DGP_TRI6_N : DGP_TRI8_N;
    const double2 v0 = loop[0];
    double amax = -1e300;
    for (int k = lane; k < (nv - 2) * n; k += G) {
        const int t = k / n, q = k - t * n;
        const double2 v1 = loop[t + 1], v2 = loop[t + 2];
        const double px = L[3 * q] * v0.x + L[3 * q + 1] * v1.x + L[3 * q + 2] * v2.x;
        const double py = L[3 * q] * v0.y + L[3 * q + 1] * v1.y + L[3 * q + 2] * v2.y;
        amax = fmax(amax, coef_a_near(pr, tc, px, py));
    }
    return amax;
}

// The element's loop edges towards neighbours (nb >= 0) in the first NS slots of
// its G lanes: whether each is the first edge towards its neighbour (bit q of
// firstm) and how many of the loop's edges face that neighbour (dup)
template <int NS>
__device__ __forceinline__ void edge_dups(const int *nb, int lane, int base, int &firstm, int *dup) {
#pragma unroll
    for (int q2 = 0; q2 < NS; ++q2)
        for (int l2 = 0; l2 < G; ++l2) {
            const int v = __shfl(nb[q2], base + l2, 64);
            const int j = l2 + G * q2;
#pragma unroll
            for (int q = 0; q < NS; ++q)
                if (v == nb[q]) {
                    if (j < lane + G * q) firstm &= ~(1 << q);
                    dup[q] += 1;
                }
        }
}

// Column ranks and value offsets of the blocks of the first NS slots' edges
// (key: the neighbour's block size at its first edge, else 0), and of the
// diagonal block (column c)
template <int NS>
__device__ __forceinline__ void edge_ranks(const int *nb, const int *key, int c, int nbc, int base, int *rank,
                                           int *voff, int &drank, int &dvoff) {
#pragma unroll
    for (int q2 = 0; q2 < NS; ++q2)
        for (int l2 = 0; l2 < G; ++l2) {
            const int v = __shfl(nb[q2], base + l2, 64);
            const int vs = __shfl(key[q2], base + l2, 64);
            const int one = vs > 0 ? 1 : 0, w = nbc * vs;  // both 0 unless edge j is a first edge
#pragma unroll
            for (int q = 0; q < NS; ++q)
                if (v < nb[q]) {
                    rank[q] += one;
                    voff[q] += w;
                }
            if (v < c) {
                drank += one;
                dvoff += w;
            }
        }
}

}  // namespace

// p_uniform > 0: every cell has that degree (no neighbour degree is read)
__global__ void __launch_bounds__(WG) k_prep(DevMesh m, DevProblem pr, PrepOut out, int p_uniform) {
    __shared__ int s_cnt[CPB][3];
    __shared__ double2 s_xy[CPB][kMaxFaces2D];  // each element's vertex loop

    const int lane = threadIdx.x % G;
    const int grp = threadIdx.x / G;
    const int base = threadIdx.x & ~(G - 1);  // first lane of this element's group
    const int tile = xcd_block(blockIdx.x, gridDim.x);
    const int c = tile * CPB + grp;
    const bool valid = c < m.n_cells;
    int64_t s = 0;
    int nv = 0, p = 1;
    if (valid) {
        s = m.cell_ptr[c];
        nv = (int)(m.cell_ptr[c + 1] - s);
        p = m.cell_p[c];
    }

    // neighbours across this lane's edges and the edges' start vertices
    int nb[SLOTS], nbsz[SLOTS], code[SLOTS], vq[SLOTS], fq[SLOTS];
    double xq[SLOTS], yq[SLOTS];
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
        const int f = lane + G * q;
        nb[q] = -1;
        nbsz[q] = 0;
        code[q] = 0;
        vq[q] = 0;
        fq[q] = -1;
        xq[q] = yq[q] = 0.0;
        if (f < nv) {
            const int F = m.cell_face[s + f];
            fq[q] = F;
            const int o = other_cell(m, F, c);
            code[q] = o >= 0 ? o : -(int)m.face_bc[F];
            out.nbr[s + f] = code[q];
            if (o >= 0 && o != c) {
                nb[q] = o;
                nbsz[q] = nb2d(p_uniform > 0 ? p_uniform : m.cell_p[o]);
            }
            vq[q] = m.cell_vtx[s + f];
            xq[q] = m.x[vq[q]];
            yq[q] = m.y[vq[q]];
        }
    }

    // ------------------------------------------------------------ geometry
    // the loop goes to LDS once; the pair and triangle loops read it from there
    // (an element's eight lanes belong to one wave)
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
        const int i = lane + G * q;
        if (i < nv) s_xy[grp][i] = make_double2(xq[q], yq[q]);
    }
    wave_sync();
    double lox = 1e300, loy = 1e300, hix = -1e300, hiy = -1e300, a2 = 0.0, d2 = 0.0, amax = -1e300;
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
        const int i = lane + G * q;
        if (i < nv) {
            const double xi = xq[q], yi = yq[q];
            lox = fmin(lox, xi);
            loy = fmin(loy, yi);
            hix = fmax(hix, xi);
            hiy = fmax(hiy, yi);
            // shoelace about the first vertex: products of exact coordinate differences
            const double2 vn = s_xy[grp][i + 1 == nv ? 0 : i + 1], v0 = s_xy[grp][0];
            a2 += (xi - v0.x) * (vn.y - v0.y) - (vn.x - v0.x) * (yi - v0.y);
            for (int j = i + 1; j < nv; ++j) {
                const double2 vj = s_xy[grp][j];
                const double dx = xi - vj.x, dy = yi - vj.y;
                d2 = fmax(d2, dx * dx + dy * dy);
            }
        }
    }
    lox = gmin_d(lox);
    loy = gmin_d(loy);
    hix = gmax_d(hix);
    hiy = gmax_d(hiy);
    a2 = gsum_d(a2);
    d2 = gmax_d(d2);
    // sin/cos at the box centre, then abar over the volume points by angle addition from it
    const double hxb = hix - lox, hyb = hiy - loy;
    // sin/cos(pi x0) on even lanes, sin/cos(pi y0) on odd lanes, then swapped inside the pair
    TrigCentre tcen;
    tcen.x0 = 0.5 * (lox + hix);
    tcen.y0 = 0.5 * (loy + hiy);
    tcen.near = kPi * 0.5 * sqrt(hxb * hxb + hyb * hyb) <= kNearT;
    tcen.sx = tcen.sy = 0.0;
    tcen.cx = tcen.cy = 1.0;
    if (needs_trig(pr)) {
        const bool odd = lane & 1;
        double s1, c1;
        sincospi(odd ? tcen.y0 : tcen.x0, &s1, &c1);
        const double s2 = dpp_d<0xB1>(s1), c2 = dpp_d<0xB1>(c1);
        tcen.sx = odd ? s2 : s1;
        tcen.cx = odd ? c2 : c1;
        tcen.sy = odd ? s1 : s2;
        tcen.cy = odd ? c1 : c2;
    }
    if (valid && pr.a1 != 0.0)
        amax = p <= 2 ? max_a_points<4>(pr, tcen, s_xy[grp], nv, lane)
             : p == 3 ? max_a_points<6>(pr, tcen, s_xy[grp], nv, lane)
                      : max_a_points<8>(pr, tcen, s_xy[grp], nv, lane);
    amax = gmax_d(amax);

    // ------------------------------------------------------ row size
    // a neighbour counts once, at its first face
    // loop slots used by some element of this wave (most polygons fill one)
    const int nvmax = __builtin_amdgcn_readfirstlane(wave_max_i(nv));
    const int nslot = (nvmax + G - 1) / G;
    int firstm = 0;  // bit q: slot q's edge is the first towards its neighbour
    int dup[SLOTS];  // edges of the loop towards the same neighbour
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
        if (nb[q] >= 0) firstm |= 1 << q;
        dup[q] = 0;
    }
    static_assert(SLOTS == 3, "one instantiation per slot count");
    if (nslot <= 1)
        edge_dups<1>(nb, lane, base, firstm, dup);
    else if (nslot == 2)
        edge_dups<2>(nb, lane, base, firstm, dup);
    else
        edge_dups<3>(nb, lane, base, firstm, dup);
    int cnt = 0, szsum = 0;
#pragma unroll
    for (int q = 0; q < SLOTS; ++q)
        if ((firstm >> q) & 1) {
            cnt += 1;
            szsum += nbsz[q];
        }
    cnt = gsum_i(cnt);
    szsum = gsum_i(szsum);
    const int nbc = nb2d(p);
    const int my_blocks = valid ? 1 + cnt : 0;
    const int my_vals = valid ? nbc * (nbc + szsum) : 0;
    const int my_dofs = valid ? nbc : 0;

    // block ranks and value offsets (columns ascending; the diagonal block is column c)
    int rank[SLOTS], voff[SLOTS];
    int key[SLOTS];  // a neighbour's block size at its first edge, else 0
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
        rank[q] = nb[q] > c ? 1 : 0;
        voff[q] = nb[q] > c ? nbc * nbc : 0;
        key[q] = ((firstm >> q) & 1) ? nbsz[q] : 0;
    }
    int drank = 0, dvoff = 0;
    if (nslot <= 1)
        edge_ranks<1>(nb, key, c, nbc, base, rank, voff, drank, dvoff);
    else if (nslot == 2)
        edge_ranks<2>(nb, key, c, nbc, base, rank, voff, drank, dvoff);
    else
        edge_ranks<3>(nb, key, c, nbc, base, rank, voff, drank, dvoff);
#pragma unroll
    for (int q = 0; q < SLOTS; ++q) {
        const int f = lane + G * q;
        if (f < nv) {
            EdgeRec r;
            r.x = xq[q];
            r.y = yq[q];
            r.vid = vq[q];
            r.o = code[q];
            r.rank = nb[q] >= 0 ? (rank[q] | (dup[q] << kEdgeDupShift) | (((firstm >> q) & 1) ? kEdgeFirst : 0)) : 0;
            r.voff = nb[q] >= 0 ? voff[q] : 0;
            out.erec[s + f] = r;
        }
    }

    if (valid && pr.penalty == 1) {
        // covering penalty (Appendix A): this element's side of each of its faces,
        // the fan sub-triangle having the face as a side
        const double area = 0.5 * a2;
        const double abar = pr.a1 != 0.0 ? amax : pr.a0;
        const double cov = double(p * p) / area;
        const double2 v0 = s_xy[grp][0];
#pragma unroll
        for (int q = 0; q < SLOTS; ++q) {
            const int f = lane + G * q;
            if (f < nv) {
                const int t = f == 0 ? 1 : (f == nv - 1 ? nv - 2 : f);
                const double2 v1 = s_xy[grp][t], v2 = s_xy[grp][t + 1];
                const double kf = 0.5 * fabs((v1.x - v0.x) * (v2.y - v0.y) - (v2.x - v0.x) * (v1.y - v0.y));
                const double inv = 1.0 / kf;  // a degenerate sub-triangle leaves the C_cov bound
                const int side = m.face_cell[2 * fq[q]] == c ? 0 : 1;
                out.pen_face[2 * fq[q] + side] = abar * double(p * p) * (inv < cov ? inv : cov);
            }
        }
    }
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
        g.sx = tcen.sx;
        g.cx = tcen.cx;
        g.sy = tcen.sy;
        g.cy = tcen.cy;
        g.ihx = 1.0 / (hix - lox);
        g.ihy = 1.0 / (hiy - loy);
        g.isq = 1.0 / g.sqrt_box;
        g.pen = g.abar * double(p * p) / g.h;
        out.geo[c] = g;
    }
    if (lane == 0) {
        s_cnt[grp][0] = my_blocks;
        s_cnt[grp][1] = my_vals;
        s_cnt[grp][2] = my_dofs;
    }
    __syncthreads();
    if (valid && lane == 0) {
        // offsets of the element inside its tile, and where its diagonal block goes
        int pb = 0, pv = 0, pd = 0;
        for (int k = 0; k < grp; ++k) {
            pb += s_cnt[k][0];
            pv += s_cnt[k][1];
            pd += s_cnt[k][2];
        }
        out.cnt[4 * c + 0] = pb;
        out.cnt[4 * c + 1] = pv;
        out.cnt[4 * c + 2] = pd;
        out.cnt[4 * c + 3] = drank | (dvoff << 8);
    }
    if (threadIdx.x < 3) {
        int64_t sum = 0;
        for (int k = 0; k < CPB; ++k) sum += s_cnt[k][threadIdx.x];
        out.tile_sum[4 * tile + threadIdx.x] = (int)sum;  // at most 32 rows of 25 blocks of 15 x 15
        if (threadIdx.x == 0) out.tile_sum[4 * tile + 3] = 0;
    }
}

// Exclusive scan of the tile sums (blocks, values, dofs) into tile_off, and
// the totals after the last tile.  One work-group: each thread sums a run of
// consecutive tiles, the runs are scanned in LDS, then written back.
__global__ void __launch_bounds__(1024) k_tile_scan(const int32_t *__restrict__ tile_sum, int n_tiles,
                                                    int64_t *__restrict__ tile_off) {
    __shared__ int64_t sh[3][1024];
    const int t = threadIdx.x;
    const int per = (n_tiles + 1023) / 1024;
    const int a = t * per, b = min(a + per, n_tiles);
    // the run's first KC tile sums are loaded together (one 16-byte load each)
    // and kept for the write-back; longer runs read the rest twice
    constexpr int KC = 16;
    const int4 *ts = reinterpret_cast<const int4 *>(tile_sum);
    int4 keep[KC];
#pragma unroll
    for (int k = 0; k < KC; ++k) keep[k] = a + k < b ? ts[a + k] : make_int4(0, 0, 0, 0);
    int64_t run[3] = {0, 0, 0};
#pragma unroll
    for (int k = 0; k < KC; ++k) {
        run[0] += keep[k].x;
        run[1] += keep[k].y;
        run[2] += keep[k].z;
    }
    for (int i = a + KC; i < b; ++i) {
        const int4 v = ts[i];
        run[0] += v.x;
        run[1] += v.y;
        run[2] += v.z;
    }
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
        if (a + k < b) {
            tile_off[3 * (a + k) + 0] = acc[0];
            tile_off[3 * (a + k) + 1] = acc[1];
            tile_off[3 * (a + k) + 2] = acc[2];
            acc[0] += keep[k].x;
            acc[1] += keep[k].y;
            acc[2] += keep[k].z;
        }
    for (int i = a + KC; i < b; ++i) {
        const int4 v = ts[i];
        tile_off[3 * i + 0] = acc[0];
        tile_off[3 * i + 1] = acc[1];
        tile_off[3 * i + 2] = acc[2];
        acc[0] += v.x;
        acc[1] += v.y;
        acc[2] += v.z;
    }
    if (t == 1023)
        for (int q = 0; q < 3; ++q) tile_off[3 * n_tiles + q] = sh[q][1023];
}

void launch_prep(const DevMesh &m, const DevProblem &pr, const PrepOut &out, hipStream_t st, bool scan, int p_uniform) {
    const int n_tiles = (m.n_cells + kPrepTile - 1) / kPrepTile;
    hipLaunchKernelGGL(k_prep, dim3(n_tiles), dim3(WG), 0, st, m, pr, out, p_uniform);
    if (scan) hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, st, out.tile_sum, n_tiles, out.tile_off);
}

}  // namespace dgp
