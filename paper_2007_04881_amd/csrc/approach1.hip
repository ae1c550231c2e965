// Approach 1 of Section 3.3 (the paper's first assembly design), kept as an
// ablation beside the row-owner assembly: every element and every face
// computes its local blocks independently and emits them as COO records
// (block row, block column, values) with duplicates; a radix sort by (row,
// column) and a segmented reduction then form the block CSR matrix, its
// pattern included.  The paper finds this slower than building the pattern
// first (Approach 2, Section 3.4) because of the index work; the same
// comparison on this hardware is what the ablation measures.
//
// Records (uniform degree p, S = n_b^2 + n_b values each: the block, row-major,
// then a load part for diagonal records):
//   record c < N                 element c: volume block and load (eq. dg-bilinear
//                                first line, eq. dg-linear volume term)
//   record N + 4 f + s           face f: s = 0 left-left (with the boundary load on
//                                a boundary face), 1 left-right, 2 right-left,
//                                3 right-right (interior faces only)
// Unused slots carry the key N^2 and sort last.
//
// Kernels: k_coo_elem (one wave per element, a point per lane, the rank-3
// factors of every point staged in LDS, then each lane sums its block entries
// over the points), k_coo_face (eight lanes per face, the same staging),
// k_rs_hist / k_scan_small / k_rs_scatter (stable LSD radix sort of 8-bit digits of
// the keys, carrying record indices), k_coo_heads, k_coo_index (pattern from
// the sorted unique keys), k_coo_reduce (each unique block summed over its
// records in sorted order: deterministic, no atomics on values).
#include "approach1.h"
#include "asm_common.h"
#include "wave.h"

namespace dgp {

namespace {

constexpr int kRsTile = 2048;  // keys per radix-sort work-group (256 threads x 8)
constexpr int kFacesPerWave = 8;

template <typename T, int P>
struct A1Cfg {
    static constexpr int NB = nb2d(P);
    static constexpr int S = NB * NB + NB;  // record stride (values)
    static constexpr int TDEG = P <= 2 ? 4 : 2 * P;
    static constexpr int NQT = Tri<TDEG>::n;
    // element LDS row per point: g0, g1, v (NB each) and six coefficients
    static constexpr int EW = 3 * NB + 6;
    // face LDS row per point: v, dn of the left and the right element, and the
    // coefficients (alpha, beta, gamma) of the four blocks and the load (2)
    static constexpr int FW = 4 * NB + 14;
};

// ------------------------------------------------------------------ element
template <typename T, int P, bool ADV>
__global__ void __launch_bounds__(64) k_coo_elem(A1Args A) {
    using C = A1Cfg<T, P>;
    constexpr int NB = C::NB, S = C::S, EW = C::EW;
    constexpr int EPL = (S + 63) / 64;  // entries per lane
    using R_ = Tri<C::TDEG>;
    __shared__ T tab[64 * EW];
    const DevMesh &m = A.m;
    const DevProblem &pr = A.pr;
    const int lane = threadIdx.x;
    const int c = blockIdx.x;
    const int64_t s = m.cell_ptr[c];
    const int nv = (int)(m.cell_ptr[c + 1] - s);
    const CellGeo g = A.geo[c];
    const Box bx = box_of(g);
    const TrigCentre tc = trig_centre_of(g);
    const int v0 = m.cell_vtx[s];
    const double X0 = m.x[v0], Y0 = m.y[v0];
    const int npts = (nv - 2) * C::NQT;
    T acc[EPL];
#pragma unroll
    for (int k = 0; k < EPL; ++k) acc[k] = T(0);
    for (int base = 0; base < npts; base += 64) {
        const int q = base + lane;
        T *row = tab + lane * EW;
        if (q < npts) {
            const int t = q / C::NQT, qi = q - t * C::NQT;
            const int va = m.cell_vtx[s + 1 + t], vb = m.cell_vtx[s + 2 + t];
            const double X1 = m.x[va], Y1 = m.y[va], X2 = m.x[vb], Y2 = m.y[vb];
            const double area = 0.5 * ((X1 - X0) * (Y2 - Y0) - (X2 - X0) * (Y1 - Y0));
            // the point as the fan apex plus an offset; box coordinates from the offset
            const double l1 = R_::l(3 * qi + 1), l2 = R_::l(3 * qi + 2);
            const double dx = l1 * (X1 - X0) + l2 * (X2 - X0), dy = l1 * (Y1 - Y0) + l2 * (Y2 - Y0);
            const double px = X0 + dx, py = Y0 + dy;
            const double W = R_::w(qi) * area;
            const PointData pd = point_data_near(pr, tc, px, py, true);
            Eval<T, P> ev;
            ev.at(T(((X0 - g.lox) - (g.hix - X0) + 2.0 * dx) / (g.hix - g.lox)),
                  T(((Y0 - g.loy) - (g.hiy - Y0) + 2.0 * dy) / (g.hiy - g.loy)));
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                row[i] = ev.g0[i];
                row[NB + i] = ev.g1[i];
                row[2 * NB + i] = ev.v[i];
            }
            row[3 * NB + 0] = T(W * pd.a * bx.cx * bx.cx);
            row[3 * NB + 1] = T(W * pd.a * bx.cy * bx.cy);
            row[3 * NB + 2] = T(ADV ? W * pr.bx * bx.cx : 0.0);
            row[3 * NB + 3] = T(ADV ? W * pr.by * bx.cy : 0.0);
            row[3 * NB + 4] = T(ADV ? W * pr.c : 0.0);
            row[3 * NB + 5] = T(W * pd.f);
        }
        __syncthreads();
        const int nq = min(64, npts - base);
#pragma unroll
        for (int k = 0; k < EPL; ++k) {
            const int e = lane + 64 * k;
            if (e < S) {
                T sum = acc[k];
                if (e < NB * NB) {
                    const int i = e / NB, j = e - i * NB;
                    for (int qq = 0; qq < nq; ++qq) {
                        const T *r = tab + qq * EW;
                        const T tj = r[3 * NB + 2] * r[j] + r[3 * NB + 3] * r[NB + j] + r[3 * NB + 4] * r[2 * NB + j];
                        sum += r[3 * NB + 0] * r[i] * r[j] + r[3 * NB + 1] * r[NB + i] * r[NB + j] + r[2 * NB + i] * tj;
                    }
                } else {
                    const int i = e - NB * NB;
                    for (int qq = 0; qq < nq; ++qq) sum += tab[qq * EW + 3 * NB + 5] * tab[qq * EW + 2 * NB + i];
                }
                acc[k] = sum;
            }
        }
        __syncthreads();
    }
    const double isq = 1.0 / g.sqrt_box;
    T *out = static_cast<T *>(A.rec_vals) + (int64_t)c * S;
#pragma unroll
    for (int k = 0; k < EPL; ++k) {
        const int e = lane + 64 * k;
        if (e < NB * NB) {
            const int i = e / NB, j = e - i * NB;
            out[e] = T(double(acc[k]) * c_norm[i] * c_norm[j] * isq * isq);
        } else if (e < S) {
            out[e] = T(double(acc[k]) * c_norm[e - NB * NB] * isq);
        }
    }
    if (lane == 0) A.keys[c] = (uint64_t)c * (uint64_t)A.m.n_cells + (uint64_t)c;
}

// ------------------------------------------------------------------ faces
// Eight lanes per face, one Gauss point per lane (at most 5 points: p <= 4).
template <typename T, int P, bool ADV>
__global__ void __launch_bounds__(64) k_coo_face(A1Args A) {
    using C = A1Cfg<T, P>;
    constexpr int NB = C::NB, S = C::S, FW = C::FW;
    constexpr int NG = P + 1 > 3 ? P + 1 : 3;  // Gauss points per edge (uniform degree)
    __shared__ T tab[64 * FW];
    const DevMesh &m = A.m;
    const DevProblem &pr = A.pr;
    const int lane = threadIdx.x;
    const int fl = lane / 8, q = lane % 8;
    const int f = blockIdx.x * kFacesPerWave + fl;
    const int N = m.n_cells;
    const bool fvalid = f < m.n_faces;
    int L = 0, Rc = -1, bc = 0;
    if (fvalid) {
        L = m.face_cell[2 * f];
        Rc = m.face_cell[2 * f + 1];
        bc = m.face_bc[f];
    }
    T *row = tab + lane * FW;
    if (fvalid) {
        const int va = m.face_vtx[2 * f], vb = m.face_vtx[2 * f + 1];  // canonical: lower id first
        const double xa = m.x[va], ya = m.y[va];
        const double tx = m.x[vb] - xa, ty = m.y[vb] - ya;
        const double len = sqrt(tx * tx + ty * ty);
        // outward normal of the left element: from the edge's direction in its
        // counter-clockwise loop (the loop entry whose face is f starts the edge)
        const int64_t sl = m.cell_ptr[L];
        const int nvl = (int)(m.cell_ptr[L + 1] - sl);
        int start = va;
        for (int k = 0; k < nvl; ++k)
            if (m.cell_face[sl + k] == f) start = m.cell_vtx[sl + k];
        const double dl = (start == va ? 1.0 : -1.0) / len;
        const double nx = ty * dl, ny = -tx * dl;
        const CellGeo gL = A.geo[L];
        const Box bL = box_of(gL);
        const double bn = pr.bx * nx + pr.by * ny;
        if (q < NG) {
            const int goff = c_gl_off[NG - 1];
            const double tq = c_gl_t[goff + q];
            const double w = c_gl_w[goff + q] * len;
            const double dx = tq * tx, dy = tq * ty, px = xa + dx, py = ya + dy;
            T Lx[P + 1], dLx[P + 1], Ly[P + 1], dLy[P + 1];
            legendre<T, P>(T(((xa - gL.lox) - (gL.hix - xa) + 2.0 * dx) / (gL.hix - gL.lox)), Lx, dLx);
            legendre<T, P>(T(((ya - gL.loy) - (gL.hiy - ya) + 2.0 * dy) / (gL.hiy - gL.loy)), Ly, dLy);
            const T cnx = T(bL.cx * nx), cny = T(bL.cy * ny);
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                row[i] = Lx[exp_a(i)] * Ly[exp_b(i)];
                row[NB + i] = cnx * dLx[exp_a(i)] * Ly[exp_b(i)] + cny * Lx[exp_a(i)] * dLy[exp_b(i)];
            }
            T *cf = row + 4 * NB;
            if (Rc >= 0) {
                const CellGeo gR = A.geo[Rc];
                const Box bR = box_of(gR);
                legendre<T, P>(T(((xa - gR.lox) - (gR.hix - xa) + 2.0 * dx) / (gR.hix - gR.lox)), Lx, dLx);
                legendre<T, P>(T(((ya - gR.loy) - (gR.hiy - ya) + 2.0 * dy) / (gR.hiy - gR.loy)), Ly, dLy);
                const T rnx = T(bR.cx * nx), rny = T(bR.cy * ny);
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    row[2 * NB + i] = Lx[exp_a(i)] * Ly[exp_b(i)];
                    row[3 * NB + i] = rnx * dLx[exp_a(i)] * Ly[exp_b(i)] + rny * Lx[exp_a(i)] * dLy[exp_b(i)];
                }
                const double a = point_data_near(pr, trig_centre_of(gL), px, py, false).a;
                double sigma;
                if (pr.penalty == 1)
                    sigma = pr.c_sigma * len * fmax(A.pen_face[2 * f], A.pen_face[2 * f + 1]);
                else
                    sigma = pr.c_sigma * fmax(gL.pen, gR.pen);
                const double upL = bn < 0.0 ? bn : 0.0, upR = -bn < 0.0 ? -bn : 0.0;
                // blocks (test side X, trial side Y): LL, LR, RL, RR; s_L = 1, s_R = -1
                const double ha = 0.5 * a * w;
                cf[0] = T(-ha), cf[1] = T((sigma - upL) * w), cf[2] = T(-ha);      // LL
                cf[3] = T(-ha), cf[4] = T((-sigma + upL) * w), cf[5] = T(ha);      // LR
                cf[6] = T(ha), cf[7] = T((-sigma + upR) * w), cf[8] = T(-ha);      // RL
                cf[9] = T(ha), cf[10] = T((sigma - upR) * w), cf[11] = T(ha);      // RR
                cf[12] = cf[13] = T(0);
            } else {
#pragma unroll
                for (int i = 0; i < 2 * NB; ++i) row[2 * NB + i] = T(0);
#pragma unroll
                for (int k = 0; k < 14; ++k) cf[k] = T(0);
                if (bc == 1) {
                    const PointData pd = point_data(pr, px, py, false);
                    const double sigma = pr.penalty == 1 ? pr.c_sigma * len * A.pen_face[2 * f]
                                                         : pr.c_sigma * gL.pen;
                    const double up = bn < 0.0 ? bn : 0.0;
                    cf[0] = T(-pd.a * w), cf[1] = T((sigma - up) * w), cf[2] = T(-pd.a * w);
                    cf[12] = T(-pd.a * w * pd.u);          // times dn_i
                    cf[13] = T((sigma - up) * w * pd.u);   // times v_i
                } else {
                    const PointData pd = point_data(pr, px, py, false);
                    cf[13] = T(w * pd.a * (pd.ux * nx + pd.uy * ny));  // Neumann data times v_i
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < FW; ++k) row[k] = T(0);
        }
    }
    __syncthreads();
    // entries: face fl, block b = 0..3, entry e of S (load part on block 0 only)
    const int64_t rec0 = (int64_t)N + 4 * (int64_t)(blockIdx.x * kFacesPerWave);
    T *out = static_cast<T *>(A.rec_vals);
    for (int e = lane; e < kFacesPerWave * 4 * S; e += 64) {
        const int ff = e / (4 * S), r = e - ff * (4 * S), b = r / S, k = r - b * S;
        const int fg = blockIdx.x * kFacesPerWave + ff;
        if (fg >= m.n_faces) continue;
        const int Lf = m.face_cell[2 * fg], Rf = m.face_cell[2 * fg + 1];
        const int64_t rec = rec0 + 4 * ff + b;
        const bool used = b == 0 || Rf >= 0;
        if (k == 0 && used) {
            const int rr = (b < 2) ? Lf : Rf, cc = (b == 0 || b == 2) ? Lf : Rf;
            A.keys[rec] = (uint64_t)rr * (uint64_t)N + (uint64_t)cc;
        } else if (k == 0) {
            A.keys[rec] = (uint64_t)N * (uint64_t)N;
        }
        if (!used) continue;
        const int X = b < 2 ? 0 : 1, Y = (b == 0 || b == 2) ? 0 : 1;
        double sX = 1.0, sY = 1.0;
        {
            const int cx_ = X == 0 ? Lf : Rf, cy_ = Y == 0 ? Lf : Rf;
            sX = A.geo[cx_].sqrt_box;
            sY = A.geo[cy_].sqrt_box;
        }
        T sum = T(0);
        if (k < NB * NB) {
            const int i = k / NB, j = k - i * NB;
            for (int qq = 0; qq < NG; ++qq) {
                const T *pr_ = tab + (ff * 8 + qq) * FW;
                const T *cf = pr_ + 4 * NB + 3 * b;
                const T vi = pr_[2 * NB * X + i], dni = pr_[2 * NB * X + NB + i];
                const T vj = pr_[2 * NB * Y + j], dnj = pr_[2 * NB * Y + NB + j];
                sum += vi * (cf[0] * dnj + cf[1] * vj) + dni * cf[2] * vj;
            }
            out[rec * S + k] = T(double(sum) * c_norm[i] * c_norm[j] / (sX * sY));
        } else {
            const int i = k - NB * NB;
            if (b == 0)
                for (int qq = 0; qq < NG; ++qq) {
                    const T *pr_ = tab + (ff * 8 + qq) * FW;
                    sum += pr_[4 * NB + 12] * pr_[NB + i] + pr_[4 * NB + 13] * pr_[i];
                }
            out[rec * S + k] = T(double(sum) * c_norm[i] / sX);
        }
    }
}

// ------------------------------------------------------------------ radix sort
__global__ void __launch_bounds__(256) k_rs_hist(const uint64_t *__restrict__ keys, int n, int shift,
                                                  int *__restrict__ hist, int n_tiles) {
    __shared__ int h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int t0 = blockIdx.x * kRsTile;
    for (int k = threadIdx.x; k < kRsTile; k += 256) {
        const int i = t0 + k;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of n ints in one work-group; out may alias in
__global__ void __launch_bounds__(1024) k_scan_small(const int *__restrict__ in, int n, int *__restrict__ out,
                                                     int *__restrict__ total) {
    __shared__ int sh[1024];
    const int t = threadIdx.x;
    const int per = (n + 1023) / 1024;
    const int a = t * per, b = min(a + per, n);
    int run = 0;
    for (int i = a; i < b; ++i) run += in[i];
    sh[t] = run;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const int v = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    int acc = sh[t] - run;
    for (int i = a; i < b; ++i) {
        const int v = in[i];
        out[i] = acc;
        acc += v;
    }
    if (t == 1023 && total) *total = sh[1023];
}

// Stable scatter: the tile's keys in order, 256 at a time; a key's position is
// its digit's offset for the tile, plus the keys of that digit in earlier
// rounds, earlier waves and lower lanes (peers found by ballots on the digit's bits).
__global__ void __launch_bounds__(256) k_rs_scatter(const uint64_t *__restrict__ kin, const int *__restrict__ vin,
                                                     int n, int shift, const int *__restrict__ off, int n_tiles,
                                                     uint64_t *__restrict__ kout, int *__restrict__ vout) {
    __shared__ int run[256];
    __shared__ int wc[4][256];
    const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
    run[t] = 0;
    for (int w = 0; w < 4; ++w) wc[w][t] = 0;
    __syncthreads();
    const int t0 = blockIdx.x * kRsTile;
    for (int r = 0; r < kRsTile / 256; ++r) {
        const int i = t0 + r * 256 + t;
        const bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0;
        const int d = valid ? (int)((key >> shift) & 255) : 0;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t mb = __ballot(valid && ((d >> bit) & 1));
            peers &= ((d >> bit) & 1) ? mb : ~mb;
        }
        const int rank = __popcll(peers & ((1ull << lane) - 1ull));
        const int leader = valid && rank == 0;
        if (leader) wc[wv][d] = __popcll(peers);
        __syncthreads();
        if (valid) {
            int pos = off[d * n_tiles + blockIdx.x] + run[d] + rank;
            for (int w = 0; w < wv; ++w) pos += wc[w][d];
            kout[pos] = key;
            vout[pos] = vin[i];
        }
        __syncthreads();
        run[t] += wc[0][t] + wc[1][t] + wc[2][t] + wc[3][t];
        for (int w = 0; w < 4; ++w) wc[w][t] = 0;
        __syncthreads();
    }
}

__global__ void k_iota(int *v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = i;
}

// ------------------------------------------------------------------ reduction
// heads[k] = 1 where a new valid key starts (keys sorted)
__global__ void k_coo_heads(const uint64_t *__restrict__ keys, int n, uint64_t invalid, int *__restrict__ heads) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) heads[k] = keys[k] != invalid && (k == 0 || keys[k] != keys[k - 1]);
}

// Block pattern from the sorted unique keys: block u = the u-th distinct key.
// (blocks beyond nnzb_bound, the caller's buffer size, are not written; the
// count the host checks afterwards then differs)
__global__ void k_coo_index(const uint64_t *__restrict__ keys, const int *__restrict__ heads,
                            const int *__restrict__ uidx, int n, int n_cells, int nb, int nnzb_bound,
                            int64_t *__restrict__ row_ptr, int32_t *__restrict__ col_idx,
                            int64_t *__restrict__ val_ptr, int64_t *__restrict__ dof_ptr, int *__restrict__ seg) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n || !heads[k]) return;
    const int u = uidx[k];
    if (u >= nnzb_bound) return;
    const uint64_t key = keys[k];
    const int r = (int)(key / (uint64_t)n_cells), c = (int)(key % (uint64_t)n_cells);
    col_idx[u] = c;
    val_ptr[u] = (int64_t)u * nb * nb;
    seg[u] = k;
    if (k == 0 || keys[k - 1] / (uint64_t)n_cells != (uint64_t)r) {
        row_ptr[r] = u;
        dof_ptr[r] = (int64_t)r * nb;
    }
}

__global__ void k_coo_tail(int n_cells, int nb, int nnzb_bound, const int *__restrict__ total,
                           const int *__restrict__ n_valid, int64_t *__restrict__ row_ptr,
                           int64_t *__restrict__ val_ptr, int64_t *__restrict__ dof_ptr, int *__restrict__ seg) {
    const int u = *total < nnzb_bound ? *total : nnzb_bound;
    row_ptr[n_cells] = u;
    val_ptr[u] = (int64_t)u * nb * nb;
    dof_ptr[n_cells] = (int64_t)n_cells * nb;
    seg[u] = *n_valid;
}

// Each unique block summed over its records, in sorted (key, record) order, in
// double; a diagonal block also gives the row's load.
template <typename T, int P>
__global__ void __launch_bounds__(64) k_coo_reduce(const uint64_t *__restrict__ keys, const int *__restrict__ perm,
                                                   const int *__restrict__ seg, const T *__restrict__ rec_vals,
                                                   const int *__restrict__ total, int n_cells, T *__restrict__ vals,
                                                   T *__restrict__ rhs) {
    using C = A1Cfg<T, P>;
    constexpr int NB = C::NB, S = C::S;
    const int u = blockIdx.x;  // the grid is the caller's block count
    if (u >= *total) return;
    const int k0 = seg[u], k1 = seg[u + 1];
    const uint64_t key = keys[k0];
    const int r = (int)(key / (uint64_t)n_cells), c = (int)(key % (uint64_t)n_cells);
    for (int e = threadIdx.x; e < S; e += 64) {
        if (e >= NB * NB && r != c) break;
        double sum = 0.0;
        for (int k = k0; k < k1; ++k) sum += double(rec_vals[(int64_t)perm[k] * S + e]);
        if (e < NB * NB)
            vals[(int64_t)u * NB * NB + e] = T(sum);
        else
            rhs[(int64_t)r * NB + (e - NB * NB)] = T(sum);
    }
}

template <typename T, int P>
static void run_t(const A1Args &a, hipStream_t st) {
    const DevMesh &m = a.m;
    const bool adv = a.pr.bx != 0.0 || a.pr.by != 0.0 || a.pr.c != 0.0;
    const int nfb = (m.n_faces + kFacesPerWave - 1) / kFacesPerWave;
    if (adv) {
        hipLaunchKernelGGL((k_coo_elem<T, P, true>), dim3(m.n_cells), dim3(64), 0, st, a);
        hipLaunchKernelGGL((k_coo_face<T, P, true>), dim3(nfb), dim3(64), 0, st, a);
    } else {
        hipLaunchKernelGGL((k_coo_elem<T, P, false>), dim3(m.n_cells), dim3(64), 0, st, a);
        hipLaunchKernelGGL((k_coo_face<T, P, false>), dim3(nfb), dim3(64), 0, st, a);
    }
    // ---- the index step: sort the record keys, carrying record numbers
    const int n = a.n_records;
    const int n_tiles = (n + kRsTile - 1) / kRsTile;
    hipLaunchKernelGGL(k_iota, dim3((n + 255) / 256), dim3(256), 0, st, a.perm[0], n);
    const uint64_t maxkey = (uint64_t)m.n_cells * (uint64_t)m.n_cells;  // unused slots
    int bits = 1;
    while (bits < 64 && (maxkey >> bits)) ++bits;
    uint64_t *kin = a.keys;
    int *vin = a.perm[0];
    int side = 0;
    for (int shift = 0; shift < bits; shift += 8) {
        uint64_t *ko = a.keys_alt[side];
        int *vo = a.perm[1 + side];
        hipLaunchKernelGGL(k_rs_hist, dim3(n_tiles), dim3(256), 0, st, kin, n, shift, a.hist, n_tiles);
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, a.hist, 256 * n_tiles, a.hist, nullptr);
        hipLaunchKernelGGL(k_rs_scatter, dim3(n_tiles), dim3(256), 0, st, kin, vin, n, shift, a.hist, n_tiles, ko,
                           vo);
        kin = ko;
        vin = vo;
        side ^= 1;
    }
    // ---- unique keys -> block pattern; duplicates -> segmented sums
    hipLaunchKernelGGL(k_coo_heads, dim3((n + 255) / 256), dim3(256), 0, st, kin, n, maxkey, a.heads);
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, st, a.heads, n, a.uidx, a.total);
    hipLaunchKernelGGL(k_coo_index, dim3((n + 255) / 256), dim3(256), 0, st, kin, a.heads, a.uidx, n, m.n_cells,
                       nb2d(P), a.nnzb_bound, a.row_ptr, a.col_idx, a.val_ptr, a.dof_ptr, a.seg);
    hipLaunchKernelGGL(k_coo_tail, dim3(1), dim3(1), 0, st, m.n_cells, nb2d(P), a.nnzb_bound, a.total,
                       a.n_valid_records, a.row_ptr, a.val_ptr, a.dof_ptr, a.seg);
    hipLaunchKernelGGL((k_coo_reduce<T, P>), dim3(a.nnzb_bound), dim3(64), 0, st, kin, vin, a.seg,
                       static_cast<const T *>(a.rec_vals), a.total, m.n_cells, static_cast<T *>(a.vals),
                       static_cast<T *>(a.rhs));
}

}  // namespace

bool launch_approach1(const A1Args &a, int precision, int p, hipStream_t st) {
#define DGP_A1(T, PP)      \
    if (p == PP) {         \
        run_t<T, PP>(a, st); \
        return true;       \
    }
    if (precision == 0) {
        DGP_A1(double, 1) DGP_A1(double, 2) DGP_A1(double, 3) DGP_A1(double, 4)
    } else {
        DGP_A1(float, 1) DGP_A1(float, 2) DGP_A1(float, 3) DGP_A1(float, 4)
    }
#undef DGP_A1
    return false;
}

size_t approach1_record_values(int p) { return (size_t)(nb2d(p) * nb2d(p) + nb2d(p)); }

}  // namespace dgp
