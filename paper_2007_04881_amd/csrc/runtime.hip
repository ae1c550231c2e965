// Host runtime behind the C ABI of include/dgpoly.h: context, mesh upload and
// validation, device buffers, kernel launches, graph capture and timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ctx.h"
#include "kernels.h"

using namespace dgp;

#define fail dgp_fail


dgp_status dgp_fail(dgp_ctx *ctx, dgp_status st, const char *fmt, ...) {
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
        va_end(ap);
    }
    return st;
}



static void free_pattern(dgp_ctx *c) {
    c->has_pattern = false;
}

static void free_graph(dgp_ctx *c) {
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->exec = nullptr;
    c->graph = nullptr;
}

static void free_mesh(dgp_ctx *c) {
    for (void *p : c->mesh_bufs) (void)hipFree(p);
    c->mesh_bufs.clear();
    if (c->rows_by_p) (void)hipFree(c->rows_by_p);
    c->rows_by_p = nullptr;
    if (c->rows_sub) (void)hipFree(c->rows_sub);
    c->rows_sub = nullptr;
    if (c->rows_lpt) (void)hipFree(c->rows_lpt);
    c->rows_lpt = nullptr;
    if (c->rows_3d) (void)hipFree(c->rows_3d);
    c->rows_3d = nullptr;
    dgp_free_approach1(c);
    for (void *p : {(void *)c->row_ptr, (void *)c->col_idx, (void *)c->val_ptr, (void *)c->dof_ptr, c->work})
        if (p) (void)hipFree(p);
    c->row_ptr = c->val_ptr = c->dof_ptr = nullptr;
    c->col_idx = nullptr;
    c->work = nullptr;
    dgp_free_qrule(c);
    c->has_mesh = false;
    c->has_last = false;
    free_pattern(c);
    free_graph(c);
}

template <typename T>
static dgp_status upload(dgp_ctx *c, const T *src, int64_t n, const T **dst) {
    void *p = nullptr;
    size_t bytes = sizeof(T) * (size_t)(n > 0 ? n : 1);
    if (hipMalloc(&p, bytes) != hipSuccess) return fail(c, DGP_ENOMEM, "hipMalloc(%zu) failed", bytes);
    c->mesh_bufs.push_back(p);
    if (n > 0) HIPCHK(c, hipMemcpy(p, src, sizeof(T) * (size_t)n, hipMemcpyHostToDevice));
    *dst = static_cast<const T *>(p);
    return DGP_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// ---- static scratch of dgp_run_static
// The preparation outputs of a step taken by dgp_run_static live in this
// array instead of the buffer the context allocates at upload.  Each device
// the library runs on holds its own copy for the life of the process.  In host
// code `scratch` only names the symbol: its device address, per device, comes
// from hipGetSymbolAddress at context creation and is the only address that
// host code passes on.
static __device__ __align__(256) unsigned char scratch[DGP_STATIC_SCRATCH_BYTES];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device `device` (looked up once per device).
static hipError_t static_scratch_address(int device, void **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_addr[device] = ptr;
    }
    *out = g_scratch_addr[device];
    return hipSuccess;
}

__global__ void k_fill_i32(int32_t *p, int n, int32_t v) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// The preparation outputs of one step (2D: per-face penalty sides, cell
// records, edge neighbours and records, row counts, tile sums and offsets)
// carved from one buffer at base;
// with base = null only the size is computed.  Returns the size in bytes.
static size_t layout2d(int64_t N, int64_t nnz_v, int64_t F, int n_tiles, char *base, PrepOut *o) {
    const size_t o_pen = 0;
    const size_t o_geo = o_pen + align256(sizeof(double) * 2 * (size_t)F);
    const size_t o_nbr = o_geo + align256(sizeof(CellGeo) * (size_t)N);
    const size_t o_erec = o_nbr + align256(sizeof(int32_t) * (size_t)nnz_v);
    const size_t o_cnt = o_erec + align256(sizeof(EdgeRec) * (size_t)nnz_v);
    const size_t o_tile = o_cnt + align256(sizeof(int32_t) * 4 * (size_t)N);
    const size_t o_off = o_tile + align256(sizeof(int32_t) * 4 * (size_t)n_tiles);
    const size_t bytes = o_off + sizeof(int64_t) * 3 * (size_t)(n_tiles + 1);
    if (base && o) {
        o->pen_face = reinterpret_cast<double *>(base + o_pen);
        o->geo = reinterpret_cast<CellGeo *>(base + o_geo);
        o->nbr = reinterpret_cast<int32_t *>(base + o_nbr);
        o->erec = reinterpret_cast<EdgeRec *>(base + o_erec);
        o->cnt = reinterpret_cast<int32_t *>(base + o_cnt);
        o->tile_sum = reinterpret_cast<int32_t *>(base + o_tile);
        o->tile_off = reinterpret_cast<int64_t *>(base + o_off);
    }
    return bytes;
}

// The same for polyhedra: cell records, face order and groups, row counts,
// tile sums and offsets, and the limit flag (which must start at zero).
static size_t layout3d(int64_t N, int64_t n_cf, int n_tiles, char *base, Prep3Out *o) {
    const size_t o_geo = 0;
    const size_t o_ord = o_geo + align256(sizeof(CellGeo3) * (size_t)N);
    const size_t o_grp = o_ord + align256(sizeof(int32_t) * (size_t)n_cf);
    const size_t o_cnt = o_grp + align256(sizeof(FaceGroup) * (size_t)n_cf);
    const size_t o_tile = o_cnt + align256(sizeof(int32_t) * 4 * (size_t)N);
    const size_t o_off = o_tile + align256(sizeof(int64_t) * 3 * (size_t)n_tiles);
    const size_t o_err = o_off + align256(sizeof(int64_t) * 3 * (size_t)(n_tiles + 1));
    const size_t bytes = o_err + 256;
    if (base && o) {
        o->geo = reinterpret_cast<CellGeo3 *>(base + o_geo);
        o->forder = reinterpret_cast<int32_t *>(base + o_ord);
        o->grp = reinterpret_cast<FaceGroup *>(base + o_grp);
        o->cnt = reinterpret_cast<int32_t *>(base + o_cnt);
        o->tile_sum = reinterpret_cast<int64_t *>(base + o_tile);
        o->tile_off = reinterpret_cast<int64_t *>(base + o_off);
        o->err = reinterpret_cast<int32_t *>(base + o_err);
    }
    return bytes;
}

extern "C" {

dgp_status dgp_create(dgp_ctx **out, int device, void *hip_stream) {
    if (!out) return DGP_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return DGP_EDEVICE;
    dgp_ctx *c = new dgp_ctx();
    c->device = device;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (hipSetDevice(device) != hipSuccess) {
        delete c;
        return DGP_EDEVICE;
    }
    for (auto &e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            delete c;
            return DGP_EDEVICE;
        }
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return DGP_EDEVICE;
    }
    if (static_scratch_address(device, &c->static_scratch) != hipSuccess) {
        (void)hipStreamDestroy(c->cap_stream);
        for (auto &e : c->ev)
            if (e) (void)hipEventDestroy(e);
        delete c;
        return DGP_EDEVICE;
    }
    *out = c;
    return DGP_OK;
}

dgp_status dgp_destroy(dgp_ctx *ctx) {
    if (!ctx) return DGP_EINVAL;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    free_mesh(ctx);
    if (ctx->mlp) (void)hipFree(ctx->mlp);
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    delete ctx;
    return DGP_OK;
}

dgp_status dgp_set_stream(dgp_ctx *ctx, void *hip_stream) {
    if (!ctx) return DGP_EINVAL;
    ctx->stream = static_cast<hipStream_t>(hip_stream);
    return DGP_OK;
}

const char *dgp_last_error(const dgp_ctx *ctx) { return ctx ? ctx->err : "null context"; }

static dgp_status upload3d(dgp_ctx *ctx, const dgp_mesh_desc *m);

static dgp_status validate3d(dgp_ctx *ctx, const dgp_mesh_desc *m, int *pmin_out, int *pmax_out);

// Host checks of a 2D mesh (no device work); err text goes to ctx->err.
static dgp_status validate2d(dgp_ctx *ctx, const dgp_mesh_desc *m, int *pmin_out, int *pmax_out) {
    if (m->n_cells <= 0 || m->n_vertices <= 0 || m->n_faces <= 0)
        return fail(ctx, DGP_EINVAL, "empty mesh (cells %lld, vertices %lld, faces %lld)", (long long)m->n_cells,
                    (long long)m->n_vertices, (long long)m->n_faces);
    if (m->n_cells > INT32_MAX / 2 || m->n_faces > INT32_MAX / 2 || m->n_vertices > INT32_MAX / 2)
        return fail(ctx, DGP_EUNSUPPORTED, "mesh too large for 32-bit ids");
    if (!m->x || !m->y || !m->cell_ptr || !m->cell_vtx || !m->cell_p || !m->cell_face_ptr || !m->cell_face ||
        !m->face_vtx || !m->face_cell || !m->face_bc)
        return fail(ctx, DGP_EINVAL, "null mesh array");
    const int64_t N = m->n_cells, F = m->n_faces, V = m->n_vertices;
    // ---- host validation: ids, loops, faces listed by the cells they bound
    if (m->cell_ptr[0] != 0) return fail(ctx, DGP_EMESH, "cell_ptr[0] != 0");
    int pmin = 99, pmax = -1;
    for (int64_t c = 0; c < N; ++c) {
        int64_t s = m->cell_ptr[c], e = m->cell_ptr[c + 1];
        if (e - s < 3) return fail(ctx, DGP_EMESH, "cell %lld has %lld vertices", (long long)c, (long long)(e - s));
        if (e - s > kMaxFaces2D)
            return fail(ctx, DGP_EUNSUPPORTED, "cell %lld has %lld faces (at most %d)", (long long)c,
                        (long long)(e - s), kMaxFaces2D);
        if (m->cell_face_ptr[c] != s || m->cell_face_ptr[c + 1] != e)
            return fail(ctx, DGP_EMESH, "2D cell_face_ptr must equal cell_ptr (cell %lld)", (long long)c);
        int p = m->cell_p[c];
        if (p < 1 || p > kMaxP) return fail(ctx, DGP_EUNSUPPORTED, "cell %lld has degree %d", (long long)c, p);
        pmin = p < pmin ? p : pmin;
        pmax = p > pmax ? p : pmax;
        for (int64_t k = s; k < e; ++k) {
            int32_t v = m->cell_vtx[k], f = m->cell_face[k];
            if (v < 0 || v >= V) return fail(ctx, DGP_EMESH, "cell %lld: vertex id %d out of range", (long long)c, v);
            if (f < 0 || f >= F) return fail(ctx, DGP_EMESH, "cell %lld: face id %d out of range", (long long)c, f);
            if (m->face_cell[2 * f] != c && m->face_cell[2 * f + 1] != c)
                return fail(ctx, DGP_EMESH, "face %d is not adjacent to cell %lld", f, (long long)c);
            int32_t w = m->cell_vtx[k + 1 < e ? k + 1 : s];
            int32_t a = m->face_vtx[2 * f], b = m->face_vtx[2 * f + 1];
            if (!((a == v && b == w) || (a == w && b == v)))
                return fail(ctx, DGP_EMESH, "face %d does not match edge %lld of cell %lld", f, (long long)(k - s),
                            (long long)c);
        }
        // the loop must run counter-clockwise around a cell of positive area: the
        // kernels take outward normals and fan weights from that orientation.
        // Twice the signed area (shoelace about the first vertex) against the
        // square of the box extent, so that the test does not depend on scale.
        const double x0 = m->x[m->cell_vtx[s]], y0 = m->y[m->cell_vtx[s]];
        double a2 = 0.0, lx = x0, hx = x0, ly = y0, hy = y0;
        for (int64_t k = s; k < e; ++k) {
            const int32_t v = m->cell_vtx[k], w = m->cell_vtx[k + 1 < e ? k + 1 : s];
            const double xv = m->x[v], yv = m->y[v];
            a2 += (xv - x0) * (m->y[w] - y0) - (m->x[w] - x0) * (yv - y0);
            lx = xv < lx ? xv : lx;
            hx = xv > hx ? xv : hx;
            ly = yv < ly ? yv : ly;
            hy = yv > hy ? yv : hy;
        }
        const double ext2 = (hx - lx) * (hx - lx) + (hy - ly) * (hy - ly);
        if (!(a2 > 1e-13 * ext2))
            return fail(ctx, DGP_EMESH, "cell %lld: %s vertex loop (twice the signed area %.3e)", (long long)c,
                        a2 < 0.0 ? "clockwise" : "zero-area", a2);
    }
    for (int64_t f = 0; f < F; ++f) {
        int32_t l = m->face_cell[2 * f], r = m->face_cell[2 * f + 1];
        int8_t bc = m->face_bc[f];
        if (l < 0 || l >= N || r < -1 || r >= N || r == l)
            return fail(ctx, DGP_EMESH, "face %lld: bad cells (%d, %d)", (long long)f, l, r);
        if ((r < 0) != (bc != 0) || bc < 0 || bc > 2)
            return fail(ctx, DGP_EMESH, "face %lld: boundary code %d inconsistent with cells", (long long)f, bc);
        if (m->face_vtx[2 * f] >= m->face_vtx[2 * f + 1])
            return fail(ctx, DGP_EMESH, "face %lld: vertices not in canonical (ascending) order", (long long)f);
    }
    *pmin_out = pmin;
    *pmax_out = pmax;
    return DGP_OK;
}

dgp_status dgp_mesh_check(const dgp_mesh_desc *m, char *msg, size_t msg_len) {
    if (msg && msg_len) msg[0] = 0;
    if (!m) return DGP_EINVAL;
    dgp_ctx tmp;  // carries the message only; no device state is touched
    int pmin = 0, pmax = 0;
    dgp_status st = m->dim == 3   ? validate3d(&tmp, m, &pmin, &pmax)
                    : m->dim == 2 ? validate2d(&tmp, m, &pmin, &pmax)
                                  : fail(&tmp, DGP_EUNSUPPORTED, "dim %d", m->dim);
    if (msg && msg_len) snprintf(msg, msg_len, "%s", tmp.err);
    return st;
}

dgp_status dgp_mesh_upload(dgp_ctx *ctx, const dgp_mesh_desc *m) {
    if (!ctx || !m) return DGP_EINVAL;
    if (m->dim == 3) return upload3d(ctx, m);
    if (m->dim != 2) return fail(ctx, DGP_EUNSUPPORTED, "dim %d", m->dim);
    int pmin = 0, pmax = 0;
    dgp_status vst = validate2d(ctx, m, &pmin, &pmax);
    if (vst != DGP_OK) return vst;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int64_t N = m->n_cells, F = m->n_faces, V = m->n_vertices;
    const int64_t nnz_v = m->cell_ptr[N];
    free_mesh(ctx);
    ctx->dim = 2;
    ctx->n_cell_face = nnz_v;
    ctx->n_cells = N;
    ctx->n_faces = F;
    ctx->n_vertices = V;
    ctx->n_cell_vtx = nnz_v;
    ctx->p_uniform = pmin == pmax ? pmin : -1;
    ctx->p_max = pmax;
    DevMesh &d = ctx->dm;
    d = DevMesh{};
    d.n_cells = (int32_t)N;
    d.n_faces = (int32_t)F;
    d.n_vertices = (int32_t)V;
    dgp_status st;
#define UP(arr, n, field)                                         \
    if ((st = upload(ctx, m->arr, (n), &d.field)) != DGP_OK) { \
        free_mesh(ctx);                                           \
        return st;                                                \
    }
    UP(x, V, x)
    UP(y, V, y)
    UP(cell_ptr, N + 1, cell_ptr)
    UP(cell_vtx, nnz_v, cell_vtx)
    UP(cell_p, N, cell_p)
    UP(cell_face_ptr, N + 1, cell_face_ptr)
    UP(cell_face, nnz_v, cell_face)
    UP(face_vtx, 2 * F, face_vtx)
    UP(face_cell, 2 * F, face_cell)
    UP(face_bc, F, face_bc)
#undef UP
    // pattern arrays at their upper bound (a row has at most 1 + #faces blocks);
    // geometry records, edge neighbours, row sizes and their tile sums
    const int64_t nnzb_max = N + nnz_v;
    ctx->n_tiles = (int)((N + kPrepTile - 1) / kPrepTile);
    const size_t work_bytes = layout2d(N, nnz_v, F, ctx->n_tiles, nullptr, nullptr);
    if (hipMalloc(&ctx->row_ptr, sizeof(int64_t) * (N + 1)) != hipSuccess ||
        hipMalloc(&ctx->col_idx, sizeof(int32_t) * nnzb_max) != hipSuccess ||
        hipMalloc(&ctx->val_ptr, sizeof(int64_t) * (nnzb_max + 1)) != hipSuccess ||
        hipMalloc(&ctx->dof_ptr, sizeof(int64_t) * (N + 1)) != hipSuccess ||
        hipMalloc(&ctx->work, work_bytes) != hipSuccess) {
        free_mesh(ctx);
        return fail(ctx, DGP_ENOMEM, "device allocation failed");
    }
    HIPCHK(ctx, hipMemset(ctx->work, 0, work_bytes));
    layout2d(N, nnz_v, F, ctx->n_tiles, static_cast<char *>(ctx->work), &ctx->prep);
    if (pmin != pmax) {
        // mixed degrees: one launch per degree over the elements of that degree (in id order)
        std::vector<int32_t> rows((size_t)N);
        int64_t cnt[kMaxP + 2] = {};
        for (int64_t c = 0; c < N; ++c) cnt[m->cell_p[c] + 1] += 1;
        for (int p = 1; p <= kMaxP + 1; ++p) cnt[p] += cnt[p - 1];
        for (int p = 0; p <= kMaxP + 1; ++p) ctx->rows_off[p] = cnt[p];
        for (int64_t c = 0; c < N; ++c) rows[(size_t)cnt[m->cell_p[c]]++] = (int32_t)c;
        if (hipMalloc(&ctx->rows_by_p, sizeof(int32_t) * (size_t)N) != hipSuccess) {
            free_mesh(ctx);
            return fail(ctx, DGP_ENOMEM, "row groups");
        }
        HIPCHK(ctx, hipMemcpy(ctx->rows_by_p, rows.data(), sizeof(int32_t) * (size_t)N, hipMemcpyHostToDevice));
    }
    {
        // boundary faces, and the most edges a cell shares with one neighbour
        int64_t nbf = 0;
        for (int64_t f = 0; f < F; ++f) nbf += m->face_cell[2 * f + 1] < 0;
        int mdup = 1;
        for (int64_t c = 0; c < N; ++c) {
            const int64_t s = m->cell_ptr[c], e = m->cell_ptr[c + 1];
            for (int64_t k = s; k < e; ++k) {
                const int32_t f = m->cell_face[k];
                const int32_t o = m->face_cell[2 * f] == c ? m->face_cell[2 * f + 1] : m->face_cell[2 * f];
                if (o < 0) continue;
                int cnt = 0;
                for (int64_t j = s; j < e; ++j) {
                    const int32_t g = m->cell_face[j];
                    cnt += (m->face_cell[2 * g] == c ? m->face_cell[2 * g + 1] : m->face_cell[2 * g]) == o;
                }
                mdup = cnt > mdup ? cnt : mdup;
            }
        }
        ctx->n_boundary_faces = nbf;
        ctx->max_dup2d = mdup;
    }
    if (pmin != pmax) {
        // one persistent launch over all degrees takes the rows bin by bin,
        // costliest first: (degree, fan sub-triangle count) descending, stable in id
        constexpr int NS = kMaxFaces2D;
        std::vector<int64_t> bc((size_t)(kMaxP + 1) * NS + 1, 0);
        auto key = [&](int64_t c) {
            return (int64_t)(kMaxP - m->cell_p[c]) * NS + (NS - 1 - (m->cell_ptr[c + 1] - m->cell_ptr[c] - 2));
        };
        for (int64_t c = 0; c < N; ++c) bc[(size_t)key(c) + 1] += 1;
        for (size_t k = 1; k < bc.size(); ++k) bc[k] += bc[k - 1];
        std::vector<int32_t> rows((size_t)N);
        for (int64_t c = 0; c < N; ++c) rows[(size_t)bc[(size_t)key(c)]++] = (int32_t)c;
        if (hipMalloc(&ctx->rows_lpt, sizeof(int32_t) * (size_t)N) != hipSuccess) {
            free_mesh(ctx);
            return fail(ctx, DGP_ENOMEM, "row bins (single launch)");
        }
        HIPCHK(ctx, hipMemcpy(ctx->rows_lpt, rows.data(), sizeof(int32_t) * (size_t)N, hipMemcpyHostToDevice));
    }
    {
        // the second row order dgp_autotune chooses from: the rows of each degree
        // (Section 3.1's grouping) in id order, cut into the eight ranges that a
        // launch over them gives the XCDs (xcd_block: XCD x runs a contiguous
        // range of blocks, in order), each range sorted by the number of fan
        // sub-triangles n_sub = n_v - 2, largest first (stable in id).  Every
        // XCD keeps the rows, and the cache lines, of the id order but starts
        // its costliest rows first, so that the launch does not end on them.
        std::vector<int64_t> pc((size_t)kMaxP + 2, 0);
        for (int64_t c = 0; c < N; ++c) pc[(size_t)m->cell_p[c] + 1] += 1;
        for (int p = 1; p <= kMaxP + 1; ++p) pc[(size_t)p] += pc[(size_t)p - 1];
        for (int p = 0; p <= kMaxP + 1; ++p) ctx->rows_off[p] = pc[(size_t)p];
        std::vector<int32_t> rows((size_t)N);
        {
            std::vector<int64_t> pos(pc.begin(), pc.end());
            for (int64_t c = 0; c < N; ++c) rows[(size_t)pos[(size_t)m->cell_p[c]]++] = (int32_t)c;
        }
        auto nsub = [&](int32_t c) { return m->cell_ptr[c + 1] - m->cell_ptr[c] - 2; };
        for (int p = 0; p <= kMaxP; ++p) {
            const int64_t o = pc[(size_t)p], n = pc[(size_t)p + 1] - o;
            const int64_t nb = (n + 3) / 4, q = nb >> 3, r = nb & 7;  // as xcd_block over nb blocks of 4 rows
            for (int64_t x = 0; x < 8; ++x) {
                const int64_t b0 = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q, bn = x < r ? q + 1 : q;
                const int64_t lo = o + std::min(4 * b0, n), hi = o + std::min(4 * (b0 + bn), n);
                std::stable_sort(rows.begin() + lo, rows.begin() + hi,
                                 [&](int32_t a, int32_t b) { return nsub(a) > nsub(b); });
            }
        }
        if (hipMalloc(&ctx->rows_sub, sizeof(int32_t) * (size_t)N) != hipSuccess) {
            free_mesh(ctx);
            return fail(ctx, DGP_ENOMEM, "row bins");
        }
        HIPCHK(ctx, hipMemcpy(ctx->rows_sub, rows.data(), sizeof(int32_t) * (size_t)N, hipMemcpyHostToDevice));
    }
    ctx->has_mesh = true;
    return DGP_OK;
}

// Polyhedral mesh: cells are unions of tetrahedra (4 ids each), faces are
// triangles with the opposite vertex of the left cell's tetrahedron.
static dgp_status validate3d(dgp_ctx *ctx, const dgp_mesh_desc *m, int *pmin_out, int *pmax_out) {
    if (m->n_cells <= 0 || m->n_vertices <= 0 || m->n_faces <= 0)
        return fail(ctx, DGP_EINVAL, "empty mesh (cells %lld, vertices %lld, faces %lld)", (long long)m->n_cells,
                    (long long)m->n_vertices, (long long)m->n_faces);
    if (m->n_cells > INT32_MAX / 2 || m->n_faces >= (int64_t(1) << 27) || m->n_vertices > INT32_MAX / 2)
        return fail(ctx, DGP_EUNSUPPORTED, "mesh too large (3D: fewer than 2^27 faces)");
    if (!m->x || !m->y || !m->z || !m->cell_ptr || !m->cell_vtx || !m->cell_p || !m->cell_face_ptr ||
        !m->cell_face || !m->face_vtx || !m->face_cell || !m->face_bc || !m->face_opp)
        return fail(ctx, DGP_EINVAL, "null mesh array");
    const int64_t N = m->n_cells, F = m->n_faces, V = m->n_vertices;
    if (m->cell_ptr[0] != 0 || m->cell_face_ptr[0] != 0) return fail(ctx, DGP_EMESH, "cell_ptr[0] or cell_face_ptr[0] != 0");
    int pmin = 99, pmax = -1;
    for (int64_t c = 0; c < N; ++c) {
        const int64_t s = m->cell_ptr[c], e = m->cell_ptr[c + 1];
        if (e - s < 4 || (e - s) % 4 || s % 4)
            return fail(ctx, DGP_EMESH, "cell %lld: %lld tetrahedron vertex ids (need a positive multiple of 4)",
                        (long long)c, (long long)(e - s));
        for (int64_t k = s; k < e; ++k)
            if (m->cell_vtx[k] < 0 || m->cell_vtx[k] >= V)
                return fail(ctx, DGP_EMESH, "cell %lld: vertex id %d out of range", (long long)c, m->cell_vtx[k]);
        // every tetrahedron must have positive volume (either orientation: the
        // volume weights use |det|); relative to the cube of its longest edge
        for (int64_t k = s; k < e; k += 4) {
            double v[4][3], l2 = 0.0;
            for (int j = 0; j < 4; ++j) {
                const int32_t id = m->cell_vtx[k + j];
                v[j][0] = m->x[id];
                v[j][1] = m->y[id];
                v[j][2] = m->z[id];
            }
            double d[3][3];
            for (int j = 0; j < 3; ++j)
                for (int q = 0; q < 3; ++q) d[j][q] = v[j + 1][q] - v[0][q];
            for (int j = 0; j < 4; ++j)
                for (int i = j + 1; i < 4; ++i) {
                    const double e2 = (v[i][0] - v[j][0]) * (v[i][0] - v[j][0]) +
                                      (v[i][1] - v[j][1]) * (v[i][1] - v[j][1]) +
                                      (v[i][2] - v[j][2]) * (v[i][2] - v[j][2]);
                    l2 = e2 > l2 ? e2 : l2;
                }
            const double det = d[0][0] * (d[1][1] * d[2][2] - d[1][2] * d[2][1]) -
                               d[0][1] * (d[1][0] * d[2][2] - d[1][2] * d[2][0]) +
                               d[0][2] * (d[1][0] * d[2][1] - d[1][1] * d[2][0]);
            if (!(fabs(det) > 1e-13 * l2 * sqrt(l2)))
                return fail(ctx, DGP_EMESH, "cell %lld: tetrahedron %lld has zero volume", (long long)c,
                            (long long)((k - s) / 4));
        }
        const int p = m->cell_p[c];
        if (p < 1 || p > kMaxP3D) return fail(ctx, DGP_EUNSUPPORTED, "3D cell %lld has degree %d (1..%d)", (long long)c, p, kMaxP3D);
        pmin = p < pmin ? p : pmin;
        pmax = p > pmax ? p : pmax;
        const int64_t fs = m->cell_face_ptr[c], fe = m->cell_face_ptr[c + 1];
        if (fe - fs < 4) return fail(ctx, DGP_EMESH, "cell %lld has %lld faces", (long long)c, (long long)(fe - fs));
        if (fe - fs > kMaxFaces3D)
            return fail(ctx, DGP_EUNSUPPORTED, "cell %lld has %lld faces (at most %d)", (long long)c, (long long)(fe - fs),
                        kMaxFaces3D);
        for (int64_t k = fs; k < fe; ++k) {
            const int32_t f = m->cell_face[k];
            if (f < 0 || f >= F) return fail(ctx, DGP_EMESH, "cell %lld: face id %d out of range", (long long)c, f);
            if (m->face_cell[2 * f] != c && m->face_cell[2 * f + 1] != c)
                return fail(ctx, DGP_EMESH, "face %d is not adjacent to cell %lld", f, (long long)c);
        }
    }
    for (int64_t f = 0; f < F; ++f) {
        const int32_t l = m->face_cell[2 * f], r = m->face_cell[2 * f + 1];
        const int8_t bc = m->face_bc[f];
        if (l < 0 || l >= N || r < -1 || r >= N || r == l)
            return fail(ctx, DGP_EMESH, "face %lld: bad cells (%d, %d)", (long long)f, l, r);
        if ((r < 0) != (bc != 0) || bc < 0 || bc > 2)
            return fail(ctx, DGP_EMESH, "face %lld: boundary code %d inconsistent with cells", (long long)f, bc);
        const int32_t o = m->face_opp[f];
        if (o < 0 || o >= V) return fail(ctx, DGP_EMESH, "face %lld: opposite vertex out of range", (long long)f);
        for (int t = 0; t < 3; ++t) {
            const int32_t v = m->face_vtx[3 * f + t];
            if (v < 0 || v >= V || v == o) return fail(ctx, DGP_EMESH, "face %lld: bad vertex %d", (long long)f, v);
        }
    }
    *pmin_out = pmin;
    *pmax_out = pmax;
    return DGP_OK;
}

static dgp_status upload3d(dgp_ctx *ctx, const dgp_mesh_desc *m) {
    int pmin = 0, pmax = 0;
    dgp_status vst = validate3d(ctx, m, &pmin, &pmax);
    if (vst != DGP_OK) return vst;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int64_t N = m->n_cells, F = m->n_faces, V = m->n_vertices;
    free_mesh(ctx);
    const int64_t n_cv = m->cell_ptr[N], n_cf = m->cell_face_ptr[N];
    ctx->dim = 3;
    ctx->n_cells = N;
    ctx->n_faces = F;
    ctx->n_vertices = V;
    ctx->n_cell_vtx = n_cv;
    ctx->n_cell_face = n_cf;
    ctx->p_uniform = pmin == pmax ? pmin : -1;
    ctx->p_max = pmax;
    DevMesh &d = ctx->dm;
    d = DevMesh{};
    d.n_cells = (int32_t)N;
    d.n_faces = (int32_t)F;
    d.n_vertices = (int32_t)V;
    dgp_status st;
#define UP(arr, n, field)                                         \
    if ((st = upload(ctx, m->arr, (n), &d.field)) != DGP_OK) { \
        free_mesh(ctx);                                           \
        return st;                                                \
    }
    UP(x, V, x)
    UP(y, V, y)
    UP(z, V, z)
    UP(cell_ptr, N + 1, cell_ptr)
    UP(cell_vtx, n_cv, cell_vtx)
    UP(cell_p, N, cell_p)
    UP(cell_face_ptr, N + 1, cell_face_ptr)
    UP(cell_face, n_cf, cell_face)
    UP(face_vtx, 3 * F, face_vtx)
    UP(face_cell, 2 * F, face_cell)
    UP(face_bc, F, face_bc)
    UP(face_opp, F, face_opp)
#undef UP
    const int64_t nnzb_max = N + n_cf;
    ctx->n_tiles = (int)((N + kPrepTile3D - 1) / kPrepTile3D);
    const size_t work_bytes = layout3d(N, n_cf, ctx->n_tiles, nullptr, nullptr);
    if (hipMalloc(&ctx->row_ptr, sizeof(int64_t) * (N + 1)) != hipSuccess ||
        hipMalloc(&ctx->col_idx, sizeof(int32_t) * nnzb_max) != hipSuccess ||
        hipMalloc(&ctx->val_ptr, sizeof(int64_t) * (nnzb_max + 1)) != hipSuccess ||
        hipMalloc(&ctx->dof_ptr, sizeof(int64_t) * (N + 1)) != hipSuccess ||
        hipMalloc(&ctx->work, work_bytes) != hipSuccess) {
        free_mesh(ctx);
        return fail(ctx, DGP_ENOMEM, "device allocation failed");
    }
    HIPCHK(ctx, hipMemset(ctx->work, 0, work_bytes));
    layout3d(N, n_cf, ctx->n_tiles, static_cast<char *>(ctx->work), &ctx->prep3);
    // the assembly takes the elements along a Morton curve of their first
    // vertex: a wave's neighbours in time are neighbours in space, so the
    // faces and vertices they share are read through one XCD's L2 (the ids
    // of agglomerated polyhedra carry no spatial order); rows are still
    // written at their own ids, so the output does not depend on the order
    std::vector<int32_t> morton((size_t)N);
    {
        double lo[3] = {m->x[0], m->y[0], m->z[0]}, hi[3] = {lo[0], lo[1], lo[2]};
        for (int64_t v = 0; v < V; ++v) {
            const double q[3] = {m->x[v], m->y[v], m->z[v]};
            for (int k = 0; k < 3; ++k) {
                lo[k] = q[k] < lo[k] ? q[k] : lo[k];
                hi[k] = q[k] > hi[k] ? q[k] : hi[k];
            }
        }
        std::vector<std::pair<uint32_t, int32_t>> key((size_t)N);
        for (int64_t c = 0; c < N; ++c) {
            const int64_t v = m->cell_vtx[m->cell_ptr[c]];
            const double q[3] = {m->x[v], m->y[v], m->z[v]};
            uint32_t code = 0;
            uint32_t b[3];
            for (int k = 0; k < 3; ++k) {
                const double t = hi[k] > lo[k] ? (q[k] - lo[k]) / (hi[k] - lo[k]) : 0.0;
                b[k] = (uint32_t)std::fmin(1023.0, std::fmax(0.0, t * 1024.0));
            }
            for (int bit = 9; bit >= 0; --bit)
                for (int k = 0; k < 3; ++k) code = (code << 1) | ((b[k] >> bit) & 1u);
            key[(size_t)c] = {code, (int32_t)c};
        }
        std::stable_sort(key.begin(), key.end(),
                         [](const std::pair<uint32_t, int32_t> &a, const std::pair<uint32_t, int32_t> &b) {
                             return a.first < b.first;
                         });
        for (int64_t i = 0; i < N; ++i) morton[(size_t)i] = key[(size_t)i].second;
    }
    // then each window of 256 rows along the curve, inside the range a launch
    // gives one XCD (xcd_block), sorted by the polyhedron's number of faces,
    // largest first (stable): the four rows of a work-group cost about the
    // same (a work-group holds its slot until its slowest wave ends), and a
    // window's rows still run close together in time, so the faces they share
    // are read once through the XCD's L2.  Measured on 32,768 agglomerated
    // polyhedra: 2.59 -> 2.34 ms FP32, 4.49 -> 3.90 ms FP64, face-kernel reads
    // +8%; sorting the XCD's whole range instead gave 2.22 ms but 4.4 x the reads.
    std::vector<int32_t> nfaces((size_t)N, 0);
    for (int64_t f = 0; f < F; ++f) {
        const int32_t l = m->face_cell[2 * f], r = m->face_cell[2 * f + 1];
        if (l >= 0) nfaces[(size_t)l] += 1;
        if (r >= 0 && r != l) nfaces[(size_t)r] += 1;
    }
    auto similar_blocks = [&](std::vector<int32_t> &rows, int64_t o, int64_t n) {
        const int64_t nb = (n + 3) / 4, q = nb >> 3, r = nb & 7;  // as xcd_block over nb blocks of 4 rows
        for (int64_t x = 0; x < 8; ++x) {
            const int64_t b0 = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q, bn = x < r ? q + 1 : q;
            const int64_t lo = o + std::min(4 * b0, n), hi = o + std::min(4 * (b0 + bn), n);
            for (int64_t w = lo; w < hi; w += 256)
                std::stable_sort(rows.begin() + w, rows.begin() + std::min(w + 256, hi),
                                 [&](int32_t a, int32_t b) { return nfaces[(size_t)a] > nfaces[(size_t)b]; });
        }
    };
    if (pmin == pmax) {
        similar_blocks(morton, 0, N);
        if (hipMalloc(&ctx->rows_3d, sizeof(int32_t) * (size_t)N) != hipSuccess) {
            free_mesh(ctx);
            return fail(ctx, DGP_ENOMEM, "row order");
        }
        HIPCHK(ctx, hipMemcpy(ctx->rows_3d, morton.data(), sizeof(int32_t) * (size_t)N, hipMemcpyHostToDevice));
    } else {
        std::vector<int32_t> rows((size_t)N);
        int64_t cnt[kMaxP + 2] = {};
        for (int64_t c = 0; c < N; ++c) cnt[m->cell_p[c] + 1] += 1;
        for (int p = 1; p <= kMaxP + 1; ++p) cnt[p] += cnt[p - 1];
        for (int p = 0; p <= kMaxP + 1; ++p) ctx->rows_off[p] = cnt[p];
        // each degree's rows along the curve too
        for (int64_t i = 0; i < N; ++i) {
            const int32_t c = morton[(size_t)i];
            rows[(size_t)cnt[m->cell_p[c]]++] = c;
        }
        for (int p = 0; p <= kMaxP; ++p) similar_blocks(rows, ctx->rows_off[p], ctx->rows_off[p + 1] - ctx->rows_off[p]);
        if (hipMalloc(&ctx->rows_by_p, sizeof(int32_t) * (size_t)N) != hipSuccess) {
            free_mesh(ctx);
            return fail(ctx, DGP_ENOMEM, "row groups");
        }
        HIPCHK(ctx, hipMemcpy(ctx->rows_by_p, rows.data(), sizeof(int32_t) * (size_t)N, hipMemcpyHostToDevice));
    }
    ctx->has_mesh = true;
    return DGP_OK;
}

static DevProblem neutral_problem() {
    DevProblem d{};
    d.a0 = 1.0;
    d.c_sigma = 10.0;
    return d;
}

static dgp_status enqueue_step(dgp_ctx *ctx, const DevProblem &dp, int precision, int rule_mode, int values,
                               int write_pattern, void *vals, void *rhs, hipStream_t st, bool timed);

// Steps that assemble values on a small 2D mesh launch no scan kernel: each
// row of the assembly sums the tile sums before its tile.  Pattern-only steps
// scan, since the host reads the totals.
static bool inline_tiles(const dgp_ctx *ctx, int values) {
    return ctx->dim == 2 && values && ctx->n_tiles <= kInlineTiles;
}

static void launch_prep_any(dgp_ctx *ctx, const DevProblem &dp, hipStream_t st, int values) {
    if (ctx->dim == 3)
        launch_prep3d(ctx->dm, dp, ctx->prep3, st);
    else
        launch_prep(ctx->dm, dp, ctx->prep, st, !inline_tiles(ctx, values), ctx->p_uniform);
}

dgp_status dgp_pattern(dgp_ctx *ctx, dgp_pattern_info *out) {
    if (!ctx || !out) return DGP_EINVAL;
    if (!ctx->has_mesh) return fail(ctx, DGP_ESTATE, "dgp_pattern before dgp_mesh_upload");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    free_pattern(ctx);
    free_graph(ctx);
    dgp_status st = enqueue_step(ctx, neutral_problem(), DGP_F64, DGP_RULE_PLAIN, 0, 1, nullptr, nullptr, ctx->stream, false);
    if (st) return st;
    int64_t tot[3];
    const int64_t *toff = ctx->dim == 3 ? ctx->prep3.tile_off : ctx->prep.tile_off;
    HIPCHK(ctx, hipMemcpyAsync(tot, toff + 3 * ctx->n_tiles, sizeof(tot), hipMemcpyDeviceToHost, ctx->stream));
    int32_t err3 = 0;
    if (ctx->dim == 3)
        HIPCHK(ctx, hipMemcpyAsync(&err3, ctx->prep3.err, sizeof(err3), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (err3)
        return fail(ctx, DGP_EUNSUPPORTED,
                    "a polyhedron exceeds the 3D kernels' limits (%d faces, %d distinct surface vertices, "
                    "%d neighbours and boundary codes)",
                    kMaxFaces3D, kMaxVtx3D, kMaxGroups3D);
    ctx->nnzb = tot[0];
    ctx->n_vals = tot[1];
    ctx->n_dofs = tot[2];
    ctx->has_pattern = true;
    out->n_rows = ctx->n_cells;
    out->nnzb = ctx->nnzb;
    out->n_vals = ctx->n_vals;
    out->n_dofs = ctx->n_dofs;
    out->row_ptr = ctx->row_ptr;
    out->col_idx = ctx->col_idx;
    out->val_ptr = ctx->val_ptr;
    out->dof_ptr = ctx->dof_ptr;
    return DGP_OK;
}

dgp_status dgp_pattern_copy(dgp_ctx *ctx, int64_t *row_ptr, int32_t *col_idx, int64_t *val_ptr, int64_t *dof_ptr) {
    if (!ctx) return DGP_EINVAL;
    if (!ctx->has_pattern) return fail(ctx, DGP_ESTATE, "dgp_pattern_copy before dgp_pattern");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    if (row_ptr) HIPCHK(ctx, hipMemcpyAsync(row_ptr, ctx->row_ptr, 8 * (ctx->n_cells + 1), k, ctx->stream));
    if (col_idx) HIPCHK(ctx, hipMemcpyAsync(col_idx, ctx->col_idx, 4 * ctx->nnzb, k, ctx->stream));
    if (val_ptr) HIPCHK(ctx, hipMemcpyAsync(val_ptr, ctx->val_ptr, 8 * (ctx->nnzb + 1), k, ctx->stream));
    if (dof_ptr) HIPCHK(ctx, hipMemcpyAsync(dof_ptr, ctx->dof_ptr, 8 * (ctx->n_cells + 1), k, ctx->stream));
    return DGP_OK;
}

static DevProblem to_dev(const dgp_problem *p) {
    DevProblem d;
    d.a0 = p->a0;
    d.a1 = p->a1;
    d.bx = p->b[0];
    d.by = p->b[1];
    d.bz = p->b[2];
    d.c = p->c;
    d.c_sigma = p->c_sigma;
    d.u_kind = p->u_kind;
    for (int i = 0; i < 10; ++i) d.u[i] = p->u_poly[i];
    d.penalty = p->penalty;
    return d;
}

static dgp_status check_assemble_args(dgp_ctx *ctx, const dgp_problem *prob, int precision, int rule_mode, void *vals,
                                      void *rhs) {
    if (!ctx || !prob || !vals || !rhs) return fail(ctx, DGP_EINVAL, "null argument");
    if (!ctx->has_pattern) return fail(ctx, DGP_ESTATE, "assembly before dgp_pattern");
    if (precision != DGP_F64 && precision != DGP_F32) return fail(ctx, DGP_EINVAL, "precision %d", precision);
    if (prob->u_kind != DGP_U_SIN && prob->u_kind != DGP_U_POLY) return fail(ctx, DGP_EINVAL, "u_kind");
    if (!(prob->c_sigma >= 0.0)) return fail(ctx, DGP_EINVAL, "c_sigma must be >= 0");
    if (prob->penalty != DGP_PEN_DIAMETER && prob->penalty != DGP_PEN_COVERING)
        return fail(ctx, DGP_EINVAL, "penalty %d", prob->penalty);
    if (prob->penalty == DGP_PEN_COVERING && ctx->dim == 3)
        return fail(ctx, DGP_EUNSUPPORTED, "the covering penalty is built for 2D meshes");
    if (rule_mode != DGP_RULE_PLAIN && rule_mode != DGP_RULE_REDUCED)
        return fail(ctx, DGP_EINVAL, "rule_mode %d", rule_mode);
    if (ctx->dim == 3) {
        if (prob->a1 != 0.0) return fail(ctx, DGP_EUNSUPPORTED, "3D meshes take a constant diffusion coefficient (a1 = 0)");
        if (rule_mode != DGP_RULE_PLAIN) return fail(ctx, DGP_EUNSUPPORTED, "reduced rules are for 2D meshes");
    }
    if (rule_mode == DGP_RULE_REDUCED) {
        if (!ctx->has_qrule) return fail(ctx, DGP_ESTATE, "reduced rules requested before dgp_qrule_build");
        if (ctx->p_max > 3) return fail(ctx, DGP_EUNSUPPORTED, "reduced rules need p <= 3");
    }
    return DGP_OK;
}

static dgp_status launch_assembly3d(dgp_ctx *ctx, const DevProblem &dp, int precision, int values, int write_pattern,
                                    void *vals, void *rhs, hipStream_t st) {
    Asm3Args a;
    a.m = ctx->dm;
    a.pr = dp;
    a.geo = ctx->prep3.geo;
    a.forder = ctx->prep3.forder;
    a.grp = ctx->prep3.grp;
    a.cnt = ctx->prep3.cnt;
    a.tile_off = ctx->prep3.tile_off;
    a.row_ptr = ctx->row_ptr;
    a.col_idx = ctx->col_idx;
    a.val_ptr = ctx->val_ptr;
    a.dof_ptr = ctx->dof_ptr;
    a.vals = vals;
    a.rhs = rhs;
    a.values = values;
    a.write_pattern = write_pattern;
    a.rows = ctx->rows_3d;
    a.n_rows = (int32_t)ctx->n_cells;
    if (ctx->p_uniform > 0) {
        if (!launch_row3d(a, precision, ctx->p_uniform, st))
            return fail(ctx, DGP_EUNSUPPORTED, "no 3D kernel for precision %d, p %d", precision, ctx->p_uniform);
    } else {
        for (int p = 1; p <= kMaxP3D; ++p) {
            const int64_t n = ctx->rows_off[p + 1] - ctx->rows_off[p];
            if (n == 0) continue;
            a.rows = ctx->rows_by_p + ctx->rows_off[p];
            a.n_rows = (int32_t)n;
            if (!launch_row3d(a, precision, p, st))
                return fail(ctx, DGP_EUNSUPPORTED, "no 3D kernel for precision %d, p %d", precision, p);
        }
    }
    return DGP_OK;
}

// The rows of degree p for launch configuration cfg: id order (uniform degree:
// all rows, no list) or, with bit 1, per XCD range most sub-triangles first.
static void row_range(const dgp_ctx *ctx, AsmArgs &a, int p, int cfg) {
    const int64_t o = ctx->rows_off[p], n = ctx->rows_off[p + 1] - o;
    if (cfg & 2)
        a.rows = ctx->rows_sub + o;
    else
        a.rows = ctx->p_uniform > 0 ? nullptr : ctx->rows_by_p + o;
    a.n_rows = (int32_t)n;
}

static dgp_status launch_assembly(dgp_ctx *ctx, const DevProblem &dp, int precision, int rule_mode, int values,
                                  int write_pattern, void *vals, void *rhs, hipStream_t st) {
    if (ctx->dim == 3) return launch_assembly3d(ctx, dp, precision, values, write_pattern, vals, rhs, st);
    AsmArgs a;
    a.m = ctx->dm;
    a.pr = dp;
    a.geo = ctx->prep.geo;
    a.nbr = ctx->prep.nbr;
    a.cnt = ctx->prep.cnt;
    a.tile_off = ctx->prep.tile_off;
    a.tile_sum = inline_tiles(ctx, values) ? reinterpret_cast<const int4 *>(ctx->prep.tile_sum) : nullptr;
    a.n_tiles = ctx->n_tiles;
    a.erec = ctx->prep.erec;
    a.pen_face = ctx->prep.pen_face;
    a.rows = nullptr;
    a.n_rows = (int32_t)ctx->n_cells;
    a.row_ptr = ctx->row_ptr;
    a.col_idx = ctx->col_idx;
    a.val_ptr = ctx->val_ptr;
    a.dof_ptr = ctx->dof_ptr;
    a.vals = vals;
    a.rhs = rhs;
    a.values = values;
    a.write_pattern = write_pattern;
    a.reduced = rule_mode == DGP_RULE_REDUCED;
    a.qr_nodes = ctx->qr_nodes;
    a.qr_w = ctx->qr_w;
    a.qr_ok = ctx->qr_ok;
    const int pi = precision == DGP_F32 ? 1 : 0;
    if (ctx->p_uniform <= 0 && ctx->fused[pi] && ctx->rows_lpt) {
        // every degree bin in one persistent launch
        a.rows = ctx->rows_lpt;
        a.n_rows = (int32_t)ctx->n_cells;
        launch_row2d_fused(a, precision, st);
        return DGP_OK;
    }
    for (int p = 1; p <= kMaxP; ++p) {
        if (ctx->p_uniform > 0 && p != ctx->p_uniform) continue;
        if (ctx->rows_off[p + 1] == ctx->rows_off[p]) continue;
        const int cfg = ctx->row_cfg[pi][p];
        row_range(ctx, a, p, cfg);
        if (!launch_row2d(a, precision, p, ctx->p_uniform <= 0, cfg & 1, st))
            return fail(ctx, DGP_EUNSUPPORTED, "no kernel for precision %d, p %d", precision, p);
    }
    return DGP_OK;
}

// One step: preparation kernels, then the assembly kernel(s) (values = 0: pattern only).
static dgp_status enqueue_step(dgp_ctx *ctx, const DevProblem &dp, int precision, int rule_mode, int values,
                               int write_pattern, void *vals, void *rhs, hipStream_t st, bool timed) {
    if (timed) HIPCHK(ctx, hipEventRecord(ctx->ev[0], st));
    launch_prep_any(ctx, dp, st, values);
    if (timed) HIPCHK(ctx, hipEventRecord(ctx->ev[1], st));
    dgp_status s = launch_assembly(ctx, dp, precision, rule_mode, values, write_pattern, vals, rhs, st);
    if (s) return s;
    if (timed) HIPCHK(ctx, hipEventRecord(ctx->ev[2], st));
    HIPCHK(ctx, hipGetLastError());
    ctx->ev_pattern = timed;
    ctx->ev_assemble = timed;
    if (values) {
        ctx->has_last = true;
        ctx->last_pr = dp;
        ctx->last_precision = precision;
        ctx->last_rule = rule_mode;
        ctx->last_vals = vals;
        ctx->last_rhs = rhs;
    }
    return DGP_OK;
}

static dgp_status enqueue_assemble(dgp_ctx *ctx, const dgp_problem *prob, int precision, int rule_mode,
                                   int write_pattern, void *vals, void *rhs, hipStream_t st, bool timed) {
    return enqueue_step(ctx, to_dev(prob), precision, rule_mode, 1, write_pattern, vals, rhs, st, timed);
}

dgp_status dgp_assemble(dgp_ctx *ctx, const dgp_problem *prob, int precision, int rule_mode, void *vals, void *rhs) {
    dgp_status st = check_assemble_args(ctx, prob, precision, rule_mode, vals, rhs);
    if (st) return st;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return enqueue_assemble(ctx, prob, precision, rule_mode, 0, vals, rhs, ctx->stream, ctx->timing);
}

dgp_status dgp_run(dgp_ctx *ctx, const dgp_problem *prob, int precision, int rule_mode, void *vals, void *rhs) {
    dgp_status st = check_assemble_args(ctx, prob, precision, rule_mode, vals, rhs);
    if (st) return st;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    return enqueue_assemble(ctx, prob, precision, rule_mode, 1, vals, rhs, ctx->stream, ctx->timing);
}

dgp_status dgp_run_static(dgp_ctx *ctx, const dgp_problem *prob, int precision, int rule_mode, void *vals,
                          void *rhs) {
    dgp_status st = check_assemble_args(ctx, prob, precision, rule_mode, vals, rhs);
    if (st) return st;
    if (!ctx->static_scratch) return fail(ctx, DGP_ESTATE, "no static scratch address for device %d", ctx->device);
    const size_t need = ctx->dim == 3 ? layout3d(ctx->n_cells, ctx->n_cell_face, ctx->n_tiles, nullptr, nullptr)
                                      : layout2d(ctx->n_cells, ctx->n_cell_vtx, ctx->n_faces, ctx->n_tiles, nullptr,
                                                 nullptr);
    if (need > (size_t)DGP_STATIC_SCRATCH_BYTES)
        return fail(ctx, DGP_EUNSUPPORTED,
                    "dgp_run_static: this mesh needs %zu bytes of scratch, the static array holds %zu", need,
                    (size_t)DGP_STATIC_SCRATCH_BYTES);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    char *base = static_cast<char *>(ctx->static_scratch);
    // the step runs with the context's preparation outputs moved into the static array
    const PrepOut own2 = ctx->prep;
    const Prep3Out own3 = ctx->prep3;
    if (ctx->dim == 3) {
        layout3d(ctx->n_cells, ctx->n_cell_face, ctx->n_tiles, base, &ctx->prep3);
        // the limit flag is only ever raised by the preparation kernel: clear the
        // previous call's value (a kernel, not a memset node, so that the call can
        // be captured into a graph)
        hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, ctx->stream, ctx->prep3.err, 1, 0);
    } else {
        layout2d(ctx->n_cells, ctx->n_cell_vtx, ctx->n_faces, ctx->n_tiles, base, &ctx->prep);
    }
    st = enqueue_assemble(ctx, prob, precision, rule_mode, 1, vals, rhs, ctx->stream, ctx->timing);
    ctx->prep = own2;
    ctx->prep3 = own3;
    // dgp_time_kernels and dgp_autotune re-launch the last step on the
    // context's own buffers, which this step did not fill
    ctx->has_last = false;
    return st;
}

dgp_status dgp_graph_capture(dgp_ctx *ctx, int what, const dgp_problem *prob, int precision, int rule_mode,
                             void *vals, void *rhs) {
    dgp_status st = check_assemble_args(ctx, prob, precision, rule_mode, vals, rhs);
    if (st) return st;
    if (what != 0 && what != 1) return fail(ctx, DGP_EINVAL, "what = %d", what);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    free_graph(ctx);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    st = enqueue_assemble(ctx, prob, precision, rule_mode, what == 0 ? 1 : 0, vals, rhs, ctx->cap_stream, false);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->cap_stream, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(ctx, DGP_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    ctx->graph = g;
    e = hipGraphInstantiate(&ctx->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        free_graph(ctx);
        return fail(ctx, DGP_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return DGP_OK;
}

dgp_status dgp_graph_launch(dgp_ctx *ctx) {
    if (!ctx) return DGP_EINVAL;
    if (!ctx->exec) return fail(ctx, DGP_ESTATE, "no captured graph");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, hipGraphLaunch(ctx->exec, ctx->stream));
    return DGP_OK;
}

dgp_status dgp_set_timing(dgp_ctx *ctx, int enable) {
    if (!ctx) return DGP_EINVAL;
    ctx->timing = enable != 0;
    return DGP_OK;
}

dgp_status dgp_time_kernels(dgp_ctx *ctx, int reps, float *prep_ms, float *assemble_ms) {
    if (!ctx || reps < 1) return DGP_EINVAL;
    if (!ctx->has_last) return fail(ctx, DGP_ESTATE, "dgp_time_kernels before an assembly");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    HIPCHK(ctx, hipEventRecord(ctx->ev[0], st));
    for (int i = 0; i < reps; ++i) launch_prep_any(ctx, ctx->last_pr, st, 1);
    HIPCHK(ctx, hipEventRecord(ctx->ev[1], st));
    for (int i = 0; i < reps; ++i) {
        dgp_status s = launch_assembly(ctx, ctx->last_pr, ctx->last_precision, ctx->last_rule, 1, 0, ctx->last_vals,
                                       ctx->last_rhs, st);
        if (s) return s;
    }
    HIPCHK(ctx, hipEventRecord(ctx->ev[2], st));
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipEventSynchronize(ctx->ev[2]));
    float a = 0.0f, b = 0.0f;
    HIPCHK(ctx, hipEventElapsedTime(&a, ctx->ev[0], ctx->ev[1]));
    HIPCHK(ctx, hipEventElapsedTime(&b, ctx->ev[1], ctx->ev[2]));
    if (prep_ms) *prep_ms = a / reps;
    if (assemble_ms) *assemble_ms = b / reps;
    ctx->ev_pattern = ctx->ev_assemble = false;
    return DGP_OK;
}

dgp_status dgp_autotune(dgp_ctx *ctx, int budget_ms, int32_t *choice) {
    if (!ctx || budget_ms < 1) return DGP_EINVAL;
    if (!ctx->has_last) return fail(ctx, DGP_ESTATE, "dgp_autotune before an assembly (it tunes the last one)");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if (ctx->dim == 2 && ctx->last_rule == DGP_RULE_PLAIN) {
        hipStream_t st = ctx->stream;
        const int pi = ctx->last_precision == DGP_F32 ? 1 : 0;
        AsmArgs a;
        a.m = ctx->dm;
        a.pr = ctx->last_pr;
        a.geo = ctx->prep.geo;
        a.nbr = ctx->prep.nbr;
        a.cnt = ctx->prep.cnt;
        a.tile_off = ctx->prep.tile_off;
        a.tile_sum = inline_tiles(ctx, 1) ? reinterpret_cast<const int4 *>(ctx->prep.tile_sum) : nullptr;
        a.n_tiles = ctx->n_tiles;
        a.erec = ctx->prep.erec;
        a.pen_face = ctx->prep.pen_face;
        a.row_ptr = ctx->row_ptr;
        a.col_idx = ctx->col_idx;
        a.val_ptr = ctx->val_ptr;
        a.dof_ptr = ctx->dof_ptr;
        a.vals = ctx->last_vals;
        a.rhs = ctx->last_rhs;
        a.values = 1;
        a.write_pattern = 0;
        a.reduced = 0;
        a.qr_nodes = ctx->qr_nodes;
        a.qr_w = ctx->qr_w;
        a.qr_ok = ctx->qr_ok;
        int bins[kMaxP + 1] = {}, nbins = 0;
        for (int p = 1; p <= kMaxP; ++p) {
            const bool present = ctx->p_uniform > 0 ? p == ctx->p_uniform : ctx->rows_off[p + 1] > ctx->rows_off[p];
            if (present) bins[nbins++] = p;
        }
        // each configuration of each bin gets an equal share of the budget (at least one launch)
        const float share = (float)budget_ms / (float)(kLaunchCfgs * (nbins > 0 ? nbins : 1));
        for (int b = 0; b < nbins; ++b) {
            const int p = bins[b];
            const bool mixed = ctx->p_uniform <= 0;
            // the larger-occupancy register budget is tried only if it spills at
            // most kAltSpillMax bytes per lane more than the default (large
            // spills write tens of MB per launch; a few dwords can still win)
            const size_t spill0 = row2d_spill_bytes(a, ctx->last_precision, p, mixed, 0);
            const size_t spill1 = row2d_spill_bytes(a, ctx->last_precision, p, mixed, 1);
            float best = 0.0f;
            int best_cfg = 0;
            for (int cfg = 0; cfg < kLaunchCfgs; ++cfg) {
                const int alt = cfg & 1;
                if (alt && spill1 > spill0 + kAltSpillMax) continue;
                row_range(ctx, a, p, cfg);
                // one warm launch, then as many timed launches as fit in the share
                HIPCHK(ctx, hipEventRecord(ctx->ev[0], st));
                launch_row2d(a, ctx->last_precision, p, mixed, alt, st);
                HIPCHK(ctx, hipEventRecord(ctx->ev[1], st));
                HIPCHK(ctx, hipEventSynchronize(ctx->ev[1]));
                float one = 0.0f;
                HIPCHK(ctx, hipEventElapsedTime(&one, ctx->ev[0], ctx->ev[1]));
                const int reps = one > 0.0f ? (int)fminf(50.0f, fmaxf(1.0f, share / one)) : 1;
                HIPCHK(ctx, hipEventRecord(ctx->ev[0], st));
                for (int r = 0; r < reps; ++r) launch_row2d(a, ctx->last_precision, p, mixed, alt, st);
                HIPCHK(ctx, hipEventRecord(ctx->ev[1], st));
                HIPCHK(ctx, hipGetLastError());
                HIPCHK(ctx, hipEventSynchronize(ctx->ev[1]));
                float ms = 0.0f;
                HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
                ms /= (float)reps;
                if (cfg == 0 || ms < best) {
                    best = ms;
                    best_cfg = cfg;
                }
            }
            ctx->row_cfg[pi][p] = (int8_t)best_cfg;
        }
        if (ctx->p_uniform <= 0 && ctx->rows_lpt) {
            // the tuned per-degree launches against one persistent launch over every bin
            auto time_ms = [&](bool fused, float *out) -> dgp_status {
                for (int pass = 0; pass < 2; ++pass) {  // a warm pass, then the timed one
                    HIPCHK(ctx, hipEventRecord(ctx->ev[0], st));
                    const int reps = pass == 0 ? 1 : 5;
                    for (int r = 0; r < reps; ++r) {
                        if (fused) {
                            a.rows = ctx->rows_lpt;
                            a.n_rows = (int32_t)ctx->n_cells;
                            launch_row2d_fused(a, ctx->last_precision, st);
                        } else {
                            for (int b = 0; b < nbins; ++b) {
                                const int cfg = ctx->row_cfg[pi][bins[b]];
                                row_range(ctx, a, bins[b], cfg);
                                launch_row2d(a, ctx->last_precision, bins[b], true, cfg & 1, st);
                            }
                        }
                    }
                    HIPCHK(ctx, hipEventRecord(ctx->ev[1], st));
                    HIPCHK(ctx, hipGetLastError());
                    HIPCHK(ctx, hipEventSynchronize(ctx->ev[1]));
                    float ms = 0.0f;
                    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->ev[0], ctx->ev[1]));
                    *out = ms / (float)reps;
                }
                return DGP_OK;
            };
            float t_sep = 0.0f, t_one = 0.0f;
            dgp_status e1 = time_ms(false, &t_sep);
            if (e1) return e1;
            dgp_status e2 = time_ms(true, &t_one);
            if (e2) return e2;
            ctx->fused[pi] = t_one < t_sep ? 1 : 0;
        }
        ctx->ev_pattern = ctx->ev_assemble = false;
    }
    if (choice) {
        for (int q = 0; q < 2; ++q)
            for (int p = 0; p <= kMaxP; ++p) choice[q * (kMaxP + 1) + p] = ctx->row_cfg[q][p];
        // entry 0 of each precision: 1 if mixed-degree meshes take one launch over all bins
        for (int q = 0; q < 2; ++q) choice[q * (kMaxP + 1)] = ctx->fused[q];
    }
    return DGP_OK;
}


dgp_status dgp_set_launch(dgp_ctx *ctx, int precision, int p, int cfg) {
    if (!ctx) return DGP_EINVAL;
    if (precision != DGP_F64 && precision != DGP_F32) return fail(ctx, DGP_EINVAL, "precision %d", precision);
    if (p == 0) {
        // mixed-degree meshes: one persistent launch over all bins (1) or one per degree (0)
        if (cfg != 0 && cfg != 1) return fail(ctx, DGP_EINVAL, "single-launch setting %d (0 or 1)", cfg);
        ctx->fused[precision == DGP_F32 ? 1 : 0] = (int8_t)cfg;
        return DGP_OK;
    }
    if (p < 1 || p > kMaxP) return fail(ctx, DGP_EUNSUPPORTED, "p = %d outside 1..%d", p, kMaxP);
    if (cfg < 0 || cfg >= kLaunchCfgs) return fail(ctx, DGP_EINVAL, "launch configuration %d outside 0..%d", cfg, kLaunchCfgs - 1);
    ctx->row_cfg[precision == DGP_F32 ? 1 : 0][p] = (int8_t)cfg;
    return DGP_OK;
}

dgp_status dgp_kernel_ms(dgp_ctx *ctx, const char *name, float *ms) {
    if (!ctx || !name || !ms) return DGP_EINVAL;
    int a, b;
    if (!strcmp(name, "prep") && ctx->ev_pattern) {
        a = 0;
        b = 1;
    } else if (!strcmp(name, "assemble") && ctx->ev_assemble) {
        a = 1;
        b = 2;
    } else {
        return fail(ctx, DGP_ESTATE, "no timing recorded for '%s'", name);
    }
    HIPCHK(ctx, hipEventSynchronize(ctx->ev[2]));
    HIPCHK(ctx, hipEventElapsedTime(ms, ctx->ev[a], ctx->ev[b]));
    return DGP_OK;
}

}  // extern "C"
