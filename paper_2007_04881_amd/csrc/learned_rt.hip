// Host runtime of the reduced volume rules: network parameters, per-element
// rule construction (features and moments, network, damped Gauss-Newton,
// acceptance),
// the training loop, and the single-step hooks used by the tests.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "ctx.h"
#include "kernels.h"

using namespace dgp;

namespace {

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    bool alloc(size_t bytes) {
        return hipMalloc(&p, bytes ? bytes : 1) == hipSuccess;
    }
    template <typename T>
    T *as() const {
        return static_cast<T *>(p);
    }
};

// splitmix64 (Steele, Lea and Flood, 2014) and Box-Muller normals, for the
// initial weights N(0, 1 / fan_in) (the output layer's scaled by 1/10); hidden
// biases start at zero, the output biases at the pre-activations of the 4 x 4
// Gauss template rule (atanh of its nodes, log of its weight products), so the
// untrained network predicts nearly the template and training refines it.
struct InitRng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return ((next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal() {
        const double u1 = uniform(), u2 = uniform();
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
    }
};

void init_params(uint64_t seed, std::vector<float> &P) {
    P.assign(kMlpParams, 0.0f);
    InitRng r{seed};
    const int dims[5] = {kQrIn, kQrHidden, kQrHidden, kQrHidden, kQrOut};
    const int woff[4] = {kMlpW1, kMlpW2, kMlpW3, kMlpW4};
    for (int l = 0; l < 4; ++l) {
        const double sd = (l == 3 ? 0.1 : 1.0) * std::sqrt(1.0 / dims[l]);
        for (int i = 0; i < dims[l] * dims[l + 1]; ++i) P[woff[l] + i] = (float)(sd * r.normal());
    }
    // 4-point Gauss-Legendre on [-1, 1]: +-sqrt(3/7 -+ (2/7) sqrt(6/5)), weights (18 +- sqrt(30)) / 36
    const double ti = std::sqrt(3.0 / 7.0 - 2.0 / 7.0 * std::sqrt(1.2)), to = std::sqrt(3.0 / 7.0 + 2.0 / 7.0 * std::sqrt(1.2));
    const double t[4] = {-to, -ti, ti, to};
    const double w[4] = {(18.0 - std::sqrt(30.0)) / 36.0, (18.0 + std::sqrt(30.0)) / 36.0, (18.0 + std::sqrt(30.0)) / 36.0,
                         (18.0 - std::sqrt(30.0)) / 36.0};
    float *b4 = P.data() + kMlpB4;
    for (int k = 0; k < kQrNodes; ++k) {
        b4[2 * k] = (float)std::atanh(t[k / 4]);
        b4[2 * k + 1] = (float)std::atanh(t[k % 4]);
        b4[2 * kQrNodes + k] = (float)std::log(w[k / 4] * w[k % 4]);
    }
}

GemmArgs gemm(const float *A, int64_t sam, int64_t sak, const float *B, int64_t sbk, int64_t sbn, float *C,
              int64_t ldc, int64_t M, int N, int K) {
    GemmArgs g{};
    g.A = A;
    g.sam = sam;
    g.sak = sak;
    g.B = B;
    g.sbk = sbk;
    g.sbn = sbn;
    g.C = C;
    g.ldc = ldc;
    g.M = (int)M;
    g.N = N;
    g.K = K;
    g.ksplit = 1;
    return g;
}

// weight gradients: K is the batch, M x N at most 128 x 128, so the product is
// split over K to occupy the device (partials summed in a fixed order)
constexpr int kSplitK = 32;
GemmArgs gemm_wgrad(const float *A, int64_t sak, const float *B, int64_t sbk, float *C, int64_t ldc, int M, int N,
                    int K, float *work) {
    GemmArgs g = gemm(A, 1, sak, B, sbk, 1, C, ldc, M, N, K);
    g.work = work;
    g.ksplit = K >= 64 * kSplitK ? kSplitK : (K >= 1024 ? K / 64 : 1);
    return g;
}

// Activations and gradients of one batch of at most `rows` rows.
struct Workspace {
    DevBuf buf;
    float *Z[3], *H[3], *O, *dO, *dA, *dB, *loss, *split;
    int64_t rows = 0;
    bool alloc(int64_t r) {
        rows = r;
        const size_t h = (size_t)r * kQrHidden, o = (size_t)r * kQrOut;
        const size_t sp = (size_t)kSplitK * kQrHidden * kQrHidden;
        if (!buf.alloc(sizeof(float) * (8 * h + 2 * o + (size_t)r + 64 + sp))) return false;
        float *p = buf.as<float>();
        split = p;
        p += sp;
        for (int i = 0; i < 3; ++i) {
            Z[i] = p;
            p += h;
            H[i] = p;
            p += h;
        }
        dA = p;
        p += h;
        dB = p;
        p += h;
        O = p;
        p += o;
        dO = p;
        p += o;
        loss = p;
        return true;
    }
};

// Forward and backward over rows [0, n) of x; gradients of the mean loss into
// grad (layout of the parameter blob), per-row losses into loss_rows.
void train_step(const float *P, const float *x, const double *mom, const double *area, int64_t n, Workspace &w,
                float *grad, float *loss_rows, hipStream_t st) {
    GemmArgs g;
    const float *in[4] = {x, w.H[0], w.H[1], w.H[2]};
    const int kin[4] = {kQrIn, kQrHidden, kQrHidden, kQrHidden};
    const int wo[4] = {kMlpW1, kMlpW2, kMlpW3, kMlpW4}, bo[4] = {kMlpB1, kMlpB2, kMlpB3, kMlpB4};
    for (int l = 0; l < 3; ++l) {
        g = gemm(in[l], kin[l], 1, P + wo[l], kQrHidden, 1, w.H[l], kQrHidden, n, kQrHidden, kin[l]);
        g.bias = P + bo[l];
        g.act = 1;
        g.Zout = w.Z[l];
        launch_gemm(g, st);
    }
    g = gemm(w.H[2], kQrHidden, 1, P + kMlpW4, kQrOut, 1, w.O, kQrOut, n, kQrOut, kQrHidden);
    g.bias = P + kMlpB4;
    launch_gemm(g, st);
    launch_loss_grad(w.O, mom, area, n, n, w.dO, loss_rows, st);
    // output layer
    launch_gemm(gemm_wgrad(w.H[2], kQrHidden, w.dO, kQrOut, grad + kMlpW4, kQrOut, kQrHidden, kQrOut, (int)n, w.split),
                st);
    launch_colsum(w.dO, n, kQrOut, grad + kMlpB4, st);
    g = gemm(w.dO, kQrOut, 1, P + kMlpW4, 1, kQrOut, w.dA, kQrHidden, n, kQrHidden, kQrOut);
    g.act = 2;
    g.Z = w.Z[2];
    launch_gemm(g, st);
    // hidden layers 3, 2, 1: dA holds dL/dZ_l on entry
    float *dz = w.dA, *dn = w.dB;
    for (int l = 2; l >= 0; --l) {
        launch_gemm(gemm_wgrad(in[l], kin[l], dz, kQrHidden, grad + wo[l], kQrHidden, kin[l], kQrHidden, (int)n, w.split),
                    st);
        launch_colsum(dz, n, kQrHidden, grad + bo[l], st);
        if (l > 0) {
            g = gemm(dz, kQrHidden, 1, P + wo[l], 1, kQrHidden, dn, kQrHidden, n, kQrHidden, kQrHidden);
            g.act = 2;
            g.Z = w.Z[l - 1];
            launch_gemm(g, st);
            float *t = dz;
            dz = dn;
            dn = t;
        }
    }
}

}  // namespace

void dgp_free_qrule(dgp_ctx *c) {
    if (c->qr_buf) (void)hipFree(c->qr_buf);
    c->qr_buf = nullptr;
    c->has_qrule = false;
    c->qr_feat = nullptr;
    c->qr_mom = c->qr_area = c->qr_nodes = c->qr_w = c->qr_res = nullptr;
    c->qr_iters = nullptr;
    c->qr_elig = c->qr_ok = nullptr;
}

extern "C" {

dgp_status dgp_mlp_load(dgp_ctx *ctx, const float *params, int64_t n_params) {
    if (!ctx || !params) return DGP_EINVAL;
    if (n_params != kMlpParams) return dgp_fail(ctx, DGP_EINVAL, "expected %d parameters, got %lld", kMlpParams,
                                                (long long)n_params);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    if (!ctx->mlp && hipMalloc(&ctx->mlp, sizeof(float) * kMlpParams) != hipSuccess)
        return dgp_fail(ctx, DGP_ENOMEM, "parameter allocation failed");
    HIPCHK(ctx, hipMemcpy(ctx->mlp, params, sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    ctx->has_mlp = true;
    return DGP_OK;
}

dgp_status dgp_qrule_build(dgp_ctx *ctx, int init, int max_iters, double tol, dgp_qrule_stats *out) {
    if (!ctx) return DGP_EINVAL;
    if (!ctx->has_mesh) return dgp_fail(ctx, DGP_ESTATE, "dgp_qrule_build before dgp_mesh_upload");
    if (!ctx->has_pattern) return dgp_fail(ctx, DGP_ESTATE, "dgp_qrule_build before dgp_pattern");
    if (ctx->dim != 2) return dgp_fail(ctx, DGP_EUNSUPPORTED, "reduced rules are built for polygons (2D meshes)");
    if (init != DGP_INIT_NETWORK && init != DGP_INIT_TEMPLATE) return dgp_fail(ctx, DGP_EINVAL, "init = %d", init);
    if (init == DGP_INIT_NETWORK && !ctx->has_mlp)
        return dgp_fail(ctx, DGP_ESTATE, "network initialisation without dgp_mlp_load or dgp_mlp_train");
    if (max_iters < 0 || max_iters > 64) return dgp_fail(ctx, DGP_EINVAL, "max_iters = %d (0..64)", max_iters);
    if (!(tol > 0.0)) return dgp_fail(ctx, DGP_EINVAL, "tol must be > 0");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int64_t N = ctx->n_cells;
    if (!ctx->qr_buf) {
        const size_t bytes = sizeof(float) * kQrIn * N + sizeof(double) * (kQrMoments + 1 + 2 * kQrNodes + kQrNodes + 1) * N +
                             sizeof(int32_t) * N + 2 * N + 16 * 256;
        if (hipMalloc(&ctx->qr_buf, bytes) != hipSuccess) return dgp_fail(ctx, DGP_ENOMEM, "rule buffers");
        char *p = static_cast<char *>(ctx->qr_buf);
        auto carve = [&](size_t b) {
            char *q = p;
            p += (b + 255) & ~size_t(255);
            return q;
        };
        ctx->qr_mom = reinterpret_cast<double *>(carve(sizeof(double) * kQrMoments * N));
        ctx->qr_nodes = reinterpret_cast<double *>(carve(sizeof(double) * 2 * kQrNodes * N));
        ctx->qr_w = reinterpret_cast<double *>(carve(sizeof(double) * kQrNodes * N));
        ctx->qr_area = reinterpret_cast<double *>(carve(sizeof(double) * N));
        ctx->qr_res = reinterpret_cast<double *>(carve(sizeof(double) * N));
        ctx->qr_feat = reinterpret_cast<float *>(carve(sizeof(float) * kQrIn * N));
        ctx->qr_iters = reinterpret_cast<int32_t *>(carve(sizeof(int32_t) * N));
        ctx->qr_elig = reinterpret_cast<uint8_t *>(carve(N));
        ctx->qr_ok = reinterpret_cast<uint8_t *>(carve(N));
    }
    ctx->has_qrule = false;
    hipStream_t st = ctx->stream;
    hipEvent_t ev[4];
    for (auto &e : ev) HIPCHK(ctx, hipEventCreate(&e));
    HIPCHK(ctx, hipEventRecord(ev[0], st));
    // element geometry (the bounding boxes) comes from the preparation kernel
    DevProblem neutral{};
    neutral.a0 = 1.0;
    neutral.c_sigma = 10.0;
    launch_prep(ctx->dm, neutral, ctx->prep, st, true, ctx->p_uniform);
    launch_cell_poly(ctx->dm, ctx->prep.geo, ctx->qr_feat, ctx->qr_mom, ctx->qr_area, ctx->qr_elig, st);
    HIPCHK(ctx, hipEventRecord(ev[1], st));
    int64_t n_start_net = 0, n_retried = 0, n_retry_ok = 0;
    if (init == DGP_INIT_NETWORK) {
        // the network's rule and the template's, each element starting from the one
        // of smaller moment residual and refined for at most 3/4 of max_iters
        // steps; elements that this first attempt leaves unaccepted are refined
        // again from the template with the full max_iters (their steps add up)
        DevBuf act, tmp;
        if (!act.alloc(sizeof(float) * (size_t)N * (2 * kQrHidden + kQrOut)) ||
            !tmp.alloc((sizeof(double) * (3 * kQrNodes + 3) + sizeof(int32_t) + 4) * (size_t)N + 4 * 256))
            return dgp_fail(ctx, DGP_ENOMEM, "network activations and rule scratch");
        float *h1 = act.as<float>(), *h2 = h1 + (size_t)N * kQrHidden, *o = h2 + (size_t)N * kQrHidden;
        double *nodes_t = tmp.as<double>(), *w_t = nodes_t + (size_t)N * 2 * kQrNodes, *res_a = w_t + (size_t)N * kQrNodes;
        double *res_b = res_a + N, *res2 = res_b + N;
        int32_t *it2 = reinterpret_cast<int32_t *>(res2 + N);
        uint8_t *start_tmpl = reinterpret_cast<uint8_t *>(it2 + N), *mask = start_tmpl + N, *acc_a = mask + N,
                *acc_b = acc_a + N;
        mlp_forward(ctx->mlp, ctx->qr_feat, N, h1, h2, o, st);
        launch_rule_init((int)N, o, ctx->qr_area, ctx->qr_nodes, ctx->qr_w, st);
        launch_rule_init((int)N, nullptr, ctx->qr_area, nodes_t, w_t, st);
        // initial residuals (no refinement step)
        launch_refine((int)N, ctx->qr_mom, ctx->qr_area, ctx->qr_elig, ctx->qr_nodes, ctx->qr_w, acc_a, res_a, it2, 0,
                      tol, 1e-6, st);
        launch_refine((int)N, ctx->qr_mom, ctx->qr_area, ctx->qr_elig, nodes_t, w_t, acc_b, res_b, it2, 0, tol, 1e-6,
                      st);
        launch_rule_pick((int)N, res_a, res_b, ctx->qr_nodes, ctx->qr_w, nodes_t, w_t, start_tmpl, st);
        HIPCHK(ctx, hipEventRecord(ev[2], st));
        const int first_iters = max_iters * 3 / 4 > 0 ? max_iters * 3 / 4 : max_iters;
        launch_refine((int)N, ctx->qr_mom, ctx->qr_area, ctx->qr_elig, ctx->qr_nodes, ctx->qr_w, ctx->qr_ok,
                      ctx->qr_res, ctx->qr_iters, first_iters, tol, 1e-6, st);
        launch_rule_retry_mask((int)N, ctx->qr_elig, ctx->qr_ok, start_tmpl, mask, st);
        launch_rule_init((int)N, nullptr, ctx->qr_area, nodes_t, w_t, st);
        launch_refine((int)N, ctx->qr_mom, ctx->qr_area, mask, nodes_t, w_t, acc_b, res2, it2, max_iters, tol, 1e-6, st);
        launch_rule_merge((int)N, mask, acc_b, res2, it2, nodes_t, w_t, ctx->qr_nodes, ctx->qr_w, ctx->qr_ok,
                          ctx->qr_res, ctx->qr_iters, st);
        HIPCHK(ctx, hipEventRecord(ev[3], st));
        HIPCHK(ctx, hipStreamSynchronize(st));  // the scratch is freed on return
        std::vector<uint8_t> st_t(N), mk(N), ok2(N), el(N);
        HIPCHK(ctx, hipMemcpy(st_t.data(), start_tmpl, N, hipMemcpyDeviceToHost));
        HIPCHK(ctx, hipMemcpy(mk.data(), mask, N, hipMemcpyDeviceToHost));
        HIPCHK(ctx, hipMemcpy(ok2.data(), acc_b, N, hipMemcpyDeviceToHost));
        HIPCHK(ctx, hipMemcpy(el.data(), ctx->qr_elig, N, hipMemcpyDeviceToHost));
        for (int64_t c = 0; c < N; ++c) {
            n_start_net += el[c] && !st_t[c];
            n_retried += mk[c];
            n_retry_ok += mk[c] && ok2[c];
        }
    } else {
        launch_rule_init((int)N, nullptr, ctx->qr_area, ctx->qr_nodes, ctx->qr_w, st);
        HIPCHK(ctx, hipEventRecord(ev[2], st));
        launch_refine((int)N, ctx->qr_mom, ctx->qr_area, ctx->qr_elig, ctx->qr_nodes, ctx->qr_w, ctx->qr_ok,
                      ctx->qr_res, ctx->qr_iters, max_iters, tol, 1e-6, st);
        HIPCHK(ctx, hipEventRecord(ev[3], st));
    }
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(st));
    if (out) {
        std::memset(out, 0, sizeof(*out));
        float ms[3];
        for (int i = 0; i < 3; ++i) HIPCHK(ctx, hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]));
        out->ms_features = ms[0];
        out->ms_network = ms[1];
        out->ms_refine = ms[2];
        std::vector<uint8_t> ok(N), el(N);
        std::vector<int32_t> it(N);
        std::vector<double> res(N);
        HIPCHK(ctx, hipMemcpy(ok.data(), ctx->qr_ok, N, hipMemcpyDeviceToHost));
        HIPCHK(ctx, hipMemcpy(el.data(), ctx->qr_elig, N, hipMemcpyDeviceToHost));
        HIPCHK(ctx, hipMemcpy(it.data(), ctx->qr_iters, sizeof(int32_t) * N, hipMemcpyDeviceToHost));
        HIPCHK(ctx, hipMemcpy(res.data(), ctx->qr_res, sizeof(double) * N, hipMemcpyDeviceToHost));
        out->n_cells = N;
        out->n_start_network = n_start_net;
        out->n_retried = n_retried;
        out->n_retry_accepted = n_retry_ok;
        for (int64_t c = 0; c < N; ++c) {
            out->n_eligible += el[c];
            if (ok[c]) {
                out->n_accepted += 1;
                out->iters_hist[it[c] < 15 ? it[c] : 15] += 1;
                out->max_residual_accepted = std::fmax(out->max_residual_accepted, res[c]);
            }
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    ctx->has_qrule = true;
    return DGP_OK;
}

dgp_status dgp_qrule_get(dgp_ctx *ctx, double *nodes, double *weights, uint8_t *accepted, double *residual,
                         int32_t *iters) {
    if (!ctx) return DGP_EINVAL;
    if (!ctx->has_qrule) return dgp_fail(ctx, DGP_ESTATE, "dgp_qrule_get before dgp_qrule_build");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int64_t N = ctx->n_cells;
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    if (nodes) HIPCHK(ctx, hipMemcpyAsync(nodes, ctx->qr_nodes, sizeof(double) * 2 * kQrNodes * N, k, ctx->stream));
    if (weights) HIPCHK(ctx, hipMemcpyAsync(weights, ctx->qr_w, sizeof(double) * kQrNodes * N, k, ctx->stream));
    if (accepted) HIPCHK(ctx, hipMemcpyAsync(accepted, ctx->qr_ok, N, k, ctx->stream));
    if (residual) HIPCHK(ctx, hipMemcpyAsync(residual, ctx->qr_res, sizeof(double) * N, k, ctx->stream));
    if (iters) HIPCHK(ctx, hipMemcpyAsync(iters, ctx->qr_iters, sizeof(int32_t) * N, k, ctx->stream));
    return DGP_OK;
}

dgp_status dgp_qrule_cell_data(dgp_ctx *ctx, float *feat, double *moments, double *area) {
    if (!ctx) return DGP_EINVAL;
    if (!ctx->has_qrule) return dgp_fail(ctx, DGP_ESTATE, "dgp_qrule_cell_data before dgp_qrule_build");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const int64_t N = ctx->n_cells;
    const hipMemcpyKind k = hipMemcpyDeviceToDevice;
    if (feat) HIPCHK(ctx, hipMemcpyAsync(feat, ctx->qr_feat, sizeof(float) * kQrIn * N, k, ctx->stream));
    if (moments) HIPCHK(ctx, hipMemcpyAsync(moments, ctx->qr_mom, sizeof(double) * kQrMoments * N, k, ctx->stream));
    if (area) HIPCHK(ctx, hipMemcpyAsync(area, ctx->qr_area, sizeof(double) * N, k, ctx->stream));
    return DGP_OK;
}

dgp_status dgp_train_polygons(dgp_ctx *ctx, uint64_t seed, int64_t first, int64_t n, float *feat, double *feat64,
                              double *moments, double *area) {
    if (!ctx || !feat || !moments || !area) return DGP_EINVAL;
    if (n < 0 || first < 0 || first + n > ((int64_t)1 << 32))
        return dgp_fail(ctx, DGP_EINVAL, "polygon indices must lie in [0, 2^32)");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    launch_train_poly(seed, first, n, feat, feat64, moments, area, ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    return DGP_OK;
}

dgp_status dgp_mlp_forward(dgp_ctx *ctx, const float *params, const float *x, int64_t n, float *out) {
    if (!ctx || !params || !x || !out || n < 0) return DGP_EINVAL;
    if (n > INT32_MAX / kQrHidden) return dgp_fail(ctx, DGP_EINVAL, "too many rows");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    DevBuf act;
    if (!act.alloc(sizeof(float) * (size_t)n * 2 * kQrHidden)) return dgp_fail(ctx, DGP_ENOMEM, "activations");
    float *h1 = act.as<float>(), *h2 = h1 + (size_t)n * kQrHidden;
    mlp_forward(params, x, n, h1, h2, out, ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return DGP_OK;
}

dgp_status dgp_mlp_loss_grad(dgp_ctx *ctx, const float *params, const float *x, const double *moments,
                             const double *area, int64_t n, float *grad, float *loss_sum) {
    if (!ctx || !params || !x || !moments || !area || !grad || !loss_sum || n <= 0) return DGP_EINVAL;
    if (n > INT32_MAX / kQrHidden) return dgp_fail(ctx, DGP_EINVAL, "too many rows");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    Workspace w;
    if (!w.alloc(n)) return dgp_fail(ctx, DGP_ENOMEM, "workspace");
    train_step(params, x, moments, area, n, w, grad, w.loss, ctx->stream);
    launch_colsum(w.loss, n, 1, loss_sum, ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return DGP_OK;
}

dgp_status dgp_adam_step(dgp_ctx *ctx, float *params, const float *grad, float *m, float *v, int64_t n, int32_t t,
                         float lr, float beta1, float beta2, float eps) {
    if (!ctx || !params || !grad || !m || !v || n < 0 || n > INT32_MAX || t < 1) return DGP_EINVAL;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    const float c1 = 1.0f - (float)std::pow((double)beta1, t), c2 = 1.0f - (float)std::pow((double)beta2, t);
    launch_adam(params, grad, m, v, (int)n, lr, beta1, beta2, eps, c1, c2, ctx->stream);
    HIPCHK(ctx, hipGetLastError());
    return DGP_OK;
}

dgp_status dgp_mlp_train(dgp_ctx *ctx, const dgp_train_cfg *cfg, float *params_out, float *epoch_loss,
                         dgp_train_stats *stats) {
    if (!ctx || !cfg) return DGP_EINVAL;
    if (cfg->n_polygons <= 0 || cfg->n_polygons > ((int64_t)1 << 32) || cfg->epochs < 1 || cfg->batch < 1 ||
        cfg->batch > (1 << 20) || !(cfg->lr > 0.0f))
        return dgp_fail(ctx, DGP_EINVAL, "bad training configuration");
    HIPCHK(ctx, hipSetDevice(ctx->device));
    hipStream_t st = ctx->stream;
    const int64_t n = cfg->n_polygons;
    const int64_t B = cfg->batch < n ? cfg->batch : n;
    DevBuf data, prm, ws;
    if (!data.alloc((sizeof(float) * kQrIn + sizeof(double) * (kQrMoments + 1) + sizeof(float)) * (size_t)n + 1024))
        return dgp_fail(ctx, DGP_ENOMEM, "training data");
    double *mom = data.as<double>();
    double *area = mom + (size_t)kQrMoments * n;
    float *feat = reinterpret_cast<float *>(area + n);
    float *loss_rows = feat + (size_t)kQrIn * n;
    if (!prm.alloc(sizeof(float) * 4 * kMlpParams + 64)) return dgp_fail(ctx, DGP_ENOMEM, "parameters");
    float *P = prm.as<float>(), *G = P + kMlpParams, *M1 = G + kMlpParams, *M2 = M1 + kMlpParams;
    Workspace w;
    if (!w.alloc(B)) return dgp_fail(ctx, DGP_ENOMEM, "workspace");
    std::vector<float> h;
    init_params(cfg->init_seed, h);
    HIPCHK(ctx, hipMemcpy(P, h.data(), sizeof(float) * kMlpParams, hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemset(M1, 0, sizeof(float) * 2 * kMlpParams));
    const auto t0 = std::chrono::steady_clock::now();
    launch_train_poly(cfg->data_seed, 0, n, feat, nullptr, mom, area, st);
    int64_t step = 0;
    float *loss_dev = w.loss;  // scratch for the epoch's loss sum
    for (int e = 0; e < cfg->epochs; ++e) {
        for (int64_t b0 = 0; b0 < n; b0 += B) {
            const int64_t nb = (n - b0) < B ? (n - b0) : B;
            train_step(P, feat + (size_t)b0 * kQrIn, mom + (size_t)b0 * kQrMoments, area + b0, nb, w, G,
                       loss_rows + b0, st);
            ++step;
            const float c1 = 1.0f - (float)std::pow((double)cfg->beta1, (double)step);
            const float c2 = 1.0f - (float)std::pow((double)cfg->beta2, (double)step);
            launch_adam(P, G, M1, M2, kMlpParams, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, c1, c2, st);
        }
        launch_colsum(loss_rows, n, 1, loss_dev, st);
        float s = 0.0f;
        HIPCHK(ctx, hipMemcpyAsync(&s, loss_dev, sizeof(float), hipMemcpyDeviceToHost, st));
        HIPCHK(ctx, hipStreamSynchronize(st));
        if (epoch_loss) epoch_loss[e] = s / (float)n;
        if (stats) {
            if (e == 0) stats->loss_first = s / (float)n;
            stats->loss_last = s / (float)n;
        }
    }
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(st));
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (!ctx->mlp && hipMalloc(&ctx->mlp, sizeof(float) * kMlpParams) != hipSuccess)
        return dgp_fail(ctx, DGP_ENOMEM, "parameter allocation failed");
    HIPCHK(ctx, hipMemcpy(ctx->mlp, P, sizeof(float) * kMlpParams, hipMemcpyDeviceToDevice));
    ctx->has_mlp = true;
    if (params_out) HIPCHK(ctx, hipMemcpy(params_out, P, sizeof(float) * kMlpParams, hipMemcpyDeviceToHost));
    if (stats) {
        stats->ms = ms;
        stats->steps = step;
    }
    return DGP_OK;
}

}  // extern "C"
