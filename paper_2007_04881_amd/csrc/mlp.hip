// The rule network: a 36 -> 128 -> 128 -> 128 -> 48 perceptron with SiLU
// hidden layers, in FP32 on the matrix cores, plus its training pieces
// (moment-loss gradient at the outputs, bias gradients, Adam).
//
// Products go through one tiled kernel: a 256-thread work-group computes a
// 64 x 64 tile of C, each wave a 32 x 32 quarter with v_mfma_f32_32x32x2f32,
// staging 64 x 16 slices of A and 16 x 64 slices of B in LDS.  A and B are
// addressed through two strides each, so the transposed products of the
// backward pass (H^T dZ, dZ W^T) need no copies.  Bias, SiLU and the SiLU'
// factor of the backward pass are applied on the way out.
#include "dgp_common.h"
#include "kernels.h"

namespace dgp {

namespace {

typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int TM = 64, TN = 64, TK = 16;

__device__ __forceinline__ float silu(float z) { return z / (1.0f + __expf(-z)); }
__device__ __forceinline__ float dsilu(float z) {
    const float s = 1.0f / (1.0f + __expf(-z));
    return s * (1.0f + z * (1.0f - s));
}

}  // namespace

__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
    __shared__ float As[TK][TM + 1];
    __shared__ float Bs[TK][TN + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave & 1, wn = wave >> 1;
    const int64_t m0 = (int64_t)blockIdx.x * TM;
    const int n0 = blockIdx.y * TN;
    floatx16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    const bool a_kfast = g.sak == 1, b_nfast = g.sbn == 1;
    // this work-group's K range (split-K: blockIdx.z of ksplit, in multiples of TK)
    const int kchunk = (g.K + g.ksplit * TK - 1) / (g.ksplit * TK) * TK;
    const int kbeg = blockIdx.z * kchunk, kend = min(g.K, kbeg + kchunk);
    for (int k0 = kbeg; k0 < kend; k0 += TK) {
        for (int e = tid; e < TM * TK; e += 256) {
            const int mm = a_kfast ? e / TK : e % TM, kk = a_kfast ? e % TK : e / TM;
            const int64_t gm = m0 + mm;
            const int gk = k0 + kk;
            As[kk][mm] = (gm < g.M && gk < kend) ? g.A[gm * g.sam + (int64_t)gk * g.sak] : 0.0f;
        }
        for (int e = tid; e < TK * TN; e += 256) {
            const int nn = b_nfast ? e % TN : e / TK, kk = b_nfast ? e / TN : e % TK;
            const int gn = n0 + nn, gk = k0 + kk;
            Bs[kk][nn] = (gn < g.N && gk < kend) ? g.B[(int64_t)gk * g.sbk + (int64_t)gn * g.sbn] : 0.0f;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < TK; kk += 2) {
            // A fragment: row lane % 32, k lane / 32; B fragment: k lane / 32, column lane % 32
            const float a = As[kk + (lane >> 5)][wm * 32 + (lane & 31)];
            const float b = Bs[kk + (lane >> 5)][wn * 32 + (lane & 31)];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    // accumulator r of lane l holds C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]
    const int gn = n0 + wn * 32 + (lane & 31);
    if (gn >= g.N) return;
    if (g.ksplit > 1) {
        float *part = g.work + (int64_t)blockIdx.z * g.M * g.N;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int64_t gm = m0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
            if (gm < g.M) part[gm * g.N + gn] = acc[r];
        }
        return;
    }
    const float bias = g.bias ? g.bias[gn] : 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        const int64_t gm = m0 + row;
        if (gm >= g.M) continue;
        float v = acc[r] + bias;
        if (g.act == 1) {
            if (g.Zout) g.Zout[gm * g.ldc + gn] = v;
            v = silu(v);
        } else if (g.act == 2) {
            v *= dsilu(g.Z[gm * g.ldc + gn]);
        }
        g.C[gm * g.ldc + gn] = v;
    }
}

// Split-K epilogue: C = epi(sum over the ksplit partial products, in order).
__global__ void k_splitk_sum(GemmArgs g) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)g.M * g.N) return;
    const int64_t m = e / g.N;
    const int n = (int)(e - m * g.N);
    float v = 0.0f;
    for (int z = 0; z < g.ksplit; ++z) v += g.work[(int64_t)z * g.M * g.N + e];
    if (g.bias) v += g.bias[n];
    if (g.act == 1) {
        if (g.Zout) g.Zout[m * g.ldc + n] = v;
        v = silu(v);
    } else if (g.act == 2) {
        v *= dsilu(g.Z[m * g.ldc + n]);
    }
    g.C[m * g.ldc + n] = v;
}

void launch_gemm(const GemmArgs &g0, hipStream_t st) {
    if (g0.M <= 0 || g0.N <= 0) return;
    GemmArgs g = g0;
    dim3 grid((unsigned)((g.M + TM - 1) / TM), (unsigned)((g.N + TN - 1) / TN), 1);
    if (g.ksplit < 1 || !g.work) g.ksplit = 1;
    grid.z = (unsigned)g.ksplit;
    hipLaunchKernelGGL(k_gemm, grid, dim3(256), 0, st, g);
    if (g.ksplit > 1) {
        const int64_t n = (int64_t)g.M * g.N;
        hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g);
    }
}

static GemmArgs dense(const float *x, int64_t n, int k_in, const float *W, const float *b, int n_out, float *y,
                      int act) {
    GemmArgs g{};
    g.A = x;
    g.sam = k_in;
    g.sak = 1;
    g.B = W;
    g.sbk = n_out;
    g.sbn = 1;
    g.C = y;
    g.ldc = n_out;
    g.M = (int)n;
    g.N = n_out;
    g.K = k_in;
    g.bias = b;
    g.act = act;
    return g;
}

void mlp_forward(const float *P, const float *x, int64_t n, float *h1, float *h2, float *out, hipStream_t st) {
    launch_gemm(dense(x, n, kQrIn, P + kMlpW1, P + kMlpB1, kQrHidden, h1, 1), st);
    launch_gemm(dense(h1, n, kQrHidden, P + kMlpW2, P + kMlpB2, kQrHidden, h2, 1), st);
    launch_gemm(dense(h2, n, kQrHidden, P + kMlpW3, P + kMlpB3, kQrHidden, h1, 1), st);
    launch_gemm(dense(h1, n, kQrHidden, P + kMlpW4, P + kMlpB4, kQrOut, out, 0), st);
}

// One row per thread: the rule read off the outputs, its moments against the
// polygon's, and d loss / d output by the chain rule through
// w = |P| softmax(s) and xi = tanh(t).
__global__ void __launch_bounds__(128) k_loss_grad(const float *__restrict__ out, const double *__restrict__ mom,
                                                   const double *__restrict__ parea, int64_t n, float inv_n,
                                                   float *dout, float *loss_rows) {
    const int64_t i = (int64_t)blockIdx.x * 128 + threadIdx.x;
    if (i >= n) return;
    constexpr int NN = kQrNodes, NM = kQrMoments;
    const float *z = out + i * kQrOut;
    const float A = (float)parea[i];
    float smax = -3.0e38f;
    for (int k = 0; k < NN; ++k) smax = fmaxf(smax, z[2 * NN + k]);
    float sm[NN], ssum = 0.0f;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
        sm[k] = __expf(z[2 * NN + k] - smax);
        ssum += sm[k];
    }
#pragma unroll
    for (int k = 0; k < NN; ++k) sm[k] /= ssum;
    float Q[NM];
#pragma unroll
    for (int q = 0; q < NM; ++q) Q[q] = 0.0f;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
        float Lx[7], dLx[7], Ly[7], dLy[7];
        legendre<float, 6>(tanhf(z[2 * k]), Lx, dLx);
        legendre<float, 6>(tanhf(z[2 * k + 1]), Ly, dLy);
        const float w = A * sm[k];
        int q = 0;
#pragma unroll
        for (int d = 0; d <= 6; ++d)
#pragma unroll
            for (int a = d; a >= 0; --a, ++q) Q[q] += w * Lx[a] * Ly[d - a];
    }
    float g[NM], loss = 0.0f;
    const float s2 = 1.0f / (A * A);
#pragma unroll
    for (int q = 0; q < NM; ++q) {
        const float r = Q[q] - (float)mom[i * NM + q];
        loss += r * r * s2;
        g[q] = 2.0f * r * s2 * inv_n;
    }
    loss_rows[i] = loss;
    float dsm[NN], dot = 0.0f;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
        const float tx = tanhf(z[2 * k]), ty = tanhf(z[2 * k + 1]);
        float Lx[7], dLx[7], Ly[7], dLy[7];
        legendre<float, 6>(tx, Lx, dLx);
        legendre<float, 6>(ty, Ly, dLy);
        float dw = 0.0f, dx = 0.0f, dy = 0.0f;
        int q = 0;
#pragma unroll
        for (int d = 0; d <= 6; ++d)
#pragma unroll
            for (int a = d; a >= 0; --a, ++q) {
                dw += g[q] * Lx[a] * Ly[d - a];
                dx += g[q] * dLx[a] * Ly[d - a];
                dy += g[q] * Lx[a] * dLy[d - a];
            }
        const float w = A * sm[k];
        dout[i * kQrOut + 2 * k] = w * dx * (1.0f - tx * tx);
        dout[i * kQrOut + 2 * k + 1] = w * dy * (1.0f - ty * ty);
        dsm[k] = dw * A;
        dot += dsm[k] * sm[k];
    }
#pragma unroll
    for (int k = 0; k < NN; ++k) dout[i * kQrOut + 2 * NN + k] = sm[k] * (dsm[k] - dot);
}

void launch_loss_grad(const float *out, const double *mom, const double *parea, int64_t n, int64_t n_mean, float *dout,
                      float *loss_rows, hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_loss_grad, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, out, mom, parea, n,
                       1.0f / (float)n_mean, dout, loss_rows);
}

// dst[c] = sum_r a[r][c]: one work-group per column, fixed reduction tree
__global__ void __launch_bounds__(256) k_colsum(const float *__restrict__ a, int64_t rows, int cols, float *dst) {
    __shared__ float s[256];
    const int c = blockIdx.x;
    float v = 0.0f;
    for (int64_t r = threadIdx.x; r < rows; r += 256) v += a[r * cols + c];
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) dst[c] = s[0];
}

void launch_colsum(const float *a, int64_t rows, int cols, float *dst, hipStream_t st) {
    hipLaunchKernelGGL(k_colsum, dim3(cols), dim3(256), 0, st, a, rows, cols, dst);
}

// Adam (Kingma and Ba, 2015) with bias corrections c1 = 1 - b1^t, c2 = 1 - b2^t
__global__ void k_adam(float *p, const float *__restrict__ g, float *m, float *v, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

void launch_adam(float *p, const float *g, float *m, float *v, int n, float lr, float b1, float b2, float eps,
                 float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_adam, dim3((n + 255) / 256), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
}

}  // namespace dgp
