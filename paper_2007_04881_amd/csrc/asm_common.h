// Device helpers shared by the 2D assembly kernels: reference rules by
// degree, basis evaluation on the bounding box, box factors, normalisation.
#pragma once

#include "dgp_common.h"
#include "rules_data.h"

namespace dgp {

template <typename T>
__device__ __forceinline__ T fmat(T a, T b, T c) {
    return fma(a, b, c);
}

template <int DEG>
struct Tri;
template <>
struct Tri<4> {
    static constexpr int n = DGP_TRI4_N;
    __device__ static double l(int i) { return c_tri4_l[i]; }
    __device__ static double w(int i) { return c_tri4_w[i]; }
};
template <>
struct Tri<6> {
    static constexpr int n = DGP_TRI6_N;
    __device__ static double l(int i) { return c_tri6_l[i]; }
    __device__ static double w(int i) { return c_tri6_w[i]; }
};
template <>
struct Tri<8> {
    static constexpr int n = DGP_TRI8_N;
    __device__ static double l(int i) { return c_tri8_l[i]; }
    __device__ static double w(int i) { return c_tri8_w[i]; }
};

// Basis of one element at a point, without normalisation.
template <typename T, int P>
struct Eval {
    static constexpr int NB = nb2d(P);
    T v[NB], g0[NB], g1[NB];  // P_a P_b, dP_a/dxi P_b, P_a dP_b/deta
    __device__ __forceinline__ void at(T xi, T eta) {
        T Lx[P + 1], dLx[P + 1], Ly[P + 1], dLy[P + 1];
        legendre<T, P>(xi, Lx, dLx);
        legendre<T, P>(eta, Ly, dLy);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            v[i] = Lx[exp_a(i)] * Ly[exp_b(i)];
            g0[i] = dLx[exp_a(i)] * Ly[exp_b(i)];
            g1[i] = Lx[exp_a(i)] * dLy[exp_b(i)];
        }
    }
};

struct Box {
    double mx, my, cx, cy;  // centre and chain factors 2/h of the bounding box
};

__device__ __forceinline__ Box box_of(const CellGeo &g) {
    Box b;
    b.mx = 0.5 * (g.lox + g.hix);
    b.my = 0.5 * (g.loy + g.hiy);
    b.cx = 2.0 * g.ihx;  // = 2 / (hix - lox) exactly (scaling by 2 commutes with rounding)
    b.cy = 2.0 * g.ihy;
    return b;
}

// sqrt(2a + 1): the normalisation of the one-dimensional Legendre factor of degree a
constexpr double kSqrt2a1[kMaxP + 1] = {1.0, 1.7320508075688772, 2.23606797749979, 2.6457513110645907, 3.0};

// sqrt((2a+1)(2b+1)) of basis function i: its normalisation times sqrt(|B|)
// the same as compile-time constants (for unrolled indices)
constexpr double kNorm[15] = {1.0, 1.7320508075688772, 1.7320508075688772, 2.23606797749979, 3.0,
                              2.23606797749979, 2.6457513110645907, 3.872983346207417, 3.872983346207417,
                              2.6457513110645907, 3.0, 4.58257569495584, 5.0, 4.58257569495584, 3.0};
static __constant__ double c_norm[15] = {1.0, 1.7320508075688772, 1.7320508075688772, 2.23606797749979, 3.0,
                                  2.23606797749979, 2.6457513110645907, 3.872983346207417, 3.872983346207417,
                                  2.6457513110645907, 3.0, 4.58257569495584, 5.0, 4.58257569495584, 3.0};

}  // namespace dgp
