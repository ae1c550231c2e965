// Cross-lane helpers shared by the assembly kernels (wave64, gfx950).
#pragma once
#include <hip/hip_runtime.h>

namespace dgp {
namespace {

// Cross-lane moves.  DPP patterns (quad_perm xor 1 / xor 2, half-row and row
// mirrors) pair lanes inside rows of 16; v_permlane16_swap / v_permlane32_swap
// exchange whole rows / halves of the wave between two registers.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

// lo <- lo + hi of the partner half (O = 32) or row (O = 16): after the swap the
// two registers hold, on every lane, the two addends of the lane's kept half
template <int O>
__device__ __forceinline__ float swap_add(float lo, float hi) {
    const auto r = O == 32 ? __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false)
                           : __builtin_amdgcn_permlane16_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
    return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}
template <int O>
__device__ __forceinline__ double swap_add(double lo, double hi) {
    const long long a = __double_as_longlong(lo), b = __double_as_longlong(hi);
    const unsigned a0 = (unsigned)(a & 0xffffffffLL), a1 = (unsigned)(a >> 32);
    const unsigned b0 = (unsigned)(b & 0xffffffffLL), b1 = (unsigned)(b >> 32);
    const auto r0 = O == 32 ? __builtin_amdgcn_permlane32_swap(a0, b0, false, false)
                            : __builtin_amdgcn_permlane16_swap(a0, b0, false, false);
    const auto r1 = O == 32 ? __builtin_amdgcn_permlane32_swap(a1, b1, false, false)
                            : __builtin_amdgcn_permlane16_swap(a1, b1, false, false);
    const double x = __longlong_as_double(((long long)r1[0] << 32) | r0[0]);
    const double y = __longlong_as_double(((long long)r1[1] << 32) | r0[1]);
    return x + y;
}

// Reduce-scatter over the 64 lanes: on return a[0] of lane l is the sum over
// lanes of entry l.  EC = entries that may be nonzero (a[EC..] are zero).  The
// stage of order O pairs lanes that differ in bit log2(O) (and possibly lower
// bits); each keeps the half of its live entries selected by that bit.
template <typename T, int O, int EC>
struct WaveRS {
    __device__ static __forceinline__ void run(T (&a)[64], int lane) {
        constexpr int NP = O < EC ? O : EC;
        const bool up = (lane & O) != 0;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
            const T lo = a[k];
            const T hi = (k + O < EC) ? a[k + O] : T(0);
            if (O >= 16) {
                a[k] = swap_add<(O >= 16 ? O : 16)>(lo, hi);
            } else {
                const T send = up ? lo : hi;
                const T keep = up ? hi : lo;
                constexpr int CTRL = O == 8 ? kDppMirror : O == 4 ? kDppHalfMirror : O == 2 ? kDppXor2 : kDppXor1;
                a[k] = keep + dpp<CTRL>(send);
            }
        }
        WaveRS<T, O / 2, (O < EC ? O : EC)>::run(a, lane);
    }
};
template <typename T, int EC>
struct WaveRS<T, 0, EC> {
    __device__ static __forceinline__ void run(T (&)[64], int) {}
};

// sum over an aligned group of FG (4 or 8) lanes, result in every lane of the group
template <int FG, typename T>
__device__ __forceinline__ T group_sum(T v) {
    v += dpp<kDppXor1>(v);
    v += dpp<kDppXor2>(v);
    if (FG == 8) v += dpp<kDppHalfMirror>(v);
    return v;
}

// Work-groups are dealt to the 8 XCDs (each with its own L2) in turn: block b
// runs on XCD b mod 8.  This renumbering gives XCD x one contiguous range of
// the grid's work (the ranges differ in length by at most one), so spatial
// neighbours, numbered close together, are mostly read through the same L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
    const int q = nb >> 3, r = nb & 7, x = b & 7, k = b >> 3;
    return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + k;
}

// Sum and maximum of an int over the 64 lanes (DPP reductions), in every lane.
__device__ __forceinline__ int wave_sum_i(int v) { return __ockl_wfred_add_i32(v); }
__device__ __forceinline__ int wave_max_i(int v) { return __ockl_wfred_max_i32(v); }

__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Orders LDS writes of the wave before its following LDS reads by other lanes.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A wave-uniform double moved to scalar registers.
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readfirstlane((int)(b & 0xffffffffLL));
    const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

}  // namespace
}  // namespace dgp
