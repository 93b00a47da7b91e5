// nyx_device.h -- device helpers for the CDNA4 (gfx950) kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nyx_types.h"

namespace nyx {

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// ------------------------------------------------------------ binning
// Fixed-bin-number level (paper: "number of bins" / grey depth, Materials and
// methods, "Feature Control and Tunability"): 1 + floor(ng (I - vmin) / D),
// clamped to ng, D = vmax - vmin; level 1 when D = 0.  ng (I - vmin) < 2^32,
// and the quotient is at most ng < 2^16, so the single-precision estimate is
// within one of the true quotient and one integer correction makes it exact.
__device__ __forceinline__ uint32_t fbn_level(uint32_t I, uint32_t vmin, uint32_t D, float rcpD,
                                              uint32_t ng) {
    if (D == 0u) return 1u;
    uint32_t num = ng * (I - vmin);
    uint32_t q = (uint32_t)((float)num * rcpD);
    uint32_t qd = q * D;
    if (qd > num) q -= 1u;
    else if (num - qd >= D) q += 1u;
    uint32_t b = q + 1u;
    return b > ng ? ng : b;
}

// ------------------------------------------------------------ wave ops
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
template <class T>
__device__ __forceinline__ T wave_max(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { T u = __shfl_xor(v, o); v = u > v ? u : v; }
    return v;
}
template <class T>
__device__ __forceinline__ T wave_min(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) { T u = __shfl_xor(v, o); v = u < v ? u : v; }
    return v;
}

// Compensated (Kahan-Babuska / Neumaier) accumulator.
template <class F>
struct Comp {
    F s, c;
    __device__ __forceinline__ Comp() : s(0), c(0) {}
    __device__ __forceinline__ void add(F x) {
        F t = s + x;
        if (fabs(s) >= fabs(x)) c += (s - t) + x;
        else c += (x - t) + s;
        s = t;
    }
    __device__ __forceinline__ F value() const { return s + c; }
};

// Sum of compensated accumulators across the wave: the partial sums are
// combined with an error-free two-sum, the compensations added.
template <class F>
__device__ __forceinline__ F wave_sum_comp(Comp<F> a) {
    F s = a.s, c = a.c;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        F s2 = __shfl_xor(s, o), c2 = __shfl_xor(c, o);
        F t = s + s2;
        F bp = t - s;
        F err = (s - (t - bp)) + (s2 - bp);
        s = t;
        c = c + c2 + err;
    }
    return s + c;
}

// ------------------------------------------------------------ 128-bit
typedef unsigned __int128 u128;
typedef __int128 i128;

__device__ __forceinline__ double u128_to_double(u128 v) {
    uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
    return (double)hi * 18446744073709551616.0 + (double)lo;
}
__device__ __forceinline__ double i128_to_double(i128 v) {
    return v < 0 ? -u128_to_double((u128)(-v)) : u128_to_double((u128)v);
}

// ------------------------------------------------------------ triangles
// Compact upper-triangle index of the unordered level pair (lo <= hi), 0-based.
__device__ __forceinline__ uint32_t tri_idx(uint32_t lo, uint32_t hi) {
    return ((hi * (hi + 1u)) >> 1) + lo;
}

__device__ __forceinline__ uint32_t hash_u32(uint32_t k) {
    k ^= k >> 16;
    k *= 0x7feb352du;
    k ^= k >> 15;
    k *= 0x846ca68bu;
    k ^= k >> 16;
    return k;
}

}  // namespace nyx
