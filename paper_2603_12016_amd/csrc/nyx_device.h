// nyx_device.h -- device helpers for the CDNA4 (gfx950) kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nyx_types.h"

namespace nyx {

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// Load through a global-address-space view of a device pointer: compiles to
// global_load (SGPR base + VGPR offset where possible) instead of the flat
// form, which also waits on the LDS counter.
template <class T>
__device__ __forceinline__ T ldg(const T *p, uint32_t i) {
    return ((const __attribute__((address_space(1))) T *)p)[i];
}

// Element at byte offset `off` (< 2^32) from a wave-uniform pointer p: the
// global_load form with the base in SGPRs and a 32-bit VGPR offset, so the
// lane's address costs no 64-bit arithmetic.
template <class T>
__device__ __forceinline__ T ldb(const T *p, uint32_t off) {
    return *(const __attribute__((address_space(1))) T *)((const __attribute__((address_space(1))) char *)p + off);
}

// ------------------------------------------------------------ binning
// Fixed-bin-number level (paper: "number of bins" / grey depth, Materials and
// methods, "Feature Control and Tunability"): 1 + floor(ng (I - vmin) / D),
// clamped to ng, D = vmax - vmin; level 1 when D = 0.  ng (I - vmin) < 2^32,
// and the quotient is at most ng < 2^16, so the single-precision estimate is
// within one of the true quotient and one integer correction makes it exact.
__device__ __forceinline__ uint32_t fbn_level(uint32_t I, uint32_t vmin, uint32_t D, float rcpD,
                                              uint32_t ng) {
    if (D == 0u) return 1u;
    // 16-bit operands: 24-bit multiplies (full rate) are exact here
    uint32_t num = __umul24(ng, I - vmin);
    uint32_t q = (uint32_t)((float)num * rcpD);
    uint32_t qd = __umul24(q, D);
    if (qd > num) q -= 1u;
    else if (num - qd >= D) q += 1u;
    uint32_t b = q + 1u;
    return b > ng ? ng : b;
}

// ------------------------------------------------------------ wave ops
// Wave-wide reductions with DPP: four in-row steps (quad_perm [1,0,3,2],
// quad_perm [2,3,0,1], row_half_mirror, row_mirror) leave every lane of each
// 16-lane row holding its row's total; the four row totals are then combined
// from lanes 0, 16, 32 and 48 with readlane.  The result is wave-uniform.
constexpr int kDppQuad1032 = 0xB1;
constexpr int kDppQuad2301 = 0x4E;
constexpr int kDppRowHalfMirror = 0x141;
constexpr int kDppRowMirror = 0x140;

template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
    // bound_ctrl: a lane whose source is outside the wave reads 0 (no register
    // has to hold an "old" value)
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, true);
}

template <int CTRL, class T>
__device__ __forceinline__ T dpp_move(T v) {
    static_assert(sizeof(T) == 4 || sizeof(T) == 8, "32/64-bit only");
    if constexpr (sizeof(T) == 4) {
        uint32_t u = __builtin_bit_cast(uint32_t, v);
        return __builtin_bit_cast(T, dpp32<CTRL>(u));
    } else {
        uint64_t u = __builtin_bit_cast(uint64_t, v);
        uint32_t lo = dpp32<CTRL>((uint32_t)u), hi = dpp32<CTRL>((uint32_t)(u >> 32));
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}

template <class T>
__device__ __forceinline__ T readlane_(T v, int l) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, (uint32_t)__builtin_amdgcn_readlane((int)__builtin_bit_cast(uint32_t, v), l));
    } else {
        uint64_t u = __builtin_bit_cast(uint64_t, v);
        uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
        uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
        return __builtin_bit_cast(T, ((uint64_t)hi << 32) | lo);
    }
}

// Row (16-lane) reduction: every lane ends with its row's combination.
template <class T, class Op>
__device__ __forceinline__ T row_reduce(T v, Op op) {
    v = op(v, dpp_move<kDppQuad1032>(v));
    v = op(v, dpp_move<kDppQuad2301>(v));
    v = op(v, dpp_move<kDppRowHalfMirror>(v));
    v = op(v, dpp_move<kDppRowMirror>(v));
    return v;
}

template <class T, class Op>
__device__ __forceinline__ T wave_reduce(T v, Op op) {
    v = row_reduce(v, op);
    return op(op(readlane_(v, 0), readlane_(v, 16)), op(readlane_(v, 32), readlane_(v, 48)));
}

// Each 16-bit half of w clamped to 1 (packed integer min): bit 0 and bit 16
// of the result say whether the low and high halves are nonzero.
__device__ __forceinline__ uint32_t nz_halves(uint32_t w) {
    uint32_t r;
    asm("v_pk_min_u16 %0, %1, %2" : "=v"(r) : "v"(w), "v"(0x00010001u));
    return r;
}

// Inclusive prefix sums by DPP: within each 16-lane row (row_shr 1, 2, 4, 8
// with zero fill), then across rows (row_bcast 15 into rows 1 and 3,
// row_bcast 31 into rows 2 and 3).
template <int CTRL, int ROWS, bool BOUND>
__device__ __forceinline__ uint32_t dpp_add(uint32_t v) {
    return v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF, BOUND);
}
__device__ __forceinline__ uint32_t row_incl_scan(uint32_t x) {
    x = dpp_add<0x111, 0xF, true>(x);
    x = dpp_add<0x112, 0xF, true>(x);
    x = dpp_add<0x114, 0xF, true>(x);
    x = dpp_add<0x118, 0xF, true>(x);
    return x;
}
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    x = row_incl_scan(x);
    x = dpp_add<0x142, 0xA, false>(x);
    x = dpp_add<0x143, 0xC, false>(x);
    return x;
}

// Batched row reduction of kSumSlots doubles by recursive halving.  Each of
// four exchange steps (row_mirror, row_half_mirror, quad_perm [2,3,0,1],
// quad_perm [1,0,3,2]) pairs lanes that hold the same set of slots; one keeps
// the lower half of the set and its partner the upper half, each adding the
// partner's copy of the half it keeps.  Afterwards the lane of row-rank r
// holds the row total of slot r: 15 exchanges instead of 16 x 4.
template <int CTRL, int N>
__device__ __forceinline__ void halve_step(double *v, bool keep_low) {
#pragma unroll
    for (int j = 0; j < N; ++j) {
        const double send = keep_low ? v[N + j] : v[j];
        const double mine = keep_low ? v[j] : v[N + j];
        v[j] = mine + dpp_move<CTRL>(send);
    }
}

__device__ __forceinline__ double row_reduce_slots(double (&v)[kSumSlots]) {
    static_assert(kSumSlots == 16, "four halving steps");
    const int r = lane() & 15;
    halve_step<kDppRowMirror, 8>(v, r < 8);
    halve_step<kDppRowHalfMirror, 4>(v, (r & 4) == 0);
    halve_step<kDppQuad2301, 2>(v, (r & 2) == 0);
    halve_step<kDppQuad1032, 1>(v, (r & 1) == 0);
    return v[0];
}

// Two values: one halving step (row_mirror), then plain row sums; lanes of
// row-rank < 8 end with the total of a, the others with that of b.
__device__ __forceinline__ double row_reduce_pair(double a, double b) {
    const bool lo = (lane() & 15) < 8;
    double v = (lo ? a : b) + dpp_move<kDppRowMirror>(lo ? b : a);
    v += dpp_move<kDppRowHalfMirror>(v);
    v += dpp_move<kDppQuad2301>(v);
    v += dpp_move<kDppQuad1032>(v);
    return v;
}

struct OpAdd { template <class T> __device__ __forceinline__ T operator()(T a, T b) const { return a + b; } };
struct OpMax { template <class T> __device__ __forceinline__ T operator()(T a, T b) const { return a > b ? a : b; } };
struct OpMin { template <class T> __device__ __forceinline__ T operator()(T a, T b) const { return a < b ? a : b; } };

template <class T> __device__ __forceinline__ T wave_sum(T v) { return wave_reduce(v, OpAdd()); }
template <class T> __device__ __forceinline__ T wave_max(T v) { return wave_reduce(v, OpMax()); }
template <class T> __device__ __forceinline__ T wave_min(T v) { return wave_reduce(v, OpMin()); }

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

// Sum of compensated accumulators across the wave: partial sums are combined
// with an error-free two-sum at each step, the compensations added.
template <class F>
struct CompPair { F s, c; };

template <class F>
__device__ __forceinline__ CompPair<F> comp_combine(CompPair<F> a, CompPair<F> b) {
    F t = a.s + b.s;
    F bp = t - a.s;
    F err = (a.s - (t - bp)) + (b.s - bp);
    return CompPair<F>{t, a.c + b.c + err};
}

template <int CTRL, class F>
__device__ __forceinline__ CompPair<F> dpp_move_pair(CompPair<F> v) {
    return CompPair<F>{dpp_move<CTRL>(v.s), dpp_move<CTRL>(v.c)};
}

template <class F>
__device__ __forceinline__ F wave_sum_comp(Comp<F> a) {
    CompPair<F> v{a.s, a.c};
    v = comp_combine(v, dpp_move_pair<kDppQuad1032>(v));
    v = comp_combine(v, dpp_move_pair<kDppQuad2301>(v));
    v = comp_combine(v, dpp_move_pair<kDppRowHalfMirror>(v));
    v = comp_combine(v, dpp_move_pair<kDppRowMirror>(v));
    CompPair<F> r0{readlane_(v.s, 0), readlane_(v.c, 0)}, r1{readlane_(v.s, 16), readlane_(v.c, 16)};
    CompPair<F> r2{readlane_(v.s, 32), readlane_(v.c, 32)}, r3{readlane_(v.s, 48), readlane_(v.c, 48)};
    CompPair<F> t = comp_combine(comp_combine(r0, r1), comp_combine(r2, r3));
    return t.s + t.c;
}

// ------------------------------------------------------------ block reductions
// Reduction over a work-group of NW wavefronts (every thread gets the
// result); red is LDS room for one 8-byte value per wavefront.
template <int NW, class T, class Op>
__device__ __forceinline__ T block_reduce(T v, uint64_t *red, Op op) {
    static_assert(sizeof(T) <= 8, "one 8-byte slot per wavefront");
    v = wave_reduce(v, op);
    __syncthreads();
    if (lane() == 0) reinterpret_cast<T *>(red)[threadIdx.x / kWave] = v;
    __syncthreads();
    T r = reinterpret_cast<const T *>(red)[0];
#pragma unroll
    for (int w = 1; w < NW; ++w) r = op(r, reinterpret_cast<const T *>(red)[w]);
    return r;
}

template <int NW, class T>
__device__ __forceinline__ T block_sum(T v, uint64_t *red) {
    return block_reduce<NW>(v, red, OpAdd());
}

// ------------------------------------------------------------ box walk
// Walks the voxels of a bounding box of W x H x D voxels, BS at a time:
// thread t visits f = t + k BS in x-fastest order, tracked as (column, row,
// plane) offsets without divisions after the first step.
template <uint32_t BS>
struct BoxWalk {
    uint32_t W, H, n, f, x, y, z, dq, dx;
    __device__ __forceinline__ BoxWalk(uint32_t W_, uint32_t H_, uint32_t D_) : W(W_), H(H_) {
        n = W * H * D_;
        f = threadIdx.x;
        dq = BS / W;
        dx = BS - dq * W;
        x = f % W;
        const uint32_t r = f / W;
        y = r % H;
        z = r / H;
    }
    __device__ __forceinline__ bool ok() const { return f < n; }
    __device__ __forceinline__ void next() {
        f += BS;
        x += dx;
        uint32_t adv = dq;
        if (x >= W) { x -= W; ++adv; }
        y += adv;
        if (y >= H) {
            const uint32_t k = y / H;
            z += k;
            y -= k * H;
        }
    }
};

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
// Levels are below 2^16, so the 24-bit multiply is exact.
__device__ __forceinline__ uint32_t tri_idx(uint32_t lo, uint32_t hi) {
    return (__umul24(hi, hi + 1u) >> 1) + lo;
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
