// nyx_features.h -- GLCM normalisation, marginals and the 30 features of one
// direction, computed by a cooperating group of lanes (a 16-lane DPP row, one
// wavefront, or a whole work-group) from the nonzero cells of the upper
// triangle of the symmetric co-occurrence matrix.
//
// Definitions: the GLCM rows of the paper's Supplementary Table S3 (NY column)
// with the standard IBSI formulas the paper defers to.  The arithmetic is
// arranged for exactness on integers where that is cheap:
//   T      = sum P                         (exact)
//   S1     = sum_i i R(i), S2 = sum_i i^2 R(i), S11 = sum i j P(i, j)
//   Nvar   = T S2 - S1^2,  Ncov = T S11 - S1^2   (exact, 128-bit)
//   mean = S1 / T, variance = Nvar / T^2, correlation = Ncov / Nvar,
//   sum-average = 2 S1 / T, sum-variance = cluster tendency = 2(Nvar+Ncov)/T^2,
//   contrast = (2 S2 - 2 S11) / T, difference variance from exact moments,
//   ASM = sum P^2 / T^2, maximum probability = max P / T.
// Entropies use H = log2 T - (sum n log2 n) / T over the integer counts n of
// the matrix or marginal, so every cell is visited once before T is known;
// homogeneities and inverse variance are weighted sums of the difference
// marginal divided by T.  Per-lane partial sums of floating terms are
// compensated in the accumulation precision Acc (float or double) and
// combined across lanes in double.  Cluster shade / prominence are centred
// double sums over the sum marginal.  The mutual information HX + HY - HXY is
// taken as 2 HX - JE and, when it is small (where the subtraction would lose
// the digits the information measure of correlation needs), re-summed cell
// by cell as sum p log(p / (px py)) with an exactly formed ratio.
#pragma once
#include "nyx_device.h"

namespace nyx {

// Feature columns (Table S3 order, AVEAMP left out).
enum Feat : int {
    F_ASM, F_ACOR, F_CLUPROM, F_CLUSHADE, F_CLUTEND, F_CONTRAST, F_CORR, F_DIFAVE, F_DIFENTRO,
    F_DIFVAR, F_DIS, F_ENERGY, F_ENTROPY, F_HOM1, F_HOM2, F_IDM, F_INFOMEAS1, F_INFOMEAS2,
    F_IDMN, F_ID, F_IDN, F_IV, F_JAVE, F_JE, F_JMAX, F_SUMAVE, F_SUMENT, F_JVAR, F_SUMVAR,
    F_VARIANCE
};

// ------------------------------------------------------------- groups
// Interface: rank()/size(), sync() (LDS visibility inside the group), sum/max
// (result in every lane of the group), ballot(pred) (group-local bit mask,
// bit r = rank r) and below() (mask of ranks lower than the caller's).

// Groups that are one wavefront or one 16-lane row also offer the batched
// reduction (kBatched): reduce_slots leaves the group total of slot r in the
// lane of rank r < kSumSlots, reduce_pair the totals of two values (rank 0 holds
// the first, rank 8 the second), bcast reads a lane's value into every lane.

// One wavefront.
struct WaveGrp {
    static constexpr bool kBatched = true;
    __device__ __forceinline__ int rank() const { return lane(); }
    __device__ __forceinline__ int size() const { return kWave; }
    __device__ __forceinline__ double reduce_slots(double (&v)[kSumSlots]) const {
        double s = row_reduce_slots(v);
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        return s;
    }
    __device__ __forceinline__ double reduce_pair(double a, double b) const {
        double s = row_reduce_pair(a, b);
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        return s;
    }
    __device__ __forceinline__ double bcast(double v, int r) const { return readlane_(v, r); }
    __device__ __forceinline__ uint32_t bcast_u32(uint32_t v, int r) const { return readlane_(v, r); }
    // exclusive prefix sum over the group; *total receives the group sum
    __device__ __forceinline__ uint32_t excl_scan(uint32_t n, uint32_t *total) const {
        const uint32_t x = wave_incl_scan(n);
        *total = readlane_(x, kWave - 1);
        return x - n;
    }
    __device__ __forceinline__ void sync() const {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    template <class T> __device__ __forceinline__ T sum(T v) const { return wave_sum(v); }
    template <class T> __device__ __forceinline__ T max(T v) const { return wave_max(v); }
    __device__ __forceinline__ uint64_t ballot(bool p) const { return __ballot(p); }
    __device__ __forceinline__ uint64_t below() const { return __lanemask_lt(); }
};

// The whole work-group; `scratch` is LDS room for one 8-byte value per wave.
struct BlockGrp {
    static constexpr bool kBatched = false;
    uint64_t *scratch;
    __device__ __forceinline__ int rank() const { return (int)threadIdx.x; }
    __device__ __forceinline__ int size() const { return (int)blockDim.x; }
    __device__ __forceinline__ void sync() const { __syncthreads(); }
    __device__ __forceinline__ int nw() const { return (int)(blockDim.x / kWave); }
    // Sum over the work-group of a value already reduced within each wave.
    template <class T> __device__ __forceinline__ T sum_of_waves(T v) const {
        __syncthreads();
        if (lane() == 0) reinterpret_cast<T *>(scratch)[threadIdx.x / kWave] = v;
        __syncthreads();
        T r = 0;
        for (int w = 0; w < nw(); ++w) r += reinterpret_cast<T *>(scratch)[w];
        return r;
    }
    template <class T> __device__ __forceinline__ T sum(T v) const { return sum_of_waves(wave_sum(v)); }
    template <class T> __device__ __forceinline__ T max(T v) const {
        v = wave_max(v);
        __syncthreads();
        if (lane() == 0) reinterpret_cast<T *>(scratch)[threadIdx.x / kWave] = v;
        __syncthreads();
        T r = reinterpret_cast<T *>(scratch)[0];
        for (int w = 1; w < nw(); ++w) { T u = reinterpret_cast<T *>(scratch)[w]; r = u > r ? u : r; }
        return r;
    }
};

// ------------------------------------------------------------- sources
// A source hands every nonzero cell of one direction's upper triangle to
// fn(lo, hi, c) (0-based levels lo <= hi, triangle count c), spread over the
// lanes of a group, and can leave its storage zeroed for the next item.

template <bool PACKED>
__device__ __forceinline__ uint32_t tri_count(const uint32_t *U, uint32_t i) {
    return PACKED ? (uint32_t)reinterpret_cast<const uint16_t *>(U)[i] : U[i];
}

// Inverse of tri_idx: the pair (lo, hi) of triangle index i.
__device__ __forceinline__ void tri_decode(uint32_t i, uint32_t &lo, uint32_t &hi) {
    // hardware square root: the estimate is corrected to the exact row below
    uint32_t h = (uint32_t)((__builtin_amdgcn_sqrtf(8.0f * (float)i + 1.0f) - 1.0f) * 0.5f);
    if ((__umul24(h, h + 1u) >> 1) > i) --h;
    else if ((__umul24(h + 1u, h + 2u) >> 1) <= i) ++h;
    hi = h;
    lo = i - (__umul24(h, h + 1u) >> 1);
}

// LDS triangle of one direction, visited in index order, in two levels.
// First, per block of kChunkRounds x size() 16-byte runs of the triangle
// (8 packed 16-bit or 4 32-bit counters each), every lane reads one run per
// round and the group lists the nonzero runs in index order (u16 run
// indices; in the workloads here most runs are empty).  Then each lane reads
// one listed run, the group forms the exclusive prefix of the runs'
// nonzero-cell counts, and each lane appends its nonzero cells, as u16 cell
// indices, to `buf` (room for size() * kPerRead entries).  fn runs over the
// buffered entries (count re-read from the triangle, index decoded to
// (lo, hi)) whenever the next round might not fit, and at the end: lanes stay
// busy however sparse the triangle is, and the order of every floating sum
// is fixed.  U must be 16-byte aligned and padded with zero words to a
// multiple of 4 words; cell indices must fit 16 bits (dense triangles in LDS
// always do).  The triangle may be held in `ncp` privatised copies `stride`
// words apart; every read sums them (packed 16-bit halves add without carry:
// a cell's total over the copies stays below 2^16, as for a single copy).
template <bool PACKED>
struct SrcTriScan {
    uint32_t *U;
    uint32_t tri;            // cells: ng (ng + 1) / 2, or ng^2 for a square
    uint16_t *buf;           // scan_buf_entries(kPerRead) entries: cells, then the run list
    uint32_t ncp = 1u;
    uint32_t stride = 0u;
    uint32_t sq_ng = 0u;     // > 0: a full row-major square of sq_ng x sq_ng ordered cells
    static constexpr uint32_t kPerRead = PACKED ? 8u : 4u;   // cells per 16-byte read
    // Cell i as (lo, hi): triangle row and column, or square row and column
    // (a single-precision quotient corrected by one step; i < 2^16 here).
    __device__ __forceinline__ void decode(uint32_t i, uint32_t &lo, uint32_t &hi) const {
        if (sq_ng) {
            uint32_t q = (uint32_t)((float)i * __builtin_amdgcn_rcpf((float)sq_ng));
            if (__umul24(q, sq_ng) > i) --q;
            else if (__umul24(q + 1u, sq_ng) <= i) ++q;
            lo = q;
            hi = i - __umul24(q, sq_ng);
        } else {
            tri_decode(i, lo, hi);
        }
    }
    __device__ __forceinline__ uint32_t count(uint32_t i) const {
        uint32_t c = 0;
        for (uint32_t k = 0; k < ncp; ++k)
            c += PACKED ? (uint32_t)reinterpret_cast<const uint16_t *>(U + k * stride)[i] : U[k * stride + i];
        return c;
    }
    // 16-byte run j summed over the copies.
    __device__ __forceinline__ uint4 run(uint32_t j) const {
        uint4 v = *reinterpret_cast<const uint4 *>(U + 4u * j);
        for (uint32_t k = 1; k < ncp; ++k) {
            const uint4 u = *reinterpret_cast<const uint4 *>(U + k * stride + 4u * j);
            v.x += u.x; v.y += u.y; v.z += u.z; v.w += u.w;
        }
        return v;
    }
    template <class Grp, class Fn>
    __device__ __forceinline__ void flush(const Grp &g, uint32_t n, Fn &&fn) const {
        g.sync();
        for (uint32_t e = (uint32_t)g.rank(); e < n; e += (uint32_t)g.size()) {
            const uint32_t i = buf[e];
            uint32_t lo, hi;
            decode(i, lo, hi);
            fn(lo, hi, count(i));
        }
        g.sync();
    }
    template <class Grp, class Fn>
    __device__ __forceinline__ void for_each(const Grp &g, Fn &&fn) const {
        const uint32_t gs = (uint32_t)g.size(), r = (uint32_t)g.rank();
        const uint32_t runs = ((PACKED ? (tri + 1u) >> 1 : tri) + 3u) >> 2;
        const uint32_t cap = gs * kPerRead;
        uint16_t *const list = buf + cap;   // room for gs * kChunkRounds run indices
        uint32_t held = 0;   // entries waiting in buf (group-uniform)
        for (uint32_t jb = 0; jb < runs; jb += gs * (uint32_t)kChunkRounds) {
            const uint32_t je = min(runs, jb + gs * (uint32_t)kChunkRounds);
            uint32_t nrun = 0;   // nonzero runs listed (group-uniform)
            for (uint32_t j0 = jb; j0 < je; j0 += gs) {
                const uint32_t j = j0 + r;
                bool nz = false;
                if (j < je) {
                    const uint4 v = run(j);
                    nz = (v.x | v.y | v.z | v.w) != 0u;
                }
                const uint64_t m = g.ballot(nz);
                if (nz) list[nrun + (uint32_t)__popcll(m & g.below())] = (uint16_t)j;
                nrun += (uint32_t)__popcll(m);
            }
            g.sync();
            for (uint32_t e0 = 0; e0 < nrun; e0 += gs) {
                const uint32_t e = e0 + r;
                uint4 v = make_uint4(0u, 0u, 0u, 0u);
                uint32_t j = 0u;
                if (e < nrun) {
                    j = list[e];
                    v = run(j);
                }
                // nonzero flags of the run's cells (cells past tri are zero
                // padding); packed: 0/1 in each 16-bit half
                uint32_t f[4];
                uint32_t n;
                if (PACKED) {
                    f[0] = nz_halves(v.x); f[1] = nz_halves(v.y); f[2] = nz_halves(v.z); f[3] = nz_halves(v.w);
                    const uint32_t s = f[0] + f[1] + f[2] + f[3];
                    n = (s & 0xFFFFu) + (s >> 16);
                } else {
                    f[0] = v.x != 0u; f[1] = v.y != 0u; f[2] = v.z != 0u; f[3] = v.w != 0u;
                    n = f[0] + f[1] + f[2] + f[3];
                }
                uint32_t cnt;
                const uint32_t pos = g.excl_scan(n, &cnt);
                if (held + cnt > cap) {
                    flush(g, held, fn);
                    held = 0;
                }
                uint16_t *p = buf + held + pos;
                const uint32_t i0 = PACKED ? 8u * j : 4u * j;   // first cell of the run
#pragma unroll
                for (uint32_t k = 0; k < 4u; ++k) {
                    if (PACKED) {
                        if (f[k] & 0xFFFFu) *p++ = (uint16_t)(i0 + 2u * k);
                        if (f[k] >> 16) *p++ = (uint16_t)(i0 + 2u * k + 1u);
                    } else {
                        if (f[k]) *p++ = (uint16_t)(i0 + k);
                    }
                }
                held += cnt;
            }
            g.sync();   // the run list is refilled by the next block
        }
        if (held) flush(g, held, fn);
    }
    template <class Grp>
    __device__ __forceinline__ void clear(const Grp &g) const {
        const uint32_t words = PACKED ? (tri + 1u) >> 1 : tri;
        for (uint32_t k = 0; k < ncp; ++k)
            for (uint32_t w = 4u * (uint32_t)g.rank(); w < words; w += 4u * (uint32_t)g.size())
                *reinterpret_cast<uint4 *>(U + k * stride + w) = make_uint4(0u, 0u, 0u, 0u);
    }
};

// LDS triangle plus a list of its touched cells (returning-atomic mode).
struct SrcDenseList {
    const uint32_t *list;
    uint32_t n;
    uint32_t *U;
    template <class Grp, class Fn>
    __device__ __forceinline__ void for_each(const Grp &g, Fn &&fn) const {
        for (uint32_t e = g.rank(); e < n; e += g.size()) {
            const uint32_t p = list[e];
            const uint32_t lo = p & 0xFFFFu, hi = p >> 16;
            const uint32_t c = U[tri_idx(lo, hi)];
            if (c) fn(lo, hi, c);
        }
    }
    template <class Grp>
    __device__ __forceinline__ void clear(const Grp &g) const {
        for (uint32_t e = g.rank(); e < n; e += g.size()) {
            const uint32_t p = list[e];
            U[tri_idx(p & 0xFFFFu, p >> 16)] = 0u;
        }
    }
};

// LDS hash slots listed per direction.
struct SrcHashList {
    const uint32_t *list;
    uint32_t n;
    uint32_t *keys;
    uint32_t *cnts;
    template <class Grp, class Fn>
    __device__ __forceinline__ void for_each(const Grp &g, Fn &&fn) const {
        for (uint32_t e = g.rank(); e < n; e += g.size()) {
            const uint32_t s = list[e];
            const uint32_t k = keys[s];
            const uint32_t c = cnts[s];
            if (c) fn(k & 0x1FFFu, (k >> 13) & 0x1FFFu, c);
        }
    }
    template <class Grp>
    __device__ __forceinline__ void clear(const Grp &g) const {
        for (uint32_t e = g.rank(); e < n; e += g.size()) {
            const uint32_t s = list[e];
            keys[s] = kNone;
            cnts[s] = 0u;
        }
    }
};

// Global dense square (upper triangle used) of a merged split ROI.
// Position (lo, hi) of a lane walking an ng x ng matrix from row r0 in
// row-major order with a fixed stride: one division at the start, then whole
// rows plus a remainder per step.
struct SquareWalk {
    uint32_t lo, hi, dq, dr;
    __device__ __forceinline__ SquareWalk(uint32_t ng, uint32_t r0, uint32_t start, uint32_t stride) {
        lo = start / ng;
        hi = start - lo * ng;
        lo += r0;
        dq = stride / ng;
        dr = stride - dq * ng;
    }
    __device__ __forceinline__ void next(uint32_t ng) {
        hi += dr;
        lo += dq;
        if (hi >= ng) { hi -= ng; ++lo; }
    }
};

struct SrcSquare {
    const uint64_t *G;
    uint32_t ng;
    bool all = false;        // every cell (ordered counts), not only the upper triangle
    template <class Grp, class Fn>
    __device__ __forceinline__ void for_each(const Grp &g, Fn &&fn) const {
        // flat over the square in row-major order, so every lane has a cell
        // whatever ng is next to the group size; the upper triangle unless all
        SquareWalk p(ng, 0u, (uint32_t)g.rank(), (uint32_t)g.size());
        for (uint64_t e = (uint32_t)g.rank(); p.lo < ng; e += (uint32_t)g.size(), p.next(ng)) {
            if (!all && p.hi < p.lo) continue;
            const uint64_t c = G[e];
            if (c) fn(p.lo, p.hi, (uint32_t)c);
        }
    }
    template <class Grp> __device__ __forceinline__ void clear(const Grp &) const {}
};

// Sorted COO segment of one ROI-direction; entries outside the matrix or of
// another (roi, dir) are skipped and flagged.
struct SrcCoo {
    const uint64_t *key;
    const uint64_t *cnt;
    uint32_t n;
    uint64_t prefix;         // expected roi << 38 | dir << 32
    uint32_t ng;
    uint32_t *err;
    bool ordered = false;    // cells below the diagonal are valid (ordered counts)
    template <class Grp, class Fn>
    __device__ __forceinline__ void for_each(const Grp &g, Fn &&fn) const {
        for (uint32_t e = g.rank(); e < n; e += g.size()) {
            const uint64_t k = key[e];
            const uint32_t lo = (uint32_t)(k >> 16) & 0xFFFFu, hi = (uint32_t)k & 0xFFFFu;
            const uint64_t c = cnt[e];
            if ((k & ~0xFFFFFFFFull) != prefix || (lo > hi && !ordered) || hi >= ng || lo >= ng ||
                c >= (1ull << 31)) {
                if (c) atomicOr(err, (uint32_t)E_COO_RANGE);
                continue;
            }
            if (c) fn(lo, hi, (uint32_t)c);
        }
    }
    template <class Grp> __device__ __forceinline__ void clear(const Grp &) const {}
};

// ------------------------------------------------------------- sums
// The 30 features of one direction from its reduced sums (one lane).
// y: the column-marginal sums of a non-symmetric matrix (nullptr: the matrix
// is symmetric and its column marginal is its row marginal).  Computed in
// double precision; out holds the output precision (OutT: float or double).
// xd (may be null): cluster shade and correlation in double as well, the two
// features whose directions can differ in sign, so that a direction mean
// formed from single-precision values does not lose their cancellation.
template <class OutT>
__device__ __noinline__ void finalize_dir(const DirSums &s, const DirSumsY *y, OutT *out, double *xd) {
    const uint64_t T = s.T;
    if (T == 0) {
        for (int f = 0; f < kNumFeat; ++f) out[f] = __builtin_nan("");
        if (xd) xd[0] = xd[1] = __builtin_nan("");
        return;
    }
    const uint64_t S1 = s.S1, S2 = s.S2, S11 = s.S11, Sm1 = s.Sm1;
    const uint64_t S1y = y ? y->S1y : S1, S2y = y ? y->S2y : S2;
    const double Td = (double)T, invT = 1.0 / Td, lgT = log2(Td);
    const double T2 = Td * Td;
    const u128 Tq = (u128)T;
    // T^2 var_x, T^2 var_y and T^2 cov as exact integers
    const u128 nvar = Tq * (u128)S2 - (u128)S1 * (u128)S1;
    const u128 nvary = Tq * (u128)S2y - (u128)S1y * (u128)S1y;
    const i128 ncov = (i128)(Tq * (u128)S11) - (i128)((u128)S1 * (u128)S1y);
    const u128 sm2 = (u128)S2 + (u128)S2y - 2 * (u128)S11;     // sum (i - j)^2 P
    const u128 ndv = Tq * sm2 - (u128)Sm1 * (u128)Sm1;
    // one occupied level in the row or the column marginal: the matrix is the
    // product of its marginals (correlation 0/0, mutual information 0)
    const bool single = nvar == 0 || nvary == 0;
    const double var = u128_to_double(nvar) / T2;
    // entropies H = log2 T - (sum n log2 n) / T
    const double JE = lgT - s.plp * invT;
    const double HX = lgT - s.rlr * invT;
    const double HY = y ? lgT - y->clc * invT : HX;
    const double MI = isnan(s.MI) ? HX + HY - JE : s.MI;
    out[F_ASM] = out[F_ENERGY] = (double)s.sumP2 / T2;
    out[F_ACOR] = (double)S11 / Td;
    out[F_CLUPROM] = s.CPROM;
    out[F_CLUSHADE] = s.CSHADE;
    out[F_CLUTEND] = out[F_SUMVAR] = i128_to_double((i128)nvar + (i128)nvary + 2 * ncov) / T2;
    out[F_CONTRAST] = u128_to_double(sm2) / Td;
    const double corr = single ? 1.0
                               : i128_to_double(ncov) / (y ? sqrt(u128_to_double(nvar)) * sqrt(u128_to_double(nvary))
                                                           : u128_to_double(nvar));
    out[F_CORR] = corr;
    if (xd) {
        xd[0] = s.CSHADE;
        xd[1] = corr;
    }
    out[F_DIFAVE] = out[F_DIS] = (double)Sm1 / Td;
    out[F_DIFENTRO] = lgT - s.slp * invT;
    out[F_DIFVAR] = u128_to_double(ndv) / T2;
    out[F_ENTROPY] = out[F_JE] = JE;
    out[F_HOM1] = out[F_ID] = s.hom1 * invT;
    out[F_HOM2] = out[F_IDM] = s.hom2 * invT;
    const double mi = MI > 0.0 ? MI : 0.0;
    out[F_INFOMEAS1] = single ? 0.0 : -MI / (HX > HY ? HX : HY);
    out[F_INFOMEAS2] = single ? 0.0 : sqrt(1.0 - exp(-2.0 * mi));
    out[F_IDMN] = s.idmn * invT;
    out[F_IDN] = s.idn * invT;
    out[F_IV] = s.iv * invT;
    out[F_JAVE] = (double)S1 / Td;
    out[F_JMAX] = (double)s.maxP / Td;
    out[F_SUMAVE] = ((double)S1 + (double)S1y) / Td;
    out[F_SUMENT] = lgT - s.plps * invT;
    out[F_JVAR] = out[F_VARIANCE] = var;
}

template <class F> __device__ __forceinline__ F log1p_(F x);
template <> __device__ __forceinline__ float log1p_<float>(float x) { return log1pf(x); }
template <> __device__ __forceinline__ double log1p_<double>(double x) { return log1p(x); }

template <class F>
__device__ __forceinline__ double comp_value(const Comp<F> &c) { return (double)c.s + (double)c.c; }

// Per-lane sum of floating terms.  Double precision path: compensated double
// sums.  Single precision path: the terms are formed in single precision with
// the hardware log2 and reciprocal (inputs are integers >= 1, so no denormal
// handling is needed) and summed in double, so the sum adds no error beyond
// the terms' own rounding (~1e-7 relative each).
template <class Acc> struct LaneSum;
template <> struct LaneSum<double> : Comp<double> {};
template <> struct LaneSum<float> {
    double s = 0.0;
    __device__ __forceinline__ void add(float x) { s += (double)x; }
};
__device__ __forceinline__ double comp_value(const LaneSum<float> &c) { return c.s; }

template <class Acc> __device__ __forceinline__ Acc term_log2(Acc x);
template <> __device__ __forceinline__ float term_log2<float>(float x) { return __log2f(x); }
template <> __device__ __forceinline__ double term_log2<double>(double x) { return log2(x); }
template <class Acc> __device__ __forceinline__ Acc term_div(Acc a, Acc b);
template <> __device__ __forceinline__ float term_div<float>(float a, float b) { return __fdividef(a, b); }
template <> __device__ __forceinline__ double term_div<double>(double a, double b) { return a / b; }

// Below this many bits of mutual information the difference 2 HX - JE is
// re-summed cell by cell.
template <class Acc> __device__ __forceinline__ double mi_resum_threshold();
template <> __device__ __forceinline__ double mi_resum_threshold<float>() { return 0.25; }
template <> __device__ __forceinline__ double mi_resum_threshold<double>() { return 1e-3; }

// Entries [0, n) of one or two LDS arrays, lane r0 taking r0, r0 + gs, ...
// in that order: U entries per lane are read before any is used, so their
// LDS round trips overlap (wide level ranges); fn(i, a[i]) or
// fn(i, a[i], b[i]).  The per-lane order, and so every sum, is the same for
// any U.
constexpr uint32_t kWideLevels = 256u;
template <class Src> struct is_tri_scan : std::false_type {};
template <bool P> struct is_tri_scan<SrcTriScan<P>> : std::true_type {};
template <uint32_t U, class Fn>
__device__ __forceinline__ void level_sweep(uint32_t r0, uint32_t gs, uint32_t n, const uint32_t *a, Fn &&fn) {
    for (uint32_t i0 = r0; i0 < n; i0 += U * gs) {
        uint32_t v[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) v[u] = i0 + u * gs < n ? a[i0 + u * gs] : 0u;
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) fn(i0 + u * gs, v[u]);
    }
}
template <uint32_t U, class Fn>
__device__ __forceinline__ void level_sweep(uint32_t r0, uint32_t gs, uint32_t n, const uint32_t *a,
                                            const uint32_t *b, Fn &&fn) {
    for (uint32_t i0 = r0; i0 < n; i0 += U * gs) {
        uint32_t v[U], w[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t i = i0 + u * gs;
            v[u] = i < n ? a[i] : 0u;
            w[u] = i < n ? b[i] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) fn(i0 + u * gs, v[u], w[u]);
    }
}

// Reduced sums of one direction.  R, Sp, Sm are zeroed LDS arrays of ng,
// 2 ng - 1 and ng u32 (row, sum and difference marginals of the symmetric
// matrix); they are zeroed again on return, and the source is cleared.
// *out (LDS or global) is written by the group.  ISum is the type of the
// per-lane integer sums: double where every partial and total stays below
// 2^53 (small work items; required by the batched reduction), uint64_t
// otherwise.  Returns T (0: direction empty).
template <class Acc, class ISum, class Grp, class Src>
__device__ uint64_t dir_sums(const Grp &g, const Src &src, uint32_t *R, uint32_t *Sp, uint32_t *Sm,
                             uint32_t ng, DirSums *out) {
    static_assert(!Grp::kBatched || std::is_same<ISum, double>::value, "batched sums are exact doubles");
    const int r0 = g.rank(), gs = g.size();
    // One sweep over the nonzero cells: marginals and cell terms.  A cell
    // (lo < hi) with count c stands for P(lo, hi) = P(hi, lo) = c, a diagonal
    // one for P = 2c.
    ISum sumP2 = 0;
    uint32_t maxP = 0;
    LaneSum<Acc> plp;
    src.for_each(g, [&](uint32_t lo, uint32_t hi, uint32_t c) {
        atomicAdd(&R[lo], c);
        atomicAdd(&R[hi], c);
        atomicAdd(&Sp[lo + hi], 2u * c);
        atomicAdd(&Sm[hi - lo], 2u * c);
        const bool diag = lo == hi;
        const uint32_t P = diag ? 2u * c : c;
        const ISum Pm = diag ? (ISum)P : (ISum)(2ull * P);    // P summed over both orders
        sumP2 += Pm * (ISum)P;
        maxP = P > maxP ? P : maxP;
        plp.add((Acc)Pm * term_log2<Acc>((Acc)P));
    });
    g.sync();
    // Level sweeps over the marginals (unnormalised).  T = sum R(i), and
    // S11 comes from the difference marginal: sum (i - j)^2 P = 2 S2 - 2 S11
    // for a symmetric matrix, so S11 = S2 - K2 / 2 with K2 = sum k^2 Sm(k)
    // (even, exact).  The slot of S11 carries K2 through the reduction.
    ISum Tl = 0, S1 = 0, S2 = 0, Sm1 = 0, S11 = 0;
    LaneSum<Acc> rlr, slp, hom1, hom2, idmn, idn, iv, plps;
    const Acc ngf = (Acc)ng, rng = (Acc)1 / ngf, rng2 = rng * rng;
    auto row_diff = [&](uint32_t i, uint32_t r, uint32_t s) {
        if (r) {
            const ISum lv = (ISum)(i + 1u);
            Tl += (ISum)r;
            S1 += lv * (ISum)r;
            S2 += lv * lv * (ISum)r;
            rlr.add((Acc)r * term_log2<Acc>((Acc)r));
        }
        if (s) {
            Sm1 += (ISum)i * (ISum)s;
            S11 += (ISum)(i * i) * (ISum)s;   // K2 (i < 2^13)
            const Acc sf = (Acc)s, k = (Acc)i;
            slp.add(sf * term_log2<Acc>(sf));
            hom1.add(term_div<Acc>(sf, (Acc)1 + k));
            hom2.add(term_div<Acc>(sf, (Acc)1 + k * k));
            idmn.add(term_div<Acc>(sf, (Acc)1 + (k * k) * rng2));
            idn.add(term_div<Acc>(sf, (Acc)1 + k * rng));
            if (i > 0) iv.add(term_div<Acc>(sf, k * k));
        }
    };
    auto sum_ent = [&](uint32_t, uint32_t s) {
        if (s) plps.add((Acc)s * term_log2<Acc>((Acc)s));
    };
    // (the scan sources serve the small level counts: one entry at a time)
    constexpr bool wide_ok = !is_tri_scan<Src>::value;
    const bool wide = wide_ok && ng >= kWideLevels;
    if (wide) {
        if constexpr (wide_ok) {
            level_sweep<4>(r0, gs, ng, R, Sm, row_diff);
            level_sweep<4>(r0, gs, 2u * ng - 1u, Sp, sum_ent);
        }
    } else {
        level_sweep<1>(r0, gs, ng, R, Sm, row_diff);
        level_sweep<1>(r0, gs, 2u * ng - 1u, Sp, sum_ent);
    }
    // Group totals.  Batched groups reduce the sixteen slots of DirSums at
    // once (rank r < 16 ends with slot r); the others reduce value by value.
    uint64_t T, S1t;
    double slot = 0.0, plp_t, rlr_t;
    const int rk = r0;
    uint64_t tot_u[6];
    double tot_d[10];
    if constexpr (Grp::kBatched) {
        double v[kSumSlots] = {(double)Tl, (double)S1, (double)S2, (double)Sm1, (double)S11, (double)sumP2,
                               comp_value(plp), comp_value(rlr), comp_value(slp), comp_value(plps),
                               comp_value(hom1), comp_value(hom2), comp_value(idmn), comp_value(idn),
                               comp_value(iv), 0.0};
        slot = g.reduce_slots(v);
        T = (uint64_t)g.bcast(slot, 0);
        S1t = (uint64_t)g.bcast(slot, 1);
        const double S2t = g.bcast(slot, 2);
        if (rk == 4) slot = S2t - 0.5 * slot;   // S11 = S2 - K2 / 2 (exact integers below 2^53)
        plp_t = g.bcast(slot, 6);
        rlr_t = g.bcast(slot, 7);
    } else {
        tot_u[0] = (uint64_t)g.sum(Tl); tot_u[1] = (uint64_t)g.sum(S1); tot_u[2] = (uint64_t)g.sum(S2);
        tot_u[3] = (uint64_t)g.sum(Sm1); tot_u[4] = tot_u[2] - (uint64_t)g.sum(S11) / 2u; tot_u[5] = (uint64_t)g.sum(sumP2);
        tot_d[0] = g.sum(comp_value(plp)); tot_d[1] = g.sum(comp_value(rlr)); tot_d[2] = g.sum(comp_value(slp));
        tot_d[3] = g.sum(comp_value(plps)); tot_d[4] = g.sum(comp_value(hom1)); tot_d[5] = g.sum(comp_value(hom2));
        tot_d[6] = g.sum(comp_value(idmn)); tot_d[7] = g.sum(comp_value(idn)); tot_d[8] = g.sum(comp_value(iv));
        tot_d[9] = 0.0;
        T = tot_u[0];
        S1t = tot_u[1];
        plp_t = tot_d[0];
        rlr_t = tot_d[1];
    }
    const uint32_t maxPt = g.max(maxP);
    if (T == 0) {
        g.sync();
        if (r0 == 0) out->T = 0;
        for (uint32_t i = r0; i < ng; i += gs) { R[i] = 0u; Sm[i] = 0u; }
        for (uint32_t k = r0; k < 2u * ng - 1u; k += gs) Sp[k] = 0u;
        src.clear(g);
        g.sync();
        return 0;
    }
    const double Td = (double)T, invT = 1.0 / Td;
    // Cluster shade / prominence: moments of the sum marginal about 2 mu.
    // (an exact integer over T, one rounding: a sum marginal on one value
    // gives d = 0 exactly)
    const double two_mu = (double)(2u * S1t) / Td;
    double cs = 0.0, cp = 0.0;
    auto shade = [&](uint32_t k, uint32_t s) {
        if (s) {
            const double p = (double)s * invT;
            const double d = (double)(k + 2u) - two_mu;
            const double d3 = d * d * d;
            cs += d3 * p;
            cp += d3 * d * p;
        }
    };
    if (wide) {
        if constexpr (wide_ok) level_sweep<4>(r0, gs, 2u * ng - 1u, Sp, shade);
    } else {
        level_sweep<1>(r0, gs, 2u * ng - 1u, Sp, shade);
    }
    double CSHADE, CPROM;
    if constexpr (Grp::kBatched) {
        const double pr = g.reduce_pair(cs, cp);
        CSHADE = g.bcast(pr, 0);
        CPROM = g.bcast(pr, 8);
    } else {
        CSHADE = g.sum(cs);
        CPROM = g.sum(cp);
    }
    // Mutual information HX + HY - HXY (HX = HY for a symmetric matrix),
    // re-summed cell by cell where the closed form 2 HX - JE loses digits.
    // Only the decision is taken here (log2 T in single precision is ample
    // for it); the closed form itself is evaluated with the features.
    const double mi_cf = (double)__log2f((float)Td) - (2.0 * rlr_t - plp_t) * invT;
    double MI = __builtin_nan("");
    if (mi_cf < mi_resum_threshold<Acc>()) {
        Comp<Acc> m;
        const Acc invTa = (Acc)invT;
        src.for_each(g, [&](uint32_t lo, uint32_t hi, uint32_t c) {
            const bool diag = lo == hi;
            const uint64_t P = diag ? 2ull * c : (uint64_t)c;
            const Acc mult = diag ? (Acc)1 : (Acc)2;
            const uint64_t A = P * T;                               // P T < 2^64
            const uint64_t B = (uint64_t)R[lo] * (uint64_t)R[hi];   // px py T^2
            const Acc delta = A >= B ? (Acc)(A - B) / (Acc)B : -((Acc)(B - A) / (Acc)B);
            const Acc p = (Acc)P * invTa;
            m.add(mult * p * log1p_<Acc>(delta) * (Acc)1.4426950408889634);
        });
        MI = g.sum(comp_value(m));
    }
    if constexpr (Grp::kBatched) {
        if (rk < kSumSlots) {
            const uint64_t bits = rk < 6 ? (uint64_t)slot : __builtin_bit_cast(uint64_t, slot);
            reinterpret_cast<uint64_t *>(out)[rk] = bits;
        }
    } else if (r0 == 0) {
        out->T = tot_u[0]; out->S1 = tot_u[1]; out->S2 = tot_u[2]; out->Sm1 = tot_u[3]; out->S11 = tot_u[4];
        out->sumP2 = tot_u[5];
        out->plp = tot_d[0]; out->rlr = tot_d[1]; out->slp = tot_d[2]; out->plps = tot_d[3];
        out->hom1 = tot_d[4]; out->hom2 = tot_d[5]; out->idmn = tot_d[6]; out->idn = tot_d[7]; out->iv = tot_d[8];
        out->spare = 0.0;
    }
    if (r0 == 0) {
        out->maxP = maxPt;
        out->CSHADE = CSHADE;
        out->CPROM = CPROM;
        out->MI = MI;
    }
    // Clean up for the next direction / item.
    g.sync();
    for (uint32_t i = r0; i < ng; i += gs) { R[i] = 0u; Sm[i] = 0u; }
    for (uint32_t k = r0; k < 2u * ng - 1u; k += gs) Sp[k] = 0u;
    src.clear(g);
    g.sync();
    return T;
}

// Reduced sums of one direction of a non-symmetric matrix (ordered counts):
// the source hands cells (a, b, c) with P(a, b) = c, a the level at v and b
// the level at v + d.  R and Cm are the row and column marginals (ng u32
// each), Sp and Sm the sum and difference marginals (2 ng - 1 and ng u32),
// all zeroed LDS arrays that are zeroed again on return; *out and *outy
// receive the sums (the column-marginal ones in *outy).  Every total is
// reduced value by value in exact integers or double.  Returns T.
template <class Acc, class Grp, class Src>
__device__ uint64_t dir_sums_ns(const Grp &g, const Src &src, uint32_t *R, uint32_t *Cm, uint32_t *Sp, uint32_t *Sm,
                                uint32_t ng, DirSums *out, DirSumsY *outy) {
    const int r0 = g.rank(), gs = g.size();
    uint64_t Tl = 0, sumP2 = 0, S11 = 0;
    uint32_t maxP = 0;
    LaneSum<Acc> plp;
    src.for_each(g, [&](uint32_t a, uint32_t b, uint32_t c) {
        atomicAdd(&R[a], c);
        atomicAdd(&Cm[b], c);
        atomicAdd(&Sp[a + b], c);
        atomicAdd(&Sm[a > b ? a - b : b - a], c);
        Tl += c;
        sumP2 += (uint64_t)c * c;
        maxP = c > maxP ? c : maxP;
        S11 += (uint64_t)c * __umul24(a + 1u, b + 1u);   // levels < 2^16: exact
        plp.add((Acc)c * term_log2<Acc>((Acc)c));
    });
    g.sync();
    uint64_t S1 = 0, S2 = 0, S1y = 0, S2y = 0, Sm1 = 0;
    LaneSum<Acc> rlr, clc, slp, hom1, hom2, idmn, idn, iv, plps;
    const Acc ngf = (Acc)ng, rng = (Acc)1 / ngf, rng2 = rng * rng;
    for (uint32_t i = r0; i < ng; i += gs) {
        const uint64_t lv = i + 1u;
        const uint32_t r = R[i];
        if (r) {
            S1 += lv * r;
            S2 += lv * lv * r;
            rlr.add((Acc)r * term_log2<Acc>((Acc)r));
        }
        const uint32_t q = Cm[i];
        if (q) {
            S1y += lv * q;
            S2y += lv * lv * q;
            clc.add((Acc)q * term_log2<Acc>((Acc)q));
        }
        const uint32_t sm = Sm[i];
        if (sm) {
            Sm1 += (uint64_t)i * sm;
            const Acc sf = (Acc)sm, k = (Acc)i;
            slp.add(sf * term_log2<Acc>(sf));
            hom1.add(term_div<Acc>(sf, (Acc)1 + k));
            hom2.add(term_div<Acc>(sf, (Acc)1 + k * k));
            idmn.add(term_div<Acc>(sf, (Acc)1 + (k * k) * rng2));
            idn.add(term_div<Acc>(sf, (Acc)1 + k * rng));
            if (i > 0) iv.add(term_div<Acc>(sf, k * k));
        }
    }
    for (uint32_t k = r0; k < 2u * ng - 1u; k += gs) {
        const uint32_t sp = Sp[k];
        if (sp) plps.add((Acc)sp * term_log2<Acc>((Acc)sp));
    }
    const uint64_t T = g.sum(Tl);
    const uint64_t S1t = g.sum(S1), S2t = g.sum(S2), S1yt = g.sum(S1y), S2yt = g.sum(S2y), Sm1t = g.sum(Sm1);
    const uint64_t S11t = g.sum(S11), sumP2t = g.sum(sumP2);
    const double plp_t = g.sum(comp_value(plp)), rlr_t = g.sum(comp_value(rlr)), clc_t = g.sum(comp_value(clc));
    const double slp_t = g.sum(comp_value(slp)), plps_t = g.sum(comp_value(plps));
    const double hom1_t = g.sum(comp_value(hom1)), hom2_t = g.sum(comp_value(hom2));
    const double idmn_t = g.sum(comp_value(idmn)), idn_t = g.sum(comp_value(idn)), iv_t = g.sum(comp_value(iv));
    const uint32_t maxPt = g.max(maxP);
    double CSHADE = 0.0, CPROM = 0.0, MI = __builtin_nan("");
    if (T) {
        const double Td = (double)T, invT = 1.0 / Td;
        // cluster shade / prominence: moments of the sum marginal about mu_x + mu_y
        const double mu_s = (double)(S1t + S1yt) / Td;   // one rounding (see dir_sums)
        double cs = 0.0, cp = 0.0;
        for (uint32_t k = r0; k < 2u * ng - 1u; k += gs) {
            const uint32_t sp = Sp[k];
            if (sp) {
                const double p = (double)sp * invT;
                const double d = (double)(k + 2u) - mu_s;
                const double d3 = d * d * d;
                cs += d3 * p;
                cp += d3 * d * p;
            }
        }
        CSHADE = g.sum(cs);
        CPROM = g.sum(cp);
        // mutual information HX + HY - HXY, re-summed cell by cell when the
        // closed form would lose the digits the information measures need
        const double mi_cf = (double)__log2f((float)Td) - (rlr_t + clc_t - plp_t) * invT;
        if (mi_cf < mi_resum_threshold<Acc>()) {
            Comp<Acc> m;
            const Acc invTa = (Acc)invT;
            src.for_each(g, [&](uint32_t a, uint32_t b, uint32_t c) {
                const uint64_t A = (uint64_t)c * T;                    // P T < 2^64
                const uint64_t B = (uint64_t)R[a] * (uint64_t)Cm[b];   // px py T^2
                const Acc delta = A >= B ? (Acc)(A - B) / (Acc)B : -((Acc)(B - A) / (Acc)B);
                m.add((Acc)c * invTa * log1p_<Acc>(delta) * (Acc)1.4426950408889634);
            });
            MI = g.sum(comp_value(m));
        }
    }
    if (r0 == 0) {
        out->T = T; out->S1 = S1t; out->S2 = S2t; out->Sm1 = Sm1t; out->S11 = S11t; out->sumP2 = sumP2t;
        out->plp = plp_t; out->rlr = rlr_t; out->slp = slp_t; out->plps = plps_t;
        out->hom1 = hom1_t; out->hom2 = hom2_t; out->idmn = idmn_t; out->idn = idn_t; out->iv = iv_t;
        out->spare = 0.0;
        out->maxP = maxPt;
        out->CSHADE = CSHADE;
        out->CPROM = CPROM;
        out->MI = MI;
        outy->S1y = S1yt; outy->S2y = S2yt; outy->clc = clc_t; outy->spare = 0.0;
    }
    g.sync();
    for (uint32_t i = r0; i < ng; i += gs) { R[i] = 0u; Cm[i] = 0u; Sm[i] = 0u; }
    for (uint32_t k = r0; k < 2u * ng - 1u; k += gs) Sp[k] = 0u;
    src.clear(g);
    g.sync();
    return T;
}

}  // namespace nyx
