// nyx_features.h -- GLCM normalisation, marginals and the 30 features of one
// direction, computed by a cooperating group of lanes (one wavefront, or a
// whole work-group) from the nonzero cells of the upper triangle.
//
// Definitions: the GLCM rows of the paper's Supplementary Table S3 (NY column)
// with the standard IBSI formulas the paper defers to.  The arithmetic is
// arranged for exactness on integers where that is cheap:
//   T      = sum P                         (exact, 64-bit)
//   S1     = sum_i i R(i), S2 = sum_i i^2 R(i), S11 = sum i j P(i, j)
//   Nvar   = T S2 - S1^2,  Ncov = T S11 - S1^2   (exact, 128-bit)
//   mean = S1 / T, variance = Nvar / T^2, correlation = Ncov / Nvar,
//   sum-average = 2 S1 / T, sum-variance = cluster tendency = 2(Nvar+Ncov)/T^2,
//   contrast = (2 S2 - 2 S11) / T, difference variance from exact moments,
//   ASM = sum P^2 / T^2, maximum probability = max P / T.
// Entropies, homogeneities and inverse variance are compensated sums of
// positive terms in the accumulation precision Acc (float or double); the
// cluster shade / prominence moments are centred double sums.  The mutual
// information (HX + HY - HXY) is taken as 2 HX - JE, and re-summed cell by
// cell as sum p log(p / (px py)) when small, where the subtraction would
// lose the digits the information measure of correlation needs.
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
// One wavefront.
struct WaveGrp {
    __device__ __forceinline__ int rank() const { return lane(); }
    __device__ __forceinline__ int size() const { return kWave; }
    __device__ __forceinline__ void sync() const {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    template <class T> __device__ __forceinline__ T sum(T v) const { return wave_sum(v); }
    template <class T> __device__ __forceinline__ T max(T v) const { return wave_max(v); }
    template <class F> __device__ __forceinline__ F csum(const Comp<F> &c) const { return wave_sum_comp(c); }
};

// The whole work-group; `scratch` is LDS room for one 8-byte value per wave.
struct BlockGrp {
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
    template <class F> __device__ __forceinline__ F csum(const Comp<F> &c) const {
        return sum_of_waves<F>(wave_sum_comp(c));
    }
};

// ------------------------------------------------------------- sources
// A source enumerates candidate cells e in [0, size()); get() returns the
// 0-based levels lo <= hi and the triangle count (0 = skip the cell).

template <bool PACKED>
struct SrcDenseList {     // fused dense mode: LDS triangle + list of touched cells
    const uint32_t *list;
    uint32_t n;
    uint32_t *U;             // u32 counts, or u16 counts packed two per word
    __device__ __forceinline__ uint32_t size() const { return n; }
    __device__ __forceinline__ uint64_t get(uint32_t e, uint32_t &lo, uint32_t &hi) const {
        uint32_t p = list[e];
        lo = p & 0xFFFFu;
        hi = p >> 16;
        const uint32_t i = tri_idx(lo, hi);
        return PACKED ? (uint64_t)reinterpret_cast<const uint16_t *>(U)[i] : (uint64_t)U[i];
    }
    __device__ __forceinline__ void clear(uint32_t e) const {
        uint32_t p = list[e];
        const uint32_t i = tri_idx(p & 0xFFFFu, p >> 16);
        if (PACKED) reinterpret_cast<uint16_t *>(U)[i] = 0u;
        else U[i] = 0u;
    }
};

struct SrcHashList {      // hash mode: LDS hash slots listed per direction
    const uint32_t *list;
    uint32_t n;
    uint32_t *keys;
    uint32_t *cnts;
    __device__ __forceinline__ uint32_t size() const { return n; }
    __device__ __forceinline__ uint64_t get(uint32_t e, uint32_t &lo, uint32_t &hi) const {
        uint32_t s = list[e];
        uint32_t k = keys[s];
        lo = k & 0x1FFFu;
        hi = (k >> 13) & 0x1FFFu;
        return cnts[s];
    }
    __device__ __forceinline__ void clear(uint32_t e) const {
        uint32_t s = list[e];
        keys[s] = kNone;
        cnts[s] = 0u;
    }
};

struct SrcSquare {        // global dense square (upper triangle used)
    const uint64_t *G;
    uint32_t ng;
    __device__ __forceinline__ uint32_t size() const { return ng * ng; }
    __device__ __forceinline__ uint64_t get(uint32_t e, uint32_t &lo, uint32_t &hi) const {
        lo = e / ng;
        hi = e - lo * ng;
        return lo <= hi ? G[e] : 0ull;
    }
    __device__ __forceinline__ void clear(uint32_t) const {}
};

struct SrcCoo {           // sorted COO segment of one ROI-direction
    const uint64_t *key;
    const uint64_t *cnt;
    uint32_t n;
    uint64_t prefix;         // expected roi << 38 | dir << 32
    uint32_t ng;
    uint32_t *err;
    __device__ __forceinline__ uint32_t size() const { return n; }
    // Cells outside the matrix or of another (roi, dir) are skipped and flagged.
    __device__ __forceinline__ uint64_t get(uint32_t e, uint32_t &lo, uint32_t &hi) const {
        uint64_t k = key[e];
        lo = (uint32_t)(k >> 16) & 0xFFFFu;
        hi = (uint32_t)k & 0xFFFFu;
        uint64_t c = cnt[e];
        if ((k & ~0xFFFFFFFFull) != prefix || lo > hi || hi >= ng || c >= (1ull << 32)) {
            if (c) atomicOr(err, (uint32_t)E_COO_RANGE);
            lo = hi = 0;
            return 0ull;
        }
        return c;
    }
    __device__ __forceinline__ void clear(uint32_t) const {}
};

// Reduced per-direction sums (wave-uniform), input of finalize_dir.
struct DirSums {
    uint64_t T, S1, S2, Sm1, S11, sumP2, maxP, pad;
    double HX, DENT, HOM1, HOM2, IDMN, IDN, IV, SENT, JE, CSHADE, CPROM, MI;
};

// The 30 features of one direction from its reduced sums (one lane).
__device__ __noinline__ void finalize_dir(const DirSums &s, double *out) {
    if (s.T == 0) {
        for (int f = 0; f < kNumFeat; ++f) out[f] = __builtin_nan("");
        return;
    }
    const uint64_t T = s.T, S1 = s.S1, S2 = s.S2, S11 = s.S11, Sm1 = s.Sm1;
    const double Td = (double)T;
    const double T2 = Td * Td;
    const u128 Tq = (u128)T;
    const u128 s1sq = (u128)S1 * (u128)S1;
    const u128 nvar = Tq * (u128)S2 - s1sq;
    const i128 ncov = (i128)(Tq * (u128)S11) - (i128)s1sq;
    const u128 sm2 = 2 * (u128)S2 - 2 * (u128)S11;     // sum (i - j)^2 P
    const u128 ndv = Tq * sm2 - (u128)Sm1 * (u128)Sm1;
    const bool single = nvar == 0;
    const double var = u128_to_double(nvar) / T2;
    out[F_ASM] = out[F_ENERGY] = (double)s.sumP2 / T2;
    out[F_ACOR] = (double)S11 / Td;
    out[F_CLUPROM] = s.CPROM;
    out[F_CLUSHADE] = s.CSHADE;
    out[F_CLUTEND] = out[F_SUMVAR] = i128_to_double(2 * (i128)nvar + 2 * ncov) / T2;
    out[F_CONTRAST] = u128_to_double(sm2) / Td;
    out[F_CORR] = single ? 1.0 : i128_to_double(ncov) / u128_to_double(nvar);
    out[F_DIFAVE] = out[F_DIS] = (double)Sm1 / Td;
    out[F_DIFENTRO] = s.DENT;
    out[F_DIFVAR] = u128_to_double(ndv) / T2;
    out[F_ENTROPY] = out[F_JE] = s.JE;
    out[F_HOM1] = out[F_ID] = s.HOM1;
    out[F_HOM2] = out[F_IDM] = s.HOM2;
    const double mi = s.MI > 0.0 ? s.MI : 0.0;
    out[F_INFOMEAS1] = single ? 0.0 : -s.MI / s.HX;
    out[F_INFOMEAS2] = sqrt(1.0 - exp(-2.0 * mi));
    out[F_IDMN] = s.IDMN;
    out[F_IDN] = s.IDN;
    out[F_IV] = s.IV;
    out[F_JAVE] = (double)S1 / Td;
    out[F_JMAX] = (double)s.maxP / Td;
    out[F_SUMAVE] = 2.0 * (double)S1 / Td;
    out[F_SUMENT] = s.SENT;
    out[F_JVAR] = out[F_VARIANCE] = var;
}

template <class F> __device__ __forceinline__ F log2_(F x);
template <> __device__ __forceinline__ float log2_<float>(float x) { return log2f(x); }
template <> __device__ __forceinline__ double log2_<double>(double x) { return log2(x); }
template <class F> __device__ __forceinline__ F log1p_(F x);
template <> __device__ __forceinline__ float log1p_<float>(float x) { return log1pf(x); }
template <> __device__ __forceinline__ double log1p_<double>(double x) { return log1p(x); }

// Reduced sums of one direction.  R, Sp, Sm are zeroed LDS arrays of ng,
// 2 ng - 1 and ng u32 (row, sum and difference marginals of the symmetric
// matrix); they are zeroed again on return, and the source cells are cleared.
// *out (LDS) is written by rank 0.  Returns T (0: direction empty).
template <class Acc, class Grp, class Src>
__device__ uint64_t dir_sums(const Grp &g, const Src &src, uint32_t *R, uint32_t *Sp,
                             uint32_t *Sm, uint32_t ng, DirSums *out) {
    const uint32_t n = src.size();
    const int r0 = g.rank(), gs = g.size();
    // Sweep 1: marginals.  An off-diagonal triangle cell (lo < hi) with count
    // c stands for P(lo, hi) = P(hi, lo) = c, a diagonal one for P = 2c.
    uint64_t Tl = 0;
    for (uint32_t e = r0; e < n; e += gs) {
        uint32_t lo, hi;
        uint64_t c = src.get(e, lo, hi);
        if (c == 0) continue;
        uint32_t c32 = (uint32_t)c;
        atomicAdd(&R[lo], c32);
        atomicAdd(&R[hi], c32);
        atomicAdd(&Sp[lo + hi], 2u * c32);
        atomicAdd(&Sm[hi - lo], 2u * c32);
        Tl += 2ull * c;
    }
    const uint64_t T = g.sum(Tl);
    g.sync();
    if (T == 0) {
        if (r0 == 0) out->T = 0;
        g.sync();
        return 0;
    }
    const double Td = (double)T;
    const Acc invT = (Acc)(1.0 / Td);
    // Level sweeps over the marginals.
    uint64_t S1 = 0, S2 = 0, Sm1 = 0;
    Comp<Acc> hx, dent, hom1, hom2, idmn, idn, iv, sent, je, mi;
    const Acc ngf = (Acc)ng;
    for (uint32_t i = r0; i < ng; i += gs) {
        uint32_t r = R[i];
        if (r) {
            uint64_t lv = i + 1u;
            S1 += lv * r;
            S2 += lv * lv * r;
            Acc p = (Acc)r * invT;
            hx.add(-p * log2_<Acc>(p));
        }
        uint32_t s = Sm[i];
        if (s) {
            Sm1 += (uint64_t)i * s;
            Acc p = (Acc)s * invT;
            Acc k = (Acc)i;
            dent.add(-p * log2_<Acc>(p));
            hom1.add(p / ((Acc)1 + k));
            hom2.add(p / ((Acc)1 + k * k));
            idmn.add(p / ((Acc)1 + (k * k) / (ngf * ngf)));
            idn.add(p / ((Acc)1 + k / ngf));
            if (i > 0) iv.add(p / (k * k));
        }
    }
    for (uint32_t k = r0; k < 2u * ng - 1u; k += gs) {
        uint32_t s = Sp[k];
        if (s) {
            Acc p = (Acc)s * invT;
            sent.add(-p * log2_<Acc>(p));
        }
    }
    // Sweep 2: cell terms.
    uint64_t sumP2 = 0, maxP = 0, S11 = 0;
    for (uint32_t e = r0; e < n; e += gs) {
        uint32_t lo, hi;
        uint64_t c = src.get(e, lo, hi);
        if (c == 0) continue;
        bool diag = lo == hi;
        uint64_t P = diag ? 2ull * c : c;
        uint64_t mult = diag ? 1ull : 2ull;
        sumP2 += mult * P * P;
        maxP = P > maxP ? P : maxP;
        S11 += mult * (uint64_t)(lo + 1u) * (uint64_t)(hi + 1u) * P;
        Acc p = (Acc)P * invT;
        je.add(-(Acc)mult * p * log2_<Acc>(p));
    }
    S1 = g.sum(S1);
    S2 = g.sum(S2);
    Sm1 = g.sum(Sm1);
    sumP2 = g.sum(sumP2);
    maxP = g.max(maxP);
    S11 = g.sum(S11);
    const double HX = (double)g.csum(hx);
    const double DENT = (double)g.csum(dent);
    const double HOM1 = (double)g.csum(hom1);
    const double HOM2 = (double)g.csum(hom2);
    const double IDMN = (double)g.csum(idmn);
    const double IDN = (double)g.csum(idn);
    const double IV = (double)g.csum(iv);
    const double SENT = (double)g.csum(sent);
    const double JE = (double)g.csum(je);
    // Cluster shade / prominence: moments of the sum marginal about 2 mu.
    const double two_mu = 2.0 * (double)S1 / Td;
    Comp<double> cs, cp;
    for (uint32_t k = r0; k < 2u * ng - 1u; k += gs) {
        uint32_t s = Sp[k];
        if (s) {
            double p = (double)s / Td;
            double d = (double)(k + 2u) - two_mu;
            double d3 = d * d * d;
            cs.add(d3 * p);
            cp.add(d3 * d * p);
        }
    }
    const double CSHADE = g.csum(cs);
    const double CPROM = g.csum(cp);
    // Mutual information HX + HY - HXY (HX = HY for a symmetric matrix).
    double MI = 2.0 * HX - JE;
    if (MI < 0.25) {
        Comp<Acc> m;
        for (uint32_t e = r0; e < n; e += gs) {
            uint32_t lo, hi;
            uint64_t c = src.get(e, lo, hi);
            if (c == 0) continue;
            bool diag = lo == hi;
            uint64_t P = diag ? 2ull * c : c;
            Acc mult = diag ? (Acc)1 : (Acc)2;
            uint64_t A = P * T;                               // P T < 2^64
            uint64_t B = (uint64_t)R[lo] * (uint64_t)R[hi];   // px py T^2
            Acc delta = A >= B ? (Acc)(A - B) / (Acc)B : -((Acc)(B - A) / (Acc)B);
            Acc p = (Acc)P * invT;
            m.add(mult * p * log1p_<Acc>(delta) * (Acc)1.4426950408889634);
        }
        MI = (double)g.csum(m);
    }
    if (r0 == 0) {
        out->T = T; out->S1 = S1; out->S2 = S2; out->Sm1 = Sm1; out->S11 = S11;
        out->sumP2 = sumP2; out->maxP = maxP;
        out->HX = HX; out->DENT = DENT; out->HOM1 = HOM1; out->HOM2 = HOM2; out->IDMN = IDMN;
        out->IDN = IDN; out->IV = IV; out->SENT = SENT; out->JE = JE; out->CSHADE = CSHADE;
        out->CPROM = CPROM; out->MI = MI;
    }
    // Clean up for the next direction / item.
    g.sync();
    for (uint32_t i = r0; i < ng; i += gs) { R[i] = 0u; Sm[i] = 0u; }
    for (uint32_t k = r0; k < 2u * ng - 1u; k += gs) Sp[k] = 0u;
    for (uint32_t e = r0; e < n; e += gs) src.clear(e);
    g.sync();
    return T;
}

}  // namespace nyx
