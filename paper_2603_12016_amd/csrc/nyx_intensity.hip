// nyx_intensity.hip -- first-order intensity features of every ROI.
//
// The intensity group of the paper's feature list (Supplementary Table S1,
// "2-dimensional intensity features", the rows with the NY mark; Table S5
// holds the same statistics for volumes).  The paper names the features and
// states their cost: O(m) in the voxel count m for the moments, O(m, h) for
// the histogram-based ones with h intensity bins (Materials and methods,
// "Feature Control and Tunability").  Each feature is the usual statistical
// definition; the choices the paper leaves open are:
//   * VARIANCE / STDDEV are unbiased (n - 1); a single voxel has variance 0;
//   * SKEWNESS, KURTOSIS, HYPERSKEWNESS, HYPERFLATNESS are the biased central
//     moments m3..m6 over m2^(k/2), 0 for a constant ROI (kurtosis not
//     excess);
//   * percentiles interpolate linearly between the closest ranks: with the n
//     values sorted and h = (n - 1) p / 100, x_(floor h) + frac(h) (x_(floor
//     h + 1) - x_(floor h));
//   * MEDIAN_ABSOLUTE_DEVIATION is the mean distance to the median;
//   * ROBUST_MEAN_ABSOLUTE_DEVIATION is the mean distance to their mean of
//     the values within [P10, P90] (NaN when no value lies there);
//   * MODE, ENTROPY (log2) and UNIFORMITY use the histogram of the
//     fixed-bin-number levels 1..n_bins over the ROI's [min, max] (the same
//     discretisation as the texture features); MODE takes the lowest level
//     among ties;
//   * UNIFORMITY_PIU = 100 (1 - (max - min) / (max + min)), 100 when both are 0;
//   * WEIGHTED_CENTROID_* use image coordinates (column, row, plane), NaN
//     when the intensities sum to 0;
//   * edge voxels are ROI voxels with a face neighbour (4 in a plane, 6 in a
//     volume) outside the image or outside the ROI; EDGE_STDDEV is unbiased.
//
// One work-group per ROI makes four passes over the ROI's bounding box (the
// values of a small ROI stay in L2 after the first):
//   A  exact integer sums (count, sum, sum of squares, coordinate-weighted
//      sums), edge-voxel sums, a 1024-bucket coarse histogram of (I - min)
//      and the level histogram;
//   B  centred moments about the mean (double) and, when the value range
//      exceeds the coarse buckets, a fine histogram of the few buckets that
//      hold the percentile ranks, so every order statistic is exact;
//   C  distance to the median and the count and sum of the values in
//      [P10, P90];
//   D  distance of those values to their mean.
#include <hip/hip_runtime.h>
#include <math.h>

#include "nyx_device.h"
#include "nyx_features.h"
#include "nyx_launch.h"

namespace nyx {

namespace {

constexpr int kFoBlock = 512;
constexpr int kFoWaves = kFoBlock / kWave;
constexpr uint32_t kFoCoarse = 1024u;      // coarse buckets of I - min
constexpr int kFoPct = 7;                  // percentiles 1, 10, 25, 50, 75, 90, 99
constexpr int kFoRanks = 2 * kFoPct;       // the two ranks each percentile interpolates between
constexpr uint32_t kFoFine = 64u;          // values per coarse bucket at most (range < 2^16)

enum FoFeat : int {
    FO_MEAN, FO_MIN, FO_MAX, FO_RANGE, FO_INTEGRATED, FO_ENERGY, FO_RMS, FO_VARIANCE, FO_STDDEV,
    FO_STDERR, FO_SKEWNESS, FO_KURTOSIS, FO_HYPERSKEWNESS, FO_HYPERFLATNESS, FO_MEANAD, FO_MEDIAN,
    FO_MEDIANAD, FO_P01, FO_P10, FO_P25, FO_P75, FO_P90, FO_P99, FO_IQR, FO_ROBUSTMAD, FO_MODE,
    FO_ENTROPY, FO_UNIFORMITY, FO_PIU, FO_WCX, FO_WCY, FO_WCZ, FO_EDGE_INTEGRATED, FO_EDGE_MIN,
    FO_EDGE_MAX, FO_EDGE_MEAN, FO_EDGE_STDDEV, FO_COUNT
};
static_assert(FO_COUNT == kNumIntensityFeat, "column count");

// Percentile i of 1, 10, 25, 50, 75, 90, 99 (one byte each).
__device__ __forceinline__ uint32_t fo_pct(uint32_t i) {
    return (uint32_t)(0x635A4B32190A01ull >> (8u * i)) & 0xFFu;
}

struct FoShared {
    uint32_t coarse[kFoCoarse];
    uint32_t fine[kFoRanks][kFoFine];
    uint8_t slot[kFoCoarse];               // coarse bucket -> fine slot + 1 (0: none)
    uint32_t rank[kFoRanks];               // 0-based rank in sorted order
    uint32_t rank_bucket[kFoRanks], rank_in[kFoRanks], rank_val[kFoRanks];
    uint32_t wave_tot[kFoWaves];
    uint64_t red[kFoWaves];
    double pct[kFoPct];
    uint32_t n_slots;
};

}  // namespace

// One work-group per ROI: the kNumIntensityFeat features of ROI blockIdx.x.
// Dynamic LDS: the level histogram (ng u32).
template <class OutT>
__global__ __launch_bounds__(kFoBlock) void k_intensity(const ImgDesc *imgs, int n_images, const RoiDesc *rois,
                                                        const uint32_t *n_rois_ptr, uint32_t roi_cap, uint32_t ng,
                                                        OutT *table, uint32_t table_rows, uint32_t *err) {
    __shared__ FoShared S;
    extern __shared__ __align__(16) uint8_t smem[];
    uint32_t *lev = reinterpret_cast<uint32_t *>(smem);
    const uint32_t r = blockIdx.x;
    const uint32_t n_rois = min(*n_rois_ptr, roi_cap);
    if (r >= n_rois) return;
    if (r >= table_rows) {
        if (threadIdx.x == 0) atomicOr(err, (uint32_t)E_TABLE_CAP);
        return;
    }
    const RoiDesc rd = rois[r];
    OutT *out = table + (uint64_t)r * kNumIntensityFeat;
    if (rd.image >= (uint32_t)n_images) return;
    const ImgDesc im = imgs[rd.image];
    if (rd.x0 < 0 || rd.y0 < 0 || rd.z0 < 0 || rd.x1 >= im.nx || rd.y1 >= im.ny || rd.z1 >= im.nz ||
        rd.x0 > rd.x1 || rd.y0 > rd.y1 || rd.z0 > rd.z1)
        return;
    const uint32_t W = (uint32_t)(rd.x1 - rd.x0 + 1), H = (uint32_t)(rd.y1 - rd.y0 + 1),
                   Dz = (uint32_t)(rd.z1 - rd.z0 + 1);
    const uint32_t nx = (uint32_t)im.nx, plane = (uint32_t)im.ny * nx;
    const uint32_t label = rd.label, vmin = rd.vmin, vmax = rd.vmax, D = vmax - vmin;
    const float rcpD = D ? 1.0f / (float)D : 0.0f;
    uint32_t sh = 0;
    while ((D >> sh) >= kFoCoarse) ++sh;
    const bool fine_needed = sh > 0;

    for (uint32_t i = threadIdx.x; i < kFoCoarse; i += kFoBlock) { S.coarse[i] = 0u; S.slot[i] = 0u; }
    for (uint32_t i = threadIdx.x; i < kFoRanks * kFoFine; i += kFoBlock) (&S.fine[0][0])[i] = 0u;
    for (uint32_t i = threadIdx.x; i < ng; i += kFoBlock) lev[i] = 0u;
    __syncthreads();

    // ---- pass A: exact integer sums, edge voxels, coarse and level histograms
    uint32_t cnt = 0, ecnt = 0, emin = 0xFFFFFFFFu, emax = 0u;
    uint64_t s1 = 0, s2 = 0, cx = 0, cy = 0, cz = 0, es1 = 0, es2 = 0;
    const bool vol = im.nz > 1;
    for (BoxWalk<kFoBlock> b(W, H, Dz); b.ok(); b.next()) {
        const int32_t X = rd.x0 + (int32_t)b.x, Y = rd.y0 + (int32_t)b.y, Z = rd.z0 + (int32_t)b.z;
        const uint32_t v = (uint32_t)Z * plane + (uint32_t)Y * nx + (uint32_t)X;
        if (ldg(im.L, v) != label) continue;
        const uint32_t x = ldg(im.I, v);
        ++cnt;
        s1 += x;
        s2 += (uint64_t)x * x;
        cx += (uint64_t)x * (uint32_t)X;
        cy += (uint64_t)x * (uint32_t)Y;
        cz += (uint64_t)x * (uint32_t)Z;
        atomicAdd(&S.coarse[(x - vmin) >> sh], 1u);
        atomicAdd(&lev[fbn_level(x, vmin, D, rcpD, ng) - 1u], 1u);
        bool edge = X == 0 || X == im.nx - 1 || Y == 0 || Y == im.ny - 1;
        if (!edge) edge = ldg(im.L, v - 1u) != label || ldg(im.L, v + 1u) != label || ldg(im.L, v - nx) != label ||
                          ldg(im.L, v + nx) != label;
        if (vol && !edge) edge = Z == 0 || Z == im.nz - 1 || ldg(im.L, v - plane) != label || ldg(im.L, v + plane) != label;
        if (edge) {
            ++ecnt;
            es1 += x;
            es2 += (uint64_t)x * x;
            emin = min(emin, x);
            emax = max(emax, x);
        }
    }
    const uint64_t n = block_sum<kFoWaves, uint64_t>(cnt, S.red);
    const uint64_t S1 = block_sum<kFoWaves>(s1, S.red), S2 = block_sum<kFoWaves>(s2, S.red);
    const uint64_t CX = block_sum<kFoWaves>(cx, S.red), CY = block_sum<kFoWaves>(cy, S.red), CZ = block_sum<kFoWaves>(cz, S.red);
    const uint64_t ne = block_sum<kFoWaves, uint64_t>(ecnt, S.red), ES1 = block_sum<kFoWaves>(es1, S.red), ES2 = block_sum<kFoWaves>(es2, S.red);
    const uint32_t EMIN = block_reduce<kFoWaves>(emin, S.red, OpMin()), EMAX = block_reduce<kFoWaves>(emax, S.red, OpMax());
    if (n == 0) {
        // (cannot happen for a ROI found by discovery)
        for (uint32_t f = threadIdx.x; f < (uint32_t)kNumIntensityFeat; f += kFoBlock) out[f] = (OutT)__builtin_nan("");
        return;
    }
    const double nd = (double)n, mean = (double)S1 / nd;

    // ---- order-statistic ranks and the coarse buckets holding them
    if (threadIdx.x < (uint32_t)kFoPct) {
        const uint32_t p = fo_pct(threadIdx.x);
        const double h = (double)((n - 1u) * (uint64_t)p) / 100.0;
        const uint64_t lo = (uint64_t)floor(h);
        S.rank[2 * threadIdx.x] = (uint32_t)lo;
        S.rank[2 * threadIdx.x + 1] = (uint32_t)min(lo + 1u, n - 1u);
    }
    {
        // exclusive prefix of the coarse counts: thread t owns buckets 2t, 2t + 1
        static_assert(kFoCoarse == 2u * kFoBlock, "two buckets per thread");
        const uint32_t b0 = 2u * threadIdx.x;
        const uint32_t c0 = S.coarse[b0], c1 = S.coarse[b0 + 1u];
        const uint32_t incl = wave_incl_scan(c0 + c1);
        if (lane() == kWave - 1) S.wave_tot[threadIdx.x / kWave] = incl;
        __syncthreads();
        uint32_t base = 0;
        for (uint32_t w = 0; w < threadIdx.x / kWave; ++w) base += S.wave_tot[w];
        const uint32_t e0 = base + incl - (c0 + c1), e1 = e0 + c0;
        for (int k = 0; k < kFoRanks; ++k) {
            const uint32_t rk = S.rank[k];
            if (rk >= e0 && rk < e0 + c0) { S.rank_bucket[k] = b0; S.rank_in[k] = rk - e0; }
            if (rk >= e1 && rk < e1 + c1) { S.rank_bucket[k] = b0 + 1u; S.rank_in[k] = rk - e1; }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t ns = 0;
        for (int k = 0; k < kFoRanks; ++k) {
            const uint32_t b = S.rank_bucket[k];
            if (!fine_needed) {
                S.rank_val[k] = vmin + b;
            } else if (S.slot[b] == 0u) {
                S.slot[b] = (uint8_t)(++ns);
            }
        }
        S.n_slots = ns;
    }
    __syncthreads();

    // ---- pass B: centred moments; fine histograms of the rank buckets
    double m2 = 0.0, m3 = 0.0, m4 = 0.0, m5 = 0.0, m6 = 0.0, mad = 0.0;
    const uint32_t fmask = (1u << sh) - 1u;
    for (BoxWalk<kFoBlock> b(W, H, Dz); b.ok(); b.next()) {
        const uint32_t v = (uint32_t)(rd.z0 + (int32_t)b.z) * plane + (uint32_t)(rd.y0 + (int32_t)b.y) * nx +
                           (uint32_t)(rd.x0 + (int32_t)b.x);
        if (ldg(im.L, v) != label) continue;
        const uint32_t x = ldg(im.I, v);
        const double d = (double)x - mean, d2 = d * d;
        m2 += d2;
        m3 += d2 * d;
        m4 += d2 * d2;
        m5 += d2 * d2 * d;
        m6 += d2 * d2 * d2;
        mad += fabs(d);
        if (fine_needed) {
            const uint32_t q = x - vmin, s = S.slot[q >> sh];
            if (s) atomicAdd(&S.fine[s - 1u][q & fmask], 1u);
        }
    }
    m2 = block_sum<kFoWaves>(m2, S.red);
    m3 = block_sum<kFoWaves>(m3, S.red);
    m4 = block_sum<kFoWaves>(m4, S.red);
    m5 = block_sum<kFoWaves>(m5, S.red);
    m6 = block_sum<kFoWaves>(m6, S.red);
    mad = block_sum<kFoWaves>(mad, S.red);
    if (fine_needed && threadIdx.x < (uint32_t)kFoRanks) {
        const uint32_t k = threadIdx.x, b = S.rank_bucket[k], s = S.slot[b] - 1u;
        uint32_t acc = 0, f = 0;
        for (; f < (1u << sh); ++f) {
            acc += S.fine[s][f];
            if (acc > S.rank_in[k]) break;
        }
        S.rank_val[k] = vmin + (b << sh) + f;
    }
    __syncthreads();
    if (threadIdx.x < (uint32_t)kFoPct) {
        const uint32_t p = fo_pct(threadIdx.x);
        const double h = (double)((n - 1u) * (uint64_t)p) / 100.0;
        const double lo = floor(h);
        const double xl = (double)S.rank_val[2 * threadIdx.x], xh = (double)S.rank_val[2 * threadIdx.x + 1];
        S.pct[threadIdx.x] = xl + (h - lo) * (xh - xl);
    }
    __syncthreads();
    const double med = S.pct[3], p10 = S.pct[1], p90 = S.pct[5];

    // ---- pass C: distance to the median; the values within [P10, P90]
    double dmed = 0.0;
    uint32_t rc = 0;
    uint64_t rs = 0;
    for (BoxWalk<kFoBlock> b(W, H, Dz); b.ok(); b.next()) {
        const uint32_t v = (uint32_t)(rd.z0 + (int32_t)b.z) * plane + (uint32_t)(rd.y0 + (int32_t)b.y) * nx +
                           (uint32_t)(rd.x0 + (int32_t)b.x);
        if (ldg(im.L, v) != label) continue;
        const double x = (double)ldg(im.I, v);
        dmed += fabs(x - med);
        if (x >= p10 && x <= p90) { ++rc; rs += (uint64_t)x; }
    }
    dmed = block_sum<kFoWaves>(dmed, S.red);
    const uint64_t RC = block_sum<kFoWaves, uint64_t>(rc, S.red), RS = block_sum<kFoWaves>(rs, S.red);
    const double mus = (double)RS / (double)RC;   // NaN when no value lies in [P10, P90]

    // ---- pass D: distance of the values within [P10, P90] to their mean
    double rmad = 0.0;
    if (RC) {
        for (BoxWalk<kFoBlock> b(W, H, Dz); b.ok(); b.next()) {
            const uint32_t v = (uint32_t)(rd.z0 + (int32_t)b.z) * plane + (uint32_t)(rd.y0 + (int32_t)b.y) * nx +
                               (uint32_t)(rd.x0 + (int32_t)b.x);
            if (ldg(im.L, v) != label) continue;
            const double x = (double)ldg(im.I, v);
            if (x >= p10 && x <= p90) rmad += fabs(x - mus);
        }
    }
    rmad = block_sum<kFoWaves>(rmad, S.red);

    // ---- level histogram: mode (lowest level among ties), entropy, uniformity
    uint32_t best_c = 0, best_l = 0xFFFFFFFFu;
    double ent = 0.0, uni = 0.0;
    for (uint32_t i = threadIdx.x; i < ng; i += kFoBlock) {
        const uint32_t c = lev[i];
        if (c > best_c) { best_c = c; best_l = i; }   // i rises: the first maximum is the lowest level
        if (c) {
            const double p = (double)c / nd;
            ent -= p * log2(p);
            uni += p * p;
        }
    }
    ent = block_sum<kFoWaves>(ent, S.red);
    uni = block_sum<kFoWaves>(uni, S.red);
    // the highest count, then its lowest level: one 64-bit key (count high, ~level low)
    const uint64_t key = ((uint64_t)best_c << 32) | (uint64_t)(0xFFFFFFFFu - best_l);
    const uint64_t kbest = block_reduce<kFoWaves>(key, S.red, OpMax());
    const uint32_t mode_level = 0xFFFFFFFFu - (uint32_t)kbest + 1u;

    if (threadIdx.x != 0) return;
    double f[FO_COUNT];
    f[FO_MEAN] = mean;
    f[FO_MIN] = (double)vmin;
    f[FO_MAX] = (double)vmax;
    f[FO_RANGE] = (double)D;
    f[FO_INTEGRATED] = (double)S1;
    f[FO_ENERGY] = (double)S2;
    f[FO_RMS] = sqrt((double)S2 / nd);
    // unbiased variance from exact integers: (n S2 - S1^2) / (n (n - 1))
    const u128 nvar = (u128)n * (u128)S2 - (u128)S1 * (u128)S1;
    f[FO_VARIANCE] = n > 1u ? u128_to_double(nvar) / (nd * (nd - 1.0)) : 0.0;
    f[FO_STDDEV] = sqrt(f[FO_VARIANCE]);
    f[FO_STDERR] = f[FO_STDDEV] / sqrt(nd);
    if (D > 0u) {
        const double c2 = m2 / nd, c3 = m3 / nd, c4 = m4 / nd, c5 = m5 / nd, c6 = m6 / nd;
        f[FO_SKEWNESS] = c3 / (c2 * sqrt(c2));
        f[FO_KURTOSIS] = c4 / (c2 * c2);
        f[FO_HYPERSKEWNESS] = c5 / (c2 * c2 * sqrt(c2));
        f[FO_HYPERFLATNESS] = c6 / (c2 * c2 * c2);
    } else {
        f[FO_SKEWNESS] = f[FO_KURTOSIS] = f[FO_HYPERSKEWNESS] = f[FO_HYPERFLATNESS] = 0.0;
    }
    f[FO_MEANAD] = mad / nd;
    f[FO_MEDIAN] = med;
    f[FO_MEDIANAD] = dmed / nd;
    f[FO_P01] = S.pct[0];
    f[FO_P10] = p10;
    f[FO_P25] = S.pct[2];
    f[FO_P75] = S.pct[4];
    f[FO_P90] = p90;
    f[FO_P99] = S.pct[6];
    f[FO_IQR] = S.pct[4] - S.pct[2];
    f[FO_ROBUSTMAD] = RC ? rmad / (double)RC : __builtin_nan("");
    f[FO_MODE] = (double)mode_level;
    f[FO_ENTROPY] = ent;
    f[FO_UNIFORMITY] = uni;
    const uint32_t tot = vmax + vmin;
    f[FO_PIU] = tot ? 100.0 * (1.0 - (double)D / (double)tot) : 100.0;
    const double nan = __builtin_nan("");
    f[FO_WCX] = S1 ? (double)CX / (double)S1 : nan;
    f[FO_WCY] = S1 ? (double)CY / (double)S1 : nan;
    f[FO_WCZ] = S1 ? (double)CZ / (double)S1 : nan;
    const double ned = (double)ne;
    f[FO_EDGE_INTEGRATED] = (double)ES1;
    f[FO_EDGE_MIN] = ne ? (double)EMIN : nan;
    f[FO_EDGE_MAX] = ne ? (double)EMAX : nan;
    f[FO_EDGE_MEAN] = ne ? (double)ES1 / ned : nan;
    const u128 nevar = (u128)ne * (u128)ES2 - (u128)ES1 * (u128)ES1;
    f[FO_EDGE_STDDEV] = ne > 1u ? sqrt(u128_to_double(nevar) / (ned * (ned - 1.0))) : (ne ? 0.0 : nan);
    for (int k = 0; k < FO_COUNT; ++k) out[k] = (OutT)f[k];
}

hipError_t launch_intensity(const StepArgs &a, uint32_t grid, int fp64, void *table, uint32_t table_rows,
                            hipStream_t st) {
    if (grid == 0) return hipSuccess;
    const size_t lds = (size_t)a.ng * 4u;
    if (fp64)
        hipLaunchKernelGGL(k_intensity<double>, dim3(grid), dim3(kFoBlock), lds, st, a.imgs, a.n_images, a.rois,
                           a.counters + C_NROIS, a.roi_cap, (uint32_t)a.ng, reinterpret_cast<double *>(table),
                           table_rows, a.counters + C_ERR);
    else
        hipLaunchKernelGGL(k_intensity<float>, dim3(grid), dim3(kFoBlock), lds, st, a.imgs, a.n_images, a.rois,
                           a.counters + C_NROIS, a.roi_cap, (uint32_t)a.ng, reinterpret_cast<float *>(table),
                           table_rows, a.counters + C_ERR);
    return hipGetLastError();
}

}  // namespace nyx
