// nyx_kernels.hip -- HIP kernels for CDNA4 (gfx950): per-ROI GLCM texture.
//
//   k_max_label        planning: largest label per image
//   k_reset            clear the per-label statistics and counters
//   k_scan             ROI discovery: per-label count, min, max, bbox
//   k_compact_*        ROI table in (image, label) order + size-sorted work queue
//   k_bin_image        per-voxel grey levels (explicit binning output)
//   k_batch            persistent work-stealing accumulation + reduced sums per direction
//   k_split_features   reduced sums of ROIs whose matrices were merged in global memory
//   k_features         the 30 features per direction and their mean, one lane per direction
//   k_coo_*            sorted COO export / import of the co-occurrence counts
//
// The method: the paper's regional texture extraction (one row per unique
// label, Supplementary Table S7) with the GLCM features of Table S3 under
// fixed-bin-number discretisation and symmetric matrices over the given
// offsets (Materials and methods, "Feature Control and Tunability").
#include <hip/hip_runtime.h>
#include <limits.h>

#include "nyx_device.h"
#include "nyx_features.h"
#include "nyx_launch.h"

namespace nyx {

__device__ __forceinline__ int find_image_chunk(const ImgDesc *imgs, int n, uint32_t chunk) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (imgs[mid].chunk_base <= chunk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

__device__ __forceinline__ int find_image_entry(const ImgDesc *imgs, int n, uint32_t e) {
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (imgs[mid].tab_base <= e) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------------ planning
__global__ void k_max_label(const ImgDesc *imgs, int n_images, uint32_t *out) {
    int im = blockIdx.y;
    if (im >= n_images) return;
    const ImgDesc d = imgs[im];
    uint32_t m = 0;
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < d.nvox; v += gridDim.x * blockDim.x)
        m = max(m, d.L[v]);
    m = wave_max(m);
    if (lane() == 0) atomicMax(&out[im], m);
}

// Distinct nonzero labels of a batch, as (image << 32 | label) entries of
// `list`: a work-group takes `chunk` voxels of image blockIdx.y, drops the
// repeats in an LDS hash table (label 0 marks a free slot) and appends the
// survivors.  A label may be listed by several work-groups (and by one when
// its hash probes fail); the host removes the repeats.  count receives the
// number of entries even beyond cap (the host then retries with room for all).
__global__ __launch_bounds__(256) void k_label_collect(const ImgDesc *imgs, int n_images, uint32_t chunk,
                                                       uint64_t *list, uint32_t cap, uint32_t *count) {
    constexpr uint32_t kSlots = 1024u;
    __shared__ uint32_t H[kSlots];
    for (uint32_t i = threadIdx.x; i < kSlots; i += blockDim.x) H[i] = 0u;
    __syncthreads();
    const int im = (int)blockIdx.y;
    const auto emit = [&](uint32_t l) {
        const uint32_t pos = atomicAdd(count, 1u);
        if (pos < cap) list[pos] = (uint64_t)(uint32_t)im << 32 | l;
    };
    if (im < n_images) {
        const ImgDesc d = imgs[im];
        const uint64_t v0 = (uint64_t)blockIdx.x * chunk;
        const uint64_t v1 = v0 + chunk < d.nvox ? v0 + chunk : d.nvox;
        uint32_t prev = 0u;
        for (uint64_t v = v0 + threadIdx.x; v < v1; v += blockDim.x) {
            const uint32_t l = d.L[v];
            if (l == 0u || l == prev) continue;
            prev = l;
            uint32_t h = hash_u32(l) & (kSlots - 1u);
            bool done = false;
            for (int probe = 0; probe < 32 && !done; ++probe) {
                const uint32_t cur = atomicCAS(&H[h], 0u, l);
                done = cur == 0u || cur == l;
                h = (h + 1u) & (kSlots - 1u);
            }
            if (!done) emit(l);
        }
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < kSlots; i += blockDim.x)
        if (H[i]) emit(H[i]);
}

// ------------------------------------------------------------------ reset
__global__ void k_reset(StepArgs a, uint32_t n_counters) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t e = i; e < a.tab.total; e += stride) {
        a.tab.cnt[e] = 0u;
        a.tab.mn[e] = 0xFFFFFFFFu;
        a.tab.mx[e] = 0u;
        a.tab.x0[e] = INT_MAX; a.tab.y0[e] = INT_MAX; a.tab.z0[e] = INT_MAX;
        a.tab.x1[e] = -1; a.tab.y1[e] = -1; a.tab.z1[e] = -1;
        a.tab.row[e] = kNone;
    }
    for (uint32_t e = i; e < n_counters; e += stride) a.counters[e] = 0u;
}

__global__ void k_fill_u64(uint64_t *p, uint64_t n, uint64_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// Zero the global matrices of the split slots the last compaction assigned.
__global__ void k_zero_split(StepArgs a) {
    uint32_t used = a.counters[C_NSPLIT];
    if (used > a.g_cap) used = a.g_cap;
    uint64_t n = (uint64_t)used * a.K_out * (uint64_t)a.ng * a.ng;
    const uint64_t t0 = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x, ts = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = t0; i < n; i += ts) a.G[i] = 0ull;
    if (a.smarg) {
        const uint64_t m = (uint64_t)used * a.K_out;
        for (uint64_t i = t0; i < m * 4u * (uint64_t)a.ng; i += ts) a.smarg[i] = 0u;
        for (uint64_t i = t0; i < m * 4u; i += ts) a.stot[i] = 0ull;
    }
}

// ------------------------------------------------------------------ scan
// ROI discovery.  A work-group covers a tile of kScanTileRows image rows (rows
// of all z-planes, flattened) by kScanTileCols columns; each lane walks one
// column down the tile, cutting it into vertical runs of equal label (a run
// also ends at a z-plane boundary).  Every load of the wave is one contiguous
// row segment, so the reads are fully coalesced.  Each run's statistics are
// folded into an LDS table keyed by label, and the table is flushed to the
// global per-label entries once per tile.  A label that finds no free LDS
// slot goes straight to the global entry.
constexpr int kScanSlots = 256;

struct ScanLds {
    uint32_t key[kScanSlots], cnt[kScanSlots], mn[kScanSlots], mx[kScanSlots];
    int32_t x0[kScanSlots], x1[kScanSlots], y0[kScanSlots], y1[kScanSlots], z0[kScanSlots], z1[kScanSlots];
};

__device__ __forceinline__ void scan_flush_global(const StepArgs &a, uint32_t K, uint32_t c, uint32_t mn, uint32_t mx,
                                                  int32_t x0, int32_t x1, int32_t y0, int32_t y1, int32_t z0,
                                                  int32_t z1) {
    atomicAdd(&a.tab.cnt[K], c);
    atomicMin(&a.tab.mn[K], mn);
    atomicMax(&a.tab.mx[K], mx);
    atomicMin(&a.tab.x0[K], x0); atomicMax(&a.tab.x1[K], x1);
    atomicMin(&a.tab.y0[K], y0); atomicMax(&a.tab.y1[K], y1);
    atomicMin(&a.tab.z0[K], z0); atomicMax(&a.tab.z1[K], z1);
}

// Statistics of one or more vertical runs of label key (0: none): voxel
// count, value range, and the box x0..x1, y0..y1, z0..z1 they span.
struct RunRec {
    uint32_t key, c, mn, mx;
    int32_t x0, x1, y0, y1, z0, z1;
};

__device__ __forceinline__ void scan_flush_run(const StepArgs &a, ScanLds &S, uint32_t K, const RunRec &r) {
    uint32_t h = hash_u32(K) & (kScanSlots - 1);
    for (int probe = 0; probe < 8; ++probe) {
        uint32_t cur = atomicCAS(&S.key[h], kNone, K);
        if (cur == kNone || cur == K) {
            atomicAdd(&S.cnt[h], r.c);
            atomicMin(&S.mn[h], r.mn);
            atomicMax(&S.mx[h], r.mx);
            atomicMin(&S.x0[h], r.x0); atomicMax(&S.x1[h], r.x1);
            atomicMin(&S.y0[h], r.y0); atomicMax(&S.y1[h], r.y1);
            atomicMin(&S.z0[h], r.z0); atomicMax(&S.z1[h], r.z1);
            return;
        }
        h = (h + 1u) & (kScanSlots - 1);
    }
    scan_flush_global(a, K, r.c, r.mn, r.mx, r.x0, r.x1, r.y0, r.y1, r.z0, r.z1);
}

// Flushes a finished run (key != 0) under its label's table entry; a label
// without one sets `bad`.
__device__ __forceinline__ void scan_flush_label(const StepArgs &a, ScanLds &S, const ImgDesc &d, const RunRec &r,
                                                 uint32_t &bad) {
    const uint32_t e = label_entry(d.dict, d.dict_n, d.max_label, r.key);
    if (e) scan_flush_run(a, S, d.tab_base + e, r);
    else bad = 1u;
}

// Segmented inclusive combination over each 16-lane row: the lanes of a
// maximal group of adjacent lanes with the same key form a segment, and
// after the row_shr 1, 2, 4, 8 steps the last lane of a segment holds the
// combination of the whole segment.  Every lane of the wave takes part.
template <int S>
__device__ __forceinline__ void run_step(RunRec &r, uint32_t seg) {
    const bool take = dpp32<0x110 + S>(seg) == seg;   // out-of-row sources read 0; seg >= 1
    const uint32_t c = dpp32<0x110 + S>(r.c), mn = dpp32<0x110 + S>(r.mn), mx = dpp32<0x110 + S>(r.mx);
    const int32_t x0 = (int32_t)dpp32<0x110 + S>((uint32_t)r.x0), x1 = (int32_t)dpp32<0x110 + S>((uint32_t)r.x1);
    const int32_t y0 = (int32_t)dpp32<0x110 + S>((uint32_t)r.y0), y1 = (int32_t)dpp32<0x110 + S>((uint32_t)r.y1);
    const int32_t z0 = (int32_t)dpp32<0x110 + S>((uint32_t)r.z0), z1 = (int32_t)dpp32<0x110 + S>((uint32_t)r.z1);
    if (take) {
        r.c += c; r.mn = min(r.mn, mn); r.mx = max(r.mx, mx);
        r.x0 = min(r.x0, x0); r.x1 = max(r.x1, x1);
        r.y0 = min(r.y0, y0); r.y1 = max(r.y1, y1);
        r.z0 = min(r.z0, z0); r.z1 = max(r.z1, z1);
    }
}

// Returns whether this lane ends its segment (and so holds its total).  The
// neighbour reads are made by every lane before any test: a DPP read inside
// a branch would see the lanes the branch disables as 0.
__device__ __forceinline__ bool row_segment_combine(RunRec &r) {
    const uint32_t rl = lane() & 15u;
    const uint32_t prev = dpp32<0x111>(r.key), next = dpp32<0x101>(r.key);   // row_shr:1, row_shl:1
    const uint32_t head = (uint32_t)(rl == 0u) | (uint32_t)(prev != r.key);
    const bool tail = (rl == 15u) | (next != r.key);
    const uint32_t seg = row_incl_scan(head);
    run_step<1>(r, seg);
    run_step<2>(r, seg);
    run_step<4>(r, seg);
    run_step<8>(r, seg);
    return tail;
}

__global__ __launch_bounds__(256) void k_scan(StepArgs a) {
    __shared__ ScanLds S;
    for (int i = threadIdx.x; i < kScanSlots; i += blockDim.x) {
        S.key[i] = kNone; S.cnt[i] = 0u; S.mn[i] = 0xFFFFFFFFu; S.mx[i] = 0u;
        S.x0[i] = INT_MAX; S.y0[i] = INT_MAX; S.z0[i] = INT_MAX;
        S.x1[i] = -1; S.y1[i] = -1; S.z1[i] = -1;
    }
    const uint32_t tile = blockIdx.x;
    const int im = find_image_chunk(a.imgs, a.n_images, tile);
    const ImgDesc d = a.imgs[im];
    const uint32_t nxc = ((uint32_t)d.nx + kScanTileCols - 1u) / kScanTileCols;
    const uint32_t t = tile - d.chunk_base;
    const uint32_t rblk = t / nxc, cblk = t - rblk * nxc;
    const uint32_t rows = (uint32_t)d.nz * (uint32_t)d.ny;
    const uint32_t row0 = rblk * kScanTileRows;
    const int32_t x = (int32_t)(cblk * kScanTileCols + threadIdx.x);
    __syncthreads();
    RunRec run{0u, 0u, 0xFFFFu, 0u, x, x, 0, 0, 0, 0};
    uint32_t bad = 0u;
    if (x < d.nx && row0 < rows && im < a.n_images) {
        const uint32_t nr = min((uint32_t)kScanTileRows, rows - row0);
        const uint32_t nx = (uint32_t)d.nx;
        uint32_t lab[kScanTileRows], val[kScanTileRows];
        // the tile's first row as a uniform base; lanes add 32-bit byte
        // offsets (kScanTileRows rows of nx voxels)
        const size_t base = (size_t)row0 * nx;
        const uint32_t *Lt = d.L + base;
        const uint16_t *It = d.I + base;
#pragma unroll
        for (uint32_t j = 0; j < kScanTileRows; ++j) {
            lab[j] = 0u;
            val[j] = 0u;
            if (j < nr) {
                const uint32_t o = j * nx + (uint32_t)x;
                lab[j] = ldb(Lt, o << 2);
                val[j] = ldb(It, o << 1);
            }
        }
        // Per voxel only the label test and the count and range of the
        // current run; the run's rows [j0, j) become its box when it ends.
        // A run never crosses a plane boundary (rows of different planes are
        // not neighbours): jb, the tile row where the next plane starts, is
        // uniform.  Background runs (key 0) are counted too and never flushed.
        const uint32_t ny = (uint32_t)d.ny;
        uint32_t jb = ny - row0 % ny;
        uint32_t key = 0u, c = 0u, mn = 0xFFFFu, mx = 0u, j0 = 0u;
        const bool flat = d.nz == 1;   // a 2D image: the row is y, no division
        const auto rec = [&](uint32_t j_end) {   // rows [j0, j_end) of the run, j_end > j0
            const uint32_t r = row0 + j0, z = flat ? 0u : r / ny, y = r - z * ny;
            return RunRec{key, c, mn, mx, x, x, (int32_t)y, (int32_t)(y + (j_end - 1u - j0)), (int32_t)z, (int32_t)z};
        };
#pragma unroll
        for (uint32_t j = 0; j < kScanTileRows; ++j) {
            if (j >= nr) break;
            const uint32_t l = lab[j];
            const bool plane = j == jb;
            if (l != key || plane) {
                if (key) scan_flush_label(a, S, d, rec(j), bad);
                key = l; c = 0u; mn = 0xFFFFu; mx = 0u; j0 = j;
            }
            if (plane) jb += ny;
            ++c;
            mn = min(mn, val[j]);
            mx = max(mx, val[j]);
        }
        if (key) run = rec(nr);
    }
    // The runs still open at the tile's last row: adjacent lanes of a row
    // holding the same label are combined first, so one lane per group
    // flushes (a wide ROI would otherwise send every lane to one slot).
    if (row_segment_combine(run) && run.key) scan_flush_label(a, S, d, run, bad);
    if (bad) atomicOr(&a.counters[C_ERR], (uint32_t)E_LABEL_RANGE);
    __syncthreads();
    for (int i = threadIdx.x; i < kScanSlots; i += blockDim.x) {
        uint32_t K = S.key[i];
        if (K != kNone)
            scan_flush_global(a, K, S.cnt[i], S.mn[i], S.mx[i], S.x0[i], S.x1[i], S.y0[i], S.y1[i], S.z0[i], S.z1[i]);
    }
}

// ------------------------------------------------------------------ compaction
__global__ __launch_bounds__(1024) void k_compact_count(StepArgs a) {
    __shared__ uint32_t wc[16];
    uint32_t e = blockIdx.x * 1024u + threadIdx.x;
    bool p = e < a.tab.total && a.tab.cnt[e] > 0u;
    uint64_t m = __ballot(p);
    if (lane() == 0) wc[threadIdx.x / 64] = (uint32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < 16; ++w) s += wc[w];
        a.counters[C_BLOCKS + blockIdx.x] = s;
    }
}

// Rows are assigned in (image, label) order.  Each ROI is cut into tiles of
// bbox rows when large, and its tiles are appended to the bucket of their size
// class, so the persistent kernel can drain the largest work first.
__global__ __launch_bounds__(1024) void k_compact_write(StepArgs a, uint32_t roi_lo, uint32_t roi_hi) {
    __shared__ uint32_t wc[16], wpre[16], s_part[16], s_prefix;
    __shared__ uint32_t cls_cnt[kClasses], cls_base[kClasses];
    if (threadIdx.x < kClasses) cls_cnt[threadIdx.x] = 0u;
    uint32_t part = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += 1024u) part += a.counters[C_BLOCKS + b];
    part = wave_sum(part);
    if (lane() == 0) s_part[threadIdx.x / 64] = part;
    uint32_t e = blockIdx.x * 1024u + threadIdx.x;
    bool p = e < a.tab.total && a.tab.cnt[e] > 0u;
    uint64_t m = __ballot(p);
    if (lane() == 0) wc[threadIdx.x / 64] = (uint32_t)__popcll(m);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0, acc = 0;
        for (int w = 0; w < 16; ++w) s += s_part[w];
        s_prefix = s;
        for (int w = 0; w < 16; ++w) { wpre[w] = acc; acc += wc[w]; }
        if (blockIdx.x == gridDim.x - 1) a.counters[C_NROIS] = s + acc;
    }
    __syncthreads();
    // Every thread reaches the block-level class aggregation below.
    const uint32_t rank = (uint32_t)__popcll(m & __lanemask_lt());
    const uint32_t row = s_prefix + wpre[threadIdx.x / 64] + rank;
    bool live = p;
    if (live && row >= a.roi_cap) { atomicOr(&a.counters[C_ERR], (uint32_t)E_ROI_CAP); live = false; }
    RoiDesc rd;
    bool enq = false;
    uint32_t cls = 0u, nt = 1u, local = 0u;
    if (live) {
    const int im = find_image_entry(a.imgs, a.n_images, e);
    const uint32_t ent = e - a.imgs[im].tab_base;   // >= 1: entry 0 never counts a voxel
    const uint32_t label = a.imgs[im].dict ? a.imgs[im].dict[ent - 1u] : ent;
    rd.label = label;
    rd.image = (uint32_t)im;
    rd.n = a.tab.cnt[e];
    rd.vmin = a.tab.mn[e];
    rd.vmax = a.tab.mx[e];
    rd.x0 = a.tab.x0[e]; rd.y0 = a.tab.y0[e]; rd.z0 = a.tab.z0[e];
    rd.x1 = a.tab.x1[e]; rd.y1 = a.tab.y1[e]; rd.z1 = a.tab.z1[e];
    rd.rows = (uint32_t)(rd.z1 - rd.z0 + 1) * (uint32_t)(rd.y1 - rd.y0 + 1);
    rd.pad1 = 0u;
    a.tab.row[e] = row;
    const bool take = a.enqueue && row >= roi_lo && row < roi_hi;
    // banded ROIs get a global matrix but no work items of the batch kernel
    const bool band = a.band_vox != 0u && rd.n > a.band_vox;
    const Tiling tl = tiles_for(rd.n, rd.rows, (uint32_t)(rd.x1 - rd.x0 + 1), a.split_vox, a.tile_vox);
    nt = band ? 0u : tl.row_blocks * tl.col_blocks;
    rd.n_tiles = nt;
    rd.tcols = band ? 1u : tl.col_blocks;
    rd.gslot = kNone;
    if (take && (nt > 1u || band || a.force_split)) {
        uint32_t s = a.force_split ? row - roi_lo : atomicAdd(&a.counters[C_NSPLIT], 1u);
        if (s >= a.g_cap) {
            atomicOr(&a.counters[C_ERR], (uint32_t)E_SPLIT_CAP);
        } else {
            rd.gslot = s;
            a.split_roi[s] = row;
            if (band) a.band_roi[atomicAdd(&a.counters[C_NBAND], 1u)] = row;   // at most one per slot
        }
    }
    a.rois[row] = rd;
    if (take && !band && (rd.gslot != kNone || nt == 1u)) {
        enq = true;
        cls = size_class((rd.n + nt - 1u) / nt);
        local = atomicAdd(&cls_cnt[cls], nt);
    }
    if (a.o_label) a.o_label[row] = label;
    if (a.o_image) a.o_image[row] = (uint32_t)im;
    if (a.o_n) a.o_n[row] = rd.n;
    if (a.o_min) a.o_min[row] = (uint16_t)rd.vmin;
    if (a.o_max) a.o_max[row] = (uint16_t)rd.vmax;
    if (a.o_bbox) {
        int32_t *b = a.o_bbox + 6ull * row;
        b[0] = rd.x0; b[1] = rd.y0; b[2] = rd.z0; b[3] = rd.x1; b[4] = rd.y1; b[5] = rd.z1;
    }
    }  // live
    __syncthreads();
    if (threadIdx.x < kClasses && cls_cnt[threadIdx.x])
        cls_base[threadIdx.x] = atomicAdd(&a.counters[C_CLASS + threadIdx.x], cls_cnt[threadIdx.x]);
    __syncthreads();
    // Each ROI's tile entries: a thread writes those of its own ROI when they
    // are few; the tiles of ROIs cut into many are written by the whole
    // work-group (one thread would take milliseconds over a huge ROI).
    constexpr uint32_t kOwnTiles = 32u, kBigMax = 64u;
    __shared__ uint32_t n_big, big_row[kBigMax], big_nt[kBigMax];
    __shared__ uint2 *big_dst[kBigMax];
    if (threadIdx.x == 0) n_big = 0u;
    __syncthreads();
    if (enq) {
        uint32_t pos = cls_base[cls] + local;
        if (pos + nt > a.bucket_cap) {
            atomicOr(&a.counters[C_ERR], (uint32_t)E_ITEM_CAP);
        } else {
            uint2 *dst = a.buckets + (uint64_t)cls * a.bucket_cap + pos;
            uint32_t b = kBigMax;
            if (nt > kOwnTiles) b = atomicAdd(&n_big, 1u);
            if (b < kBigMax) {
                big_row[b] = row;
                big_nt[b] = nt;
                big_dst[b] = dst;
            } else {
                for (uint32_t t = 0; t < nt; ++t) dst[t] = make_uint2(row, t);
            }
        }
    }
    __syncthreads();
    const uint32_t nb = min(n_big, kBigMax);
    for (uint32_t b = 0; b < nb; ++b)
        for (uint32_t t = threadIdx.x; t < big_nt[b]; t += blockDim.x) big_dst[b][t] = make_uint2(big_row[b], t);
}

// In force_split mode the split-slot count is the ROI range size.
__global__ void k_set_nsplit(StepArgs a, uint32_t roi_lo, uint32_t roi_hi) {
    uint32_t n = a.counters[C_NROIS];
    uint32_t hi = roi_hi < n ? roi_hi : n;
    a.counters[C_NSPLIT] = hi > roi_lo ? hi - roi_lo : 0u;
}

// ------------------------------------------------------------------ binning
__global__ __launch_bounds__(256) void k_bin_image(StepArgs a, uint16_t *bins_out, uint64_t total_vox,
                                                   const uint64_t *img_vox_base) {
    for (uint64_t g = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; g < total_vox;
         g += (uint64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = a.n_images - 1;
        while (lo < hi) {
            int mid = (lo + hi + 1) >> 1;
            if (img_vox_base[mid] <= g) lo = mid; else hi = mid - 1;
        }
        const ImgDesc &d = a.imgs[lo];
        uint32_t v = (uint32_t)(g - img_vox_base[lo]);
        uint32_t l = d.L[v];
        uint16_t b = 0;
        const uint32_t ent = label_entry(d.dict, d.dict_n, d.max_label, l);
        if (ent) {
            uint32_t r = a.tab.row[d.tab_base + ent];
            if (r != kNone && r < a.roi_cap) {
                const RoiDesc &rd = a.rois[r];
                uint32_t D = rd.vmax - rd.vmin;
                b = (uint16_t)fbn_level(d.I[v], rd.vmin, D, D ? 1.0f / (float)D : 0.0f, (uint32_t)a.ng);
            }
        }
        bins_out[g] = b;
    }
}

// ------------------------------------------------------------------ batch
// ------------------------------------------------------------------ work queue
// Tickets follow ticket_offsets / ticket_range (nyx_types.h).  misc[64 + cl]:
// first ticket of class cl; misc[96 + cl]: its entries (clamped to the bucket
// capacity); misc[63]: number of tickets.  The class counts are loaded by
// lanes 0..kClasses-1 at once (ticket_load, every thread calls it), then one
// thread forms the offsets (ticket_prefix) after a barrier.
__device__ __forceinline__ void ticket_load(uint32_t *misc, const uint32_t *cls_cnt, uint32_t cap, uint32_t tid) {
    if (tid < (uint32_t)kClasses) misc[96 + tid] = min(cls_cnt[tid], cap);
}

__device__ void ticket_prefix(uint32_t *misc) { misc[63] = ticket_offsets(misc + 96, misc + 64); }

// Claims ticket `atomicAdd(ctr) * lanes + lane` and writes its entries as
// (roi, tile) pairs to misc[0..); returns how many (0 once the queue is
// drained).  The counters of lanes 0..lanes-1 together hand out every ticket
// once.
__device__ uint32_t ticket_claim(uint32_t *misc, uint32_t *ctr, uint32_t lane_, uint32_t lanes, const uint2 *buckets,
                                 uint32_t cap) {
    const uint32_t t = atomicAdd(ctr, 1u) * lanes + lane_;
    if (t >= misc[63]) return 0u;
    int cl;
    uint32_t e0, e1;
    ticket_range(t, misc + 96, misc + 64, &cl, &e0, &e1);
    uint32_t n = 0;
    for (uint32_t e = e0; e < e1; ++e, ++n) {
        const uint2 it = buckets[(uint32_t)cl * cap + e];
        misc[2 * n] = it.x;
        misc[2 * n + 1] = it.y;
    }
    return n;
}

struct ItemCtx {
    const uint16_t *I;
    const uint32_t *L;
    const uint16_t *B;
    int32_t nx, ny, nz;
    uint32_t label, vmin, ng;
    double rcp;       // 1 / max(vmax - vmin, 1), rounded up (fbn_level_rd)
    uint32_t *err;
    // The stored value under voxel v (bin or intensity) and its level, split
    // so a caller can issue many loads before converting any of them.  A
    // caller-supplied bin image is clamped to [1, ng] (flagging the error) so
    // no LDS address can leave its triangle.
    __device__ __forceinline__ uint32_t raw(uint32_t v) const {
        return B ? (uint32_t)ldg(B, v) : (uint32_t)ldg(I, v);
    }
    __device__ __forceinline__ uint32_t lab(uint32_t v) const { return ldg(L, v); }
    __device__ __forceinline__ uint32_t level_of(uint32_t r) const {
        if (!B) return fbn_level_rd(r, vmin, rcp, ng);
        if (r == 0u || r > ng) {
            atomicOr(err, (uint32_t)E_BIN_RANGE);
            r = r == 0u ? 1u : ng;
        }
        return r;
    }
};

// One queue entry with everything its processing reads: written to LDS by
// one thread per entry when the ticket is claimed (the descriptor loads of a
// whole ticket overlap), then read by every wave as uniform values.
struct ItemDesc {
    RoiDesc rd;
    const uint16_t *I;
    const uint32_t *L;
    const uint16_t *B;
    int32_t nx, ny, nz;
    uint32_t roi;                   // kNone: the entry names no valid ROI tile (skipped)
    uint32_t ra, rb, ca, cb;        // bbox rows [ra, rb) and columns [ca, cb) of the tile
    double rcp;                     // 1 / max(vmax - vmin, 1), rounded up (fbn_level_rd)
};
static_assert(sizeof(ItemDesc) <= kItemBytes, "staged descriptor exceeds its LDS slot");

__device__ void stage_item(const StepArgs &a, uint32_t roi, uint32_t tile, ItemDesc *dst) {
    ItemDesc it;
    it.roi = kNone;
    if (roi < a.roi_cap) {
        const RoiDesc rd = a.rois[roi];
        it.rd = rd;
        if (tile < rd.n_tiles && rd.image < (uint32_t)a.n_images) {
            const ImgDesc im = a.imgs[rd.image];
            if (!(rd.x0 < 0 || rd.y0 < 0 || rd.z0 < 0 || rd.x1 >= im.nx || rd.y1 >= im.ny || rd.z1 >= im.nz ||
                  rd.x0 > rd.x1 || rd.y0 > rd.y1 || rd.z0 > rd.z1 || rd.tcols == 0u)) {
                it.I = im.I; it.L = im.L; it.B = im.B;
                it.nx = im.nx; it.ny = im.ny; it.nz = im.nz;
                tile_bounds(rd.rows, (uint32_t)(rd.x1 - rd.x0 + 1), rd.n_tiles, rd.tcols, tile, &it.ra, &it.rb,
                            &it.ca, &it.cb);
                const uint32_t D = rd.vmax - rd.vmin;
                it.rcp = fbn_rcp_up(D ? D : 1u);
                it.roi = roi;
            }
        }
    }
    *dst = it;
}

// A work-group-uniform copy of an LDS object, held in scalar registers.
template <class T> __device__ __forceinline__ T lds_uniform(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "word-sized objects only");
    T out;
    const uint32_t *s = reinterpret_cast<const uint32_t *>(p);
    uint32_t *o = reinterpret_cast<uint32_t *>(&out);
#pragma unroll
    for (uint32_t i = 0; i < sizeof(T) / 4; ++i) o[i] = __builtin_amdgcn_readfirstlane(s[i]);
    return out;
}

// Triangle offset of a 1-based level x: the index of cell (lo, hi = x - 1)
// is row_off(x) + lo + 1, so a pair (a <= b) lands at row_off(b) + a.
__device__ __forceinline__ uint32_t row_off(uint32_t x) { return (__umul24(x - 1u, x) >> 1) - 1u; }
struct RowOff {
    __device__ __forceinline__ uint32_t operator()(uint32_t x) const { return row_off(x); }
};
// No triangle row offsets (adders that index by the levels alone).
struct NoRowOff {
    __device__ __forceinline__ uint32_t operator()(uint32_t) const { return 0u; }
};
// The same offsets read from an LDS table of levels 0..ng (entry 0 unused).
struct RowOffTab {
    const uint32_t *t;
    __device__ __forceinline__ uint32_t operator()(uint32_t x) const { return t[x]; }
};
// Square (ordered counts) offset of a 1-based level x: the ordered pair
// (a, b) lands at sq_off(a) + b = (a - 1) ng + b - 1.
struct SqOff {
    uint32_t ng;
    __device__ __forceinline__ uint32_t operator()(uint32_t x) const { return __umul24(x - 1u, ng) - 1u; }
};

// i >> 1 as an opaque shift: the compiler would otherwise fold the word
// address (i >> 1) * 4 + base into three operations instead of two.
__device__ __forceinline__ uint32_t half_index(uint32_t i) {
    uint32_t w;
    asm("v_lshrrev_b32 %0, 1, %1" : "=v"(w) : "v"(i));
    return w;
}

// Add one level pair (1-based la, lb, with their row offsets ta, tb) to
// local direction dl: unordered into the triangle (SQ false), or ordered
// (la at v, lb at v + d) into the square of ordered counts (SQ true; ta from
// SqOff, hash keys keep the order).
template <int MODE, bool SQ = false>
__device__ __forceinline__ void add_pair(const StepArgs &a, uint8_t *smem, uint32_t dl, uint32_t la, uint32_t ta,
                                         uint32_t lb, uint32_t tb) {
    const LdsLayout &Ly = a.lds;
    uint32_t lo = (SQ || la < lb ? la : lb) - 1u, hi = (SQ || la < lb ? lb : la) - 1u;
    uint32_t *LCNT = reinterpret_cast<uint32_t *>(smem + Ly.lcnt_off);
    uint32_t *LST = reinterpret_cast<uint32_t *>(smem + Ly.list_off) + dl * Ly.list_cap;
    if (MODE == 2 || MODE == 3) {
        // privatised copies: lane l adds to copy l mod copies (copies is a power
        // of two); 24-bit multiply (full rate): both factors are small
        const uint32_t cp = Ly.copies > 1u ? (uint32_t)lane() & (Ly.copies - 1u) : 0u;
        uint32_t *U = reinterpret_cast<uint32_t *>(smem + Ly.u_off) + __umul24(dl * Ly.copies + cp, Ly.tri_pad);
        // the triangle index of the unordered pair is the larger of the two
        // candidates: row_off(b) + a - (row_off(a) + b) = sum over x in [a, b)
        // of (x - 1) >= 0 for 1 <= a <= b, so no comparison of the levels
        const uint32_t i = SQ ? ta + lb : max(tb + la, ta + lb);
        if (MODE == 2)
            __hip_atomic_fetch_add(&U[i], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
            __hip_atomic_fetch_add(&U[half_index(i)], 1u << ((i & 1u) << 4), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
    } else if (MODE == 0) {
        uint32_t *U = reinterpret_cast<uint32_t *>(smem + Ly.u_off) + dl * Ly.tri_pad;
        uint32_t old = atomicAdd(&U[tri_idx(lo, hi)], 1u);
        bool fresh = old == 0u;
        uint64_t m = __ballot(fresh);
        if (m) {
            int leader = __ffsll((unsigned long long)m) - 1;
            uint32_t base = 0;
            if (lane() == leader) base = atomicAdd(&LCNT[dl], (uint32_t)__popcll(m));
            base = __shfl(base, leader);
            if (fresh) {
                uint32_t pos = base + (uint32_t)__popcll(m & __lanemask_lt());
                if (pos < Ly.list_cap) LST[pos] = lo | (hi << 16);
                else atomicOr(&a.counters[C_ERR], (uint32_t)E_LIST_CAP);
            }
        }
    } else {
        uint32_t *HK = reinterpret_cast<uint32_t *>(smem + Ly.hkey_off);
        uint32_t *HC = reinterpret_cast<uint32_t *>(smem + Ly.hcnt_off);
        const uint32_t key = (dl << 26) | (hi << 13) | lo;
        const uint32_t mask = Ly.hash_cap - 1u;
        uint32_t h = hash_u32(key) & mask;
        bool done = false;
        for (uint32_t probe = 0; probe < Ly.hash_cap; ++probe) {
            uint32_t cur = atomicCAS(&HK[h], kNone, key);
            if (cur == kNone || cur == key) {
                atomicAdd(&HC[h], 1u);
                if (cur == kNone) {
                    uint32_t pos = atomicAdd(&LCNT[dl], 1u);
                    if (pos < Ly.list_cap) LST[pos] = h;
                    else atomicOr(&a.counters[C_ERR], (uint32_t)E_LIST_CAP);
                }
                done = true;
                break;
            }
            h = (h + 1u) & mask;
        }
        if (!done) atomicOr(&a.counters[C_ERR], (uint32_t)E_HASH_FULL);
    }
}

constexpr uint32_t kStagedMinRows = 4;   // fewer rows per ring chunk: gather instead
constexpr uint32_t kStageBatch = 8;      // voxels staged per lane and round
constexpr int kStagedDirs = 13;          // neighbour levels read per group

// Offset d with the sign that makes it point forward in raster order (z,
// then y, then x).  Counts are symmetric, so (v, v + d) and (v, v - d) name
// the same unordered pairs.
__device__ __forceinline__ void forward_offset(const StepArgs &a, int d, int32_t &dz, int32_t &dy, int32_t &dx) {
    dz = a.off[d][0]; dy = a.off[d][1]; dx = a.off[d][2];
    if (dz < 0 || (dz == 0 && (dy < 0 || (dy == 0 && dx < 0)))) { dz = -dz; dy = -dy; dx = -dx; }
}

// Largest forward distance, in flattened bbox rows (z * H + y), from a voxel
// to a neighbour of [d0, d1) that can lie in the bbox (|dy| < H, |dx| < W).
__device__ __forceinline__ uint32_t staged_reach(const StepArgs &a, int d0, int d1, uint32_t H, uint32_t W) {
    uint32_t m = 0u;
    for (int d = d0; d < d1; ++d) {
        int32_t dz, dy, dx;
        forward_offset(a, d, dz, dy, dx);
        if ((uint32_t)abs(dy) >= H || (uint32_t)abs(dx) >= W) continue;
        m = max(m, (uint32_t)(dz * (int32_t)H + dy));
    }
    return m;
}

// Staged accumulation for offsets the row sweep does not cover (volumes,
// longer distances), over full-width tiles: rows [ra, rb) are taken in
// chunks of C = ring_rows - reach rows.  Before a chunk, the levels of the
// rows it reaches that are not yet staged are written once to an LDS ring of
// ring_rows x W bytes (0 outside the ROI or past the bbox); every pair then
// reads both levels from the ring, so each voxel is loaded and binned once
// per pass instead of once per offset that reaches it.  Levels fit a byte
// (ng <= 255).
template <class Add>
__device__ void accumulate_staged(const StepArgs &a, const RoiDesc &rd, const ItemCtx &c, uint32_t ra, uint32_t rb,
                                  int d0, int d1, uint8_t *ring, uint32_t ring_rows, uint32_t reach, Add &&add) {
    const uint32_t W = (uint32_t)(rd.x1 - rd.x0 + 1), H = (uint32_t)(rd.y1 - rd.y0 + 1), rows = rd.rows;
    const uint32_t C = ring_rows - reach;
    const uint32_t plane = (uint32_t)c.ny * (uint32_t)c.nx;
    const uint32_t t0 = threadIdx.x, ts = blockDim.x;
    const uint32_t dq = ts / W, dxo = ts - dq * W;
    // Walks (row r, its ring slot, its (z, y), column x) by ts voxels.
    struct Pos {
        uint32_t r, slot, z, y, x;
    };
    const auto start = [&](uint32_t r_first) {
        Pos p;
        p.x = t0 % W;
        p.r = r_first + t0 / W;
        p.slot = (p.r - ra) % ring_rows;
        p.z = p.r / H;
        p.y = p.r - p.z * H;
        return p;
    };
    const auto advance = [&](Pos &p) {
        p.x += dxo;
        uint32_t adv = dq;
        if (p.x >= W) { p.x -= W; ++adv; }
        p.r += adv;
        p.slot += adv;
        if (p.slot >= ring_rows) p.slot %= ring_rows;
        p.y += adv;
        if (p.y >= H) {
            const uint32_t k = p.y / H;
            p.z += k;
            p.y -= k * H;
        }
    };
    uint32_t staged = ra;   // rows [ra, staged) are in the ring
    for (uint32_t r0 = ra; r0 < rb; r0 += C) {
        const uint32_t r1 = min(r0 + C, rb), s1 = r1 + reach;
        {
            // kStageBatch voxels per lane and round: their loads are all in
            // flight before the first level is formed
            const uint32_t n = (s1 - staged) * W;
            Pos p = start(staged);
            for (uint32_t f = t0; f < n; f += ts * kStageBatch) {
                uint32_t lab[kStageBatch], val[kStageBatch], at[kStageBatch];
#pragma unroll
                for (uint32_t k = 0; k < kStageBatch; ++k) {
                    lab[k] = 0u;
                    val[k] = 0u;
                    at[k] = kNone;
                    if (f + k * ts < n) {
                        at[k] = __umul24(p.slot, W) + p.x;
                        if (p.r < rows) {
                            const uint32_t v = (uint32_t)(rd.z0 + (int32_t)p.z) * plane +
                                               (uint32_t)(rd.y0 + (int32_t)p.y) * (uint32_t)c.nx +
                                               (uint32_t)(rd.x0 + (int32_t)p.x);
                            lab[k] = c.lab(v);
                            val[k] = c.raw(v);
                        }
                    }
                    advance(p);
                }
#pragma unroll
                for (uint32_t k = 0; k < kStageBatch; ++k)
                    if (at[k] != kNone) ring[at[k]] = (uint8_t)(lab[k] == c.label ? c.level_of(val[k]) : 0u);
            }
        }
        staged = s1;
        __syncthreads();
        {
            const uint32_t n = (r1 - r0) * W;
            Pos p = start(r0);
            // two voxels per lane in flight: their neighbour reads are all
            // issued before the first pair add
            for (uint32_t f = t0; f < n; f += 2u * ts) {
                Pos q = p;
                advance(q);
                const bool second = f + ts < n;
                const uint32_t lv0 = ring[__umul24(p.slot, W) + p.x];
                const uint32_t lv1 = second ? (uint32_t)ring[__umul24(q.slot, W) + q.x] : 0u;
                if (lv0 | lv1) {
                    const uint32_t tv0 = row_off(lv0), tv1 = row_off(lv1);
                    for (int db = d0; db < d1; db += kStagedDirs) {
                        uint32_t lw0[kStagedDirs], lw1[kStagedDirs];
#pragma unroll
                        for (int k = 0; k < kStagedDirs; ++k) {
                            lw0[k] = 0u;
                            lw1[k] = 0u;
                            const int d = db + k;
                            if (d < d1) {
                                int32_t dz, dy, dx;
                                forward_offset(a, d, dz, dy, dx);
                                const uint32_t dr = (uint32_t)(dz * (int32_t)H + dy);
                                const uint32_t yy0 = p.y + (uint32_t)dy, xx0 = p.x + (uint32_t)dx;
                                if (lv0 && yy0 < H && xx0 < W) {
                                    uint32_t s2 = p.slot + dr;
                                    if (s2 >= ring_rows) s2 -= ring_rows;
                                    lw0[k] = ring[__umul24(s2, W) + xx0];
                                }
                                const uint32_t yy1 = q.y + (uint32_t)dy, xx1 = q.x + (uint32_t)dx;
                                if (lv1 && yy1 < H && xx1 < W) {
                                    uint32_t s2 = q.slot + dr;
                                    if (s2 >= ring_rows) s2 -= ring_rows;
                                    lw1[k] = ring[__umul24(s2, W) + xx1];
                                }
                            }
                        }
#pragma unroll
                        for (int k = 0; k < kStagedDirs; ++k) {
                            if (lw0[k]) add((uint32_t)(db + k - d0), lv0, tv0, lw0[k], row_off(lw0[k]));
                            if (lw1[k]) add((uint32_t)(db + k - d0), lv1, tv1, lw1[k], row_off(lw1[k]));
                        }
                    }
                }
                p = q;
                advance(p);
            }
        }
        __syncthreads();
    }
}

// Accumulate the pairs owned by the voxels of bbox rows [ra, rb) (rows of
// all planes, flattened) and columns [ca, cb) for the directions [d0, d1):
// each voxel owns the pair (v, v + d) of each offset.  Lanes take voxels
// t0, t0 + ts, ...; for each voxel the label and value of the voxel and of up
// to kGatherDirs neighbours are loaded in one batch before any is used.
constexpr int kGatherDirs = 8;

template <class Add, class Off = RowOff>
__device__ void accumulate_rows(const StepArgs &a, const RoiDesc &rd, const ItemCtx &c, uint32_t ra, uint32_t rb,
                                uint32_t ca, uint32_t cb, int d0, int d1, uint32_t t0, uint32_t ts, Add &&add,
                                Off off = Off{}) {
    const uint32_t W = cb - ca, H = (uint32_t)(rd.y1 - rd.y0 + 1);
    const uint32_t nv = (rb - ra) * W;
    const uint32_t plane = (uint32_t)c.ny * (uint32_t)c.nx;
    // voxel f = t0 + k ts of the tile: column xo = f % W, row ra + f / W of
    // the flattened bbox rows (plane zq, row yo), advanced incrementally
    const uint32_t dq = ts / W, dxo = ts - dq * W;
    uint32_t xo = t0 % W, yo = ra + t0 / W, zq = 0;
    if (yo >= H) { zq = yo / H; yo -= zq * H; }
    for (uint32_t f = t0; f < nv; f += ts) {
        const int32_t x = rd.x0 + (int32_t)(ca + xo);
        const int32_t y = rd.y0 + (int32_t)yo;
        const int32_t z = rd.z0 + (int32_t)zq;
        const uint32_t v = (uint32_t)z * plane + (uint32_t)y * (uint32_t)c.nx + (uint32_t)x;
        uint32_t lv = c.lab(v), rv = c.raw(v);
        for (int db = d0; db < d1; db += kGatherDirs) {
            uint32_t nl[kGatherDirs], nr[kGatherDirs];
#pragma unroll
            for (int k = 0; k < kGatherDirs; ++k) {
                nl[k] = 0u;
                nr[k] = 0u;
                // a uniform index keeps the offset table reads scalar
                const int d = __builtin_amdgcn_readfirstlane(db + k);
                if (d < d1) {
                    const int32_t wz = z + a.off[d][0], wy = y + a.off[d][1], wx = x + a.off[d][2];
                    if (wz >= 0 && wz < c.nz && wy >= 0 && wy < c.ny && wx >= 0 && wx < c.nx) {
                        const uint32_t wv = (uint32_t)wz * plane + (uint32_t)wy * (uint32_t)c.nx + (uint32_t)wx;
                        nl[k] = c.lab(wv);
                        nr[k] = c.raw(wv);
                    }
                }
            }
            // every load of the group is issued before the first use
            asm volatile("" : "+v"(lv), "+v"(rv));
            if (lv != c.label) continue;
            const uint32_t bv = c.level_of(rv);
#pragma unroll
            for (int k = 0; k < kGatherDirs; ++k)
                if (db + k < d1 && nl[k] == c.label) {
                    const uint32_t bw = c.level_of(nr[k]);
                    add((uint32_t)(db + k - d0), bv, off(bv), bw, off(bw));
                }
        }
        xo += dxo;
        uint32_t adv = dq;
        if (xo >= W) { xo -= W; ++adv; }
        yo += adv;
        if (yo >= H) {
            const uint32_t k2 = yo / H;
            zq += k2;
            yo -= k2 * H;
        }
    }
}

// 2D distance-1 accumulation by row sweep.  A wavefront is split into S
// sub-rows of Wl = 64/S lanes (S = 1, 2 or 4, chosen per item to need the
// fewest steps for the tile's width); each step covers S consecutive image
// rows of a strip of Wl - 1 owned columns (the last lane of a sub-row only
// supplies the right neighbour).  A unit of kSweepSteps steps loads the labels
// and values of all its rows, and of the row above it, in one batch, so it
// costs a single round trip to memory; levels of the row above come from the
// sub-row above in the same step (one lane permute), or from the last
// sub-row's previous step, and right neighbours from the next lane by a DPP
// wave shift.  Owned pairs per lane (column x, row y):
//   H    (y, x)-(y, x+1)      V    (y, x)-(y-1, x)
//   D45  (y, x)-(y-1, x+1)    D135 (y-1, x)-(y, x+1)
// h, v, d45, d135 are the local direction slots of the four classes (-1: not
// in this pass).  Units (strip x block of rows) are dealt to the nw
// wavefronts round robin; w is the caller's index among them.
constexpr uint32_t kSweepSteps = 8;

__device__ __forceinline__ uint32_t lane_next(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130, 0xF, 0xF, true);  // wave_shl1; lane 63 reads 0
}

// BINS: levels from a caller-supplied bin image (else from intensity); ro:
// the triangle row offsets of the levels.
template <bool BINS, class RO, class Add>
__device__ void accumulate_sweep2d(const RoiDesc &rd, const ItemCtx &c, uint32_t ra, uint32_t rb, uint32_t ca,
                                   uint32_t cb, int h, int v, int d45, int d135, int w, int nw, RO ro, Add &&add) {
    // a voxel's level, 0 outside the ROI: computed for every lane and then
    // selected by label (no branch per voxel)
    const auto level = [&](uint32_t lab, uint32_t raw) -> uint32_t {
        if constexpr (BINS) {
            return lab == c.label ? c.level_of(raw) : 0u;
        } else {
            const uint32_t b = fbn_level_rd(raw, c.vmin, c.rcp, c.ng);
            return lab == c.label ? b : 0u;
        }
    };
    const uint16_t *const V = BINS ? c.B : c.I;   // the stored values (bins or intensity)
    const uint32_t ln = (uint32_t)lane();
    const uint32_t Wt = cb - ca, H = rb - ra;
    // sub-rows per step: the fewest steps over the tile (ties: fewer sub-rows)
    uint32_t lg = 0, best = ((Wt + 62u) / 63u) * H;
    for (uint32_t q = 1; q <= 2u; ++q) {
        const uint32_t wo = (64u >> q) - 1u;
        const uint32_t steps = ((Wt + wo - 1u) / wo) * ((H + (1u << q) - 1u) >> q);
        if (steps < best) { best = steps; lg = q; }
    }
    const uint32_t S = 1u << lg, Wl = 64u >> lg, Wo = Wl - 1u;
    const uint32_t sub = ln >> (6u - lg), col = ln & (Wl - 1u);
    // (constant divisors: no division sequence per item)
    const uint32_t nstrip = lg == 0u ? (Wt + 62u) / 63u : (lg == 1u ? (Wt + 30u) / 31u : (Wt + 14u) / 15u);
    // steps per unit: kSweepSteps, or fewer (at least 2) when a small tile
    // would otherwise leave some of the nw wavefronts without a unit (nw is
    // a power of two: work-groups are 256 threads)
    uint32_t su = (((H + S - 1u) >> lg) * nstrip + (uint32_t)nw - 1u) >> __builtin_ctz((uint32_t)nw);
    su = su < 2u ? 2u : (su > kSweepSteps ? kSweepSteps : su);
    const uint32_t unit_rows = su * S;
    // row blocks ceil(H / unit_rows): single-precision estimate, one correction
    const uint32_t nrows_up = H + unit_rows - 1u;   // < 2^17: exact in single precision
    uint32_t nblk = (uint32_t)((float)nrows_up * __builtin_amdgcn_rcpf((float)unit_rows));
    if (nblk * unit_rows > nrows_up) --nblk;
    else if ((nblk + 1u) * unit_rows <= nrows_up) ++nblk;
    const uint32_t units = nstrip * nblk;
    const int32_t xt0 = rd.x0 + (int32_t)ca, xt1 = rd.x0 + (int32_t)cb;   // owned columns [xt0, xt1)
    const uint32_t nx = (uint32_t)c.nx;
    const uint32_t up_lane = ((ln - Wl) & 63u) << 2;   // byte index of the lane above (permute address)
    // unit u is strip s = u mod nstrip of row block ch = u / nstrip, walked
    // incrementally (no division per unit)
    uint32_t s = (uint32_t)w, ch = 0u;
    while (s >= nstrip) { s -= nstrip; ++ch; }
    for (uint32_t u = (uint32_t)w; u < units; u += (uint32_t)nw) {
        if (u != (uint32_t)w) {
            s += (uint32_t)nw;
            while (s >= nstrip) { s -= nstrip; ++ch; }
        }
        const int32_t x = xt0 + (int32_t)(Wo * s + col);
        const bool xin = x < c.nx && x <= xt1;   // owned columns and the right neighbour of the last
        const bool owner = col < Wo && x < xt1;
        const uint32_t r0 = ra + ch * unit_rows, nr = min(rb - r0, unit_rows);
        const int32_t y0 = rd.y0 + (int32_t)r0;
        // step j: image row y0 + j S + sub; the last sub-row also fetches the
        // row above the unit (its "previous step")
        uint32_t lab[kSweepSteps], val[kSweepSteps], lab_up = 0u, val_up = 0u;
        // the unit's row y0 as a uniform base; lanes add 32-bit byte offsets
        // (at most (kSweepSteps * 4 + 1) rows of nx voxels)
        const size_t row0 = (size_t)(uint32_t)y0 * nx;
        const uint32_t *Lu = c.L + row0;
        const uint16_t *Vu = V + row0;
        const uint32_t o0 = sub * nx + (uint32_t)x;
        if (xin && sub == S - 1u && y0 > rd.y0) {
            lab_up = ldb(Lu - nx, (uint32_t)x << 2);
            val_up = ldb(Vu - nx, (uint32_t)x << 1);
        }
#pragma unroll
        for (uint32_t j = 0; j < kSweepSteps; ++j) {
            lab[j] = 0u;
            val[j] = 0u;
            if (xin && j * S + sub < nr) {
                const uint32_t o = o0 + j * S * nx;
                lab[j] = ldb(Lu, o << 2);
                val[j] = ldb(Vu, o << 1);
            }
        }
        uint32_t prev = level(lab_up, val_up);   // this lane's previous step
#pragma unroll
        for (uint32_t j = 0; j < kSweepSteps; ++j) {
            if (j * S >= nr) break;
            const uint32_t cur = level(lab[j], val[j]);
            uint32_t above = prev;
            if (S > 1u) {
                const uint32_t offer = sub == S - 1u ? prev : cur;
                above = (uint32_t)__builtin_amdgcn_ds_bpermute((int)up_lane, (int)offer);
            }
            const uint32_t tcur = ro(cur), tabove = ro(above);
            const uint32_t cur_r = lane_next(cur), above_r = lane_next(above);
            const uint32_t tcur_r = lane_next(tcur), tabove_r = lane_next(tabove);
            if (owner && cur) {
                if (h >= 0 && cur_r) add((uint32_t)h, cur, tcur, cur_r, tcur_r);
                if (v >= 0 && above) add((uint32_t)v, cur, tcur, above, tabove);
                if (d45 >= 0 && above_r) add((uint32_t)d45, cur, tcur, above_r, tabove_r);
            }
            if (owner && above && cur_r && d135 >= 0) add((uint32_t)d135, above, tabove, cur_r, tcur_r);
            prev = cur;
        }
    }
}

// One direction of a finished item: features (unsplit ROI) or a 64-bit
// atomic merge into the ROI's global matrix (tile of a split ROI).
template <class Acc, bool NS, class Src>
__device__ __forceinline__ void dir_or_flush(const StepArgs &a, const WaveGrp &g, const Src &s, bool split,
                                             const RoiDesc &rd, uint32_t roi, int d, uint32_t *MARG, uint32_t ng) {
    if (split) {
        uint64_t *G = a.G + ((uint64_t)rd.gslot * a.K_out + d) * (uint64_t)ng * ng;
        s.for_each(g, [&](uint32_t lo, uint32_t hi, uint32_t c) {
            atomicAdd(reinterpret_cast<unsigned long long *>(&G[(uint64_t)lo * ng + hi]), (unsigned long long)c);
        });
        g.sync();
        s.clear(g);
        g.sync();
    } else if constexpr (NS) {
        // marginals: row, column, sum, difference
        const uint64_t at = (uint64_t)roi * a.K_out + d;
        dir_sums_ns<Acc>(g, s, MARG, MARG + ng, MARG + 2u * ng, MARG + 4u * ng - 1u, ng, a.dsums + at, a.dsums_y + at);
    } else {
        dir_sums<Acc, double>(g, s, MARG, MARG + ng, MARG + 3u * ng - 1u, ng, a.dsums + (uint64_t)roi * a.K_out + d);
    }
}

// Single precision: at most 102 VGPRs, five waves per SIMD (a few bytes of
// spill at item level; measured faster than four), which with ~30 KB of LDS
// per work-group at 64 levels keeps five work-groups on a CU; double
// precision keeps its registers.  NS: ordered (non-symmetric) counts, a
// separate instantiation so the symmetric kernel carries none of its code
// (and none of its registers).  BS: threads per work-group, 256, or 512 for
// layouts whose LDS leaves room for one work-group per CU only (eight waves
// instead of four then share the CU's latency).
template <int MODE, class OutT, bool NS, int BS>
__global__ __launch_bounds__(BS, ((BS == 256 && sizeof(OutT) == 4) ? 5 : 1)) void k_batch(StepArgs a,
                                                                                      uint32_t direct_roi) {
    extern __shared__ __align__(16) uint8_t smem[];
    typedef typename std::conditional<sizeof(OutT) == 8, double, float>::type Acc;
    const LdsLayout &Ly = a.lds;
    uint32_t *LCNT = reinterpret_cast<uint32_t *>(smem + Ly.lcnt_off);
    uint32_t *LST = reinterpret_cast<uint32_t *>(smem + Ly.list_off);
    uint32_t *BUF = reinterpret_cast<uint32_t *>(smem + Ly.buf_off);
    uint32_t *MISC = reinterpret_cast<uint32_t *>(smem + Ly.misc_off);
    ItemDesc *ITEMS = reinterpret_cast<ItemDesc *>(smem + Ly.item_off);
    const int nw = (int)(blockDim.x / kWave);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));   // wave index: uniform
    const int K = a.K;
    const uint32_t ng = (uint32_t)a.ng;
    constexpr bool ns = NS;   // ordered counts: squares, gather accumulation, four marginals
    const uint32_t marg_words = (ns ? 5u : 4u) * ng;
    uint32_t *MARG = reinterpret_cast<uint32_t *>(smem + Ly.marg_off) + w * marg_words;

    // LDS starts clean and every item leaves it clean.
    if (MODE != 1) {
        uint32_t *U = reinterpret_cast<uint32_t *>(smem + Ly.u_off);
        for (uint32_t i = threadIdx.x; i < Ly.n_tri * Ly.copies * Ly.tri_pad; i += blockDim.x) U[i] = 0u;
    } else {
        uint32_t *HK = reinterpret_cast<uint32_t *>(smem + Ly.hkey_off);
        uint32_t *HC = reinterpret_cast<uint32_t *>(smem + Ly.hcnt_off);
        for (uint32_t i = threadIdx.x; i < Ly.hash_cap; i += blockDim.x) { HK[i] = kNone; HC[i] = 0u; }
    }
    // marginal sets exist for the waves that reduce a direction (w < kp)
    for (uint32_t i = threadIdx.x; i < Ly.marg_sets * marg_words; i += blockDim.x)
        reinterpret_cast<uint32_t *>(smem + Ly.marg_off)[i] = 0u;
    for (uint32_t i = threadIdx.x; i < Ly.kp; i += blockDim.x) LCNT[i] = 0u;
    if ((MODE == 2 || MODE == 3) && !NS)
        for (uint32_t x = threadIdx.x; x <= ng; x += blockDim.x)
            reinterpret_cast<uint32_t *>(smem + Ly.ro_off)[x] = x ? row_off(x) : 0u;
    if (direct_roi == kNone) ticket_load(MISC, a.counters + C_CLASS, a.bucket_cap, threadIdx.x);
    __syncthreads();
    if (threadIdx.x == 0 && direct_roi == kNone) ticket_prefix(MISC);
    __syncthreads();

    for (uint32_t iter = 0;; ++iter) {
        if (threadIdx.x == 0) {
            uint32_t n = 0;
            if (direct_roi != kNone) {
                if (iter == 0 && direct_roi < a.roi_cap && blockIdx.x < a.rois[direct_roi].n_tiles) {
                    MISC[0] = direct_roi;
                    MISC[1] = blockIdx.x;
                    n = 1;
                }
            } else {
                // (every lane has a work-group: a grid below kTicketLanes uses fewer)
                const uint32_t lanes = min(kTicketLanes, gridDim.x), tl = blockIdx.x % lanes;
                n = ticket_claim(MISC, &a.counters[C_TICKETS + tl * kTicketStride], tl, lanes, a.buckets,
                                 a.bucket_cap);
            }
            MISC[32] = n;
        }
        __syncthreads();
        // queue entries are work-group uniform: their staged descriptors are
        // read into scalar registers
        const uint32_t n_items = __builtin_amdgcn_readfirstlane(MISC[32]);
        if (n_items == 0u) break;
        if (threadIdx.x < n_items) stage_item(a, MISC[2 * threadIdx.x], MISC[2 * threadIdx.x + 1], ITEMS + threadIdx.x);
        __syncthreads();
        for (uint32_t q = 0; q < n_items; ++q) {
            // an entry that does not name a valid ROI tile is skipped
            if (__builtin_amdgcn_readfirstlane(ITEMS[q].roi) == kNone) continue;
            const ItemDesc it = lds_uniform(ITEMS + q);
            const RoiDesc &rd = it.rd;
            const uint32_t roi = it.roi;
            ItemCtx c;
            c.I = it.I; c.L = it.L; c.B = it.B;
            c.nx = it.nx; c.ny = it.ny; c.nz = it.nz;
            c.label = rd.label; c.vmin = rd.vmin; c.ng = ng;
            c.rcp = it.rcp;
            c.err = &a.counters[C_ERR];
            const uint32_t ra = it.ra, rb = it.rb, ca = it.ca, cb = it.cb;
            const bool split = rd.gslot != kNone;
            for (int d0 = 0, pass = 0; d0 < K; d0 += (int)Ly.kp, ++pass) {
                const int d1 = min(K, d0 + (int)Ly.kp);
                if constexpr (NS) {
                    // ordered pairs (level at v, level at v + d) by gather, into squares
                    if (MODE != 0 && ra < rb && ca < cb) {
                        const bool merged = MODE >= 2 && a.merged;
                        auto add = [&](uint32_t dl, uint32_t la, uint32_t ta, uint32_t lb, uint32_t tb) {
                            add_pair<MODE, true>(a, smem, merged ? 0u : dl, la, ta, lb, tb);
                        };
                        accumulate_rows(a, rd, c, ra, rb, ca, cb, d0, d1, threadIdx.x, blockDim.x, add, SqOff{ng});
                    }
                } else if (ra < rb && ca < cb) {
                    // merged matrices: every offset counts into the one triangle
                    const bool merged = MODE >= 2 && a.merged;
                    auto add = [&](uint32_t dl, uint32_t la, uint32_t ta, uint32_t lb, uint32_t tb) {
                        add_pair<MODE>(a, smem, merged ? 0u : dl, la, ta, lb, tb);
                    };
                    const uint32_t W = (uint32_t)(rd.x1 - rd.x0 + 1), H = (uint32_t)(rd.y1 - rd.y0 + 1);
                    const uint32_t ring_rows = Ly.ring_bytes / W;
                    const uint32_t reach = Ly.ring_bytes ? staged_reach(a, d0, d1, H, W) : 0u;
                    if (a.sweep_ok && pass < kMaxSweepPasses && !c.B) {
                        // (a caller-supplied bin image takes the gather below)
                        const int8_t *sw = a.sweep[pass];
                        if constexpr (MODE == 2 || MODE == 3) {
                            const RowOffTab ro{reinterpret_cast<const uint32_t *>(smem + Ly.ro_off)};
                            accumulate_sweep2d<false>(rd, c, ra, rb, ca, cb, sw[0], sw[1], sw[2], sw[3], w, nw, ro, add);
                        } else {
                            accumulate_sweep2d<false>(rd, c, ra, rb, ca, cb, sw[0], sw[1], sw[2], sw[3], w, nw, RowOff{},
                                                      add);
                        }
                    } else if (MODE != 1 && Ly.ring_bytes && ca == 0u && cb == W && ring_rows >= reach + kStagedMinRows) {
                        // (the hash layout reserves no ring)
                        if constexpr (MODE != 1)
                            accumulate_staged(a, rd, c, ra, rb, d0, d1, smem + Ly.ring_off, ring_rows, reach, add);
                    } else
                        accumulate_rows(a, rd, c, ra, rb, ca, cb, d0, d1, threadIdx.x, blockDim.x, add);
                }
                __syncthreads();
                const int n_mat = (MODE >= 2 && a.merged) ? 1 : d1 - d0;
                for (int dl = w; dl < n_mat; dl += nw) {
                    uint32_t *Ud = reinterpret_cast<uint32_t *>(smem + Ly.u_off) + dl * Ly.copies * Ly.tri_pad;
                    const uint32_t n = min(LCNT[dl], Ly.list_cap);
                    const uint32_t *lst = LST + dl * Ly.list_cap;
                    WaveGrp g;
                    if (MODE == 2 || MODE == 3) {
                        SrcTriScan<MODE == 3> s{Ud, ns ? ng * ng : (ng * (ng + 1u)) >> 1,
                                                reinterpret_cast<uint16_t *>(BUF) +
                                                    (uint32_t)w * scan_buf_entries(SrcTriScan<MODE == 3>::kPerRead),
                                                Ly.copies, Ly.tri_pad, ns ? ng : 0u};
                        dir_or_flush<Acc, NS>(a, g, s, split, rd, roi, a.merged ? 0 : d0 + dl, MARG, ng);
                    } else if (MODE == 0) {
                        SrcDenseList s{lst, n, Ud};
                        dir_or_flush<Acc, NS>(a, g, s, split, rd, roi, d0 + dl, MARG, ng);
                    } else {
                        SrcHashList s{lst, n, reinterpret_cast<uint32_t *>(smem + Ly.hkey_off),
                                      reinterpret_cast<uint32_t *>(smem + Ly.hcnt_off)};
                        dir_or_flush<Acc, NS>(a, g, s, split, rd, roi, d0 + dl, MARG, ng);
                    }
                    if (lane() == 0) LCNT[dl] = 0u;
                }
                __syncthreads();
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ banded ROIs
// Large split ROIs whose triangle does not fit LDS (many levels): a work item
// is one (ROI, direction, block of bbox rows); the work-group takes the
// block's pairs of that direction (by the row sweep for an in-plane
// distance-1 offset of a 2D image, else by gather) and counts every pair with
// |i - j| <
// band_w into an LDS band of ng x band_w 32-bit cells (cell (lo, hi) at
// lo * band_w + hi - lo), the rare wider pairs straight into the ROI's
// global matrix; the band is then added once, cell by nonzero cell, into
// the global matrix.  Smooth images put nearly every pair near the diagonal,
// so a block of hundreds of thousands of voxels costs one merge of a few
// thousand cells instead of one per small tile.  Tickets: one atomic per
// work item, mapped onto the banded ROIs in list order.
__global__ __launch_bounds__(1024) void k_band(StepArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    uint32_t *band = reinterpret_cast<uint32_t *>(smem);
    __shared__ uint32_t s_it[5];   // ROI row, direction, block, blocks, found
    const uint32_t ng = (uint32_t)a.ng, B = a.band_w, lgB = 31u - (uint32_t)__builtin_clz(B);
    const uint32_t cells = ng * B;
    const uint32_t nb = min(a.counters[C_NBAND], a.g_cap);
    for (;;) {
        if (threadIdx.x == 0) {
            uint32_t t = atomicAdd(&a.counters[C_BAND_TICKET], 1u);
            s_it[4] = 0u;
            for (uint32_t j = 0; j < nb; ++j) {
                const uint32_t row = a.band_roi[j];
                if (row >= a.roi_cap) continue;
                const RoiDesc &rd = a.rois[row];
                const uint32_t nrb = band_blocks(rd.rows, (uint32_t)(rd.x1 - rd.x0 + 1), a.band_tile);
                const uint32_t items = nrb * (uint32_t)a.K;
                if (t < items) {
                    s_it[0] = row; s_it[1] = t / nrb; s_it[2] = t - (t / nrb) * nrb; s_it[3] = nrb; s_it[4] = 1u;
                    break;
                }
                t -= items;
            }
        }
        __syncthreads();
        if (s_it[4] == 0u) break;
        const uint32_t row = s_it[0], nrb = s_it[3];
        const int d = (int)s_it[1];
        const uint32_t blk = s_it[2];
        const RoiDesc rd = a.rois[row];
        __syncthreads();   // every thread has read s_it before thread 0 rewrites it
        bool ok = rd.gslot < a.g_cap && rd.image < (uint32_t)a.n_images;
        ImgDesc im{};
        if (ok) {
            im = a.imgs[rd.image];
            ok = !(rd.x0 < 0 || rd.y0 < 0 || rd.z0 < 0 || rd.x1 >= im.nx || rd.y1 >= im.ny || rd.z1 >= im.nz ||
                   rd.x0 > rd.x1 || rd.y0 > rd.y1 || rd.z0 > rd.z1);
        }
        if (!ok) continue;   // uniform: every thread skips the item
        for (uint32_t i = threadIdx.x; i < cells; i += blockDim.x) band[i] = 0u;
        __syncthreads();
        ItemCtx c;
        c.I = im.I; c.L = im.L; c.B = im.B;
        c.nx = im.nx; c.ny = im.ny; c.nz = im.nz;
        c.label = rd.label; c.vmin = rd.vmin; c.ng = ng;
        c.rcp = fbn_rcp_up(rd.vmax > rd.vmin ? rd.vmax - rd.vmin : 1u);
        c.err = &a.counters[C_ERR];
        const uint32_t W = (uint32_t)(rd.x1 - rd.x0 + 1);
        const uint32_t rpb = (rd.rows + nrb - 1u) / nrb;
        const uint32_t ra = min(blk * rpb, rd.rows), rb = min(ra + rpb, rd.rows);
        uint64_t *G = a.G + ((uint64_t)rd.gslot * a.K_out + (a.merged ? 0 : d)) * (uint64_t)ng * ng;
        auto add = [&](uint32_t, uint32_t la, uint32_t, uint32_t lb, uint32_t) {
            const uint32_t lo = (la < lb ? la : lb) - 1u, hi = (la < lb ? lb : la) - 1u;
            if (hi - lo < B)
                atomicAdd(&band[(lo << lgB) + hi - lo], 1u);
            else
                atomicAdd(reinterpret_cast<unsigned long long *>(&G[(uint64_t)lo * ng + hi]), 1ull);
        };
        // an in-plane distance-1 offset of a 2D image: the row sweep (each
        // voxel's level once, neighbours by lane exchange); others: gather
        const int32_t oz = a.off[d][0], oy = a.off[d][1], ox = a.off[d][2];
        int cls = -1;
        if (im.nz == 1 && !c.B && oz == 0 && (oy | ox) != 0 && oy >= -1 && oy <= 1 && ox >= -1 && ox <= 1)
            cls = oy == 0 ? 0 : (ox == 0 ? 1 : (oy * ox < 0 ? 2 : 3));
        if (ra < rb) {
            if (cls >= 0) {
                const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
                accumulate_sweep2d<false>(rd, c, ra, rb, 0u, W, cls == 0 ? 0 : -1, cls == 1 ? 0 : -1,
                                          cls == 2 ? 0 : -1, cls == 3 ? 0 : -1, w, (int)(blockDim.x / kWave),
                                          NoRowOff{}, add);
            } else {
                accumulate_rows(a, rd, c, ra, rb, 0u, W, d, d + 1, threadIdx.x, blockDim.x, add);
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cells; i += blockDim.x) {
            const uint32_t v = band[i];
            if (v) {
                const uint32_t lo = i >> lgB, hi = lo + (i & (B - 1u));
                atomicAdd(reinterpret_cast<unsigned long long *>(&G[(uint64_t)lo * ng + hi]), (unsigned long long)v);
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ split ROIs
// One work-group per (split slot, direction): features from the merged global
// matrix (dense square, upper triangle).
template <class Acc>
__global__ __launch_bounds__(1024) void k_split_features(StepArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t ng = (uint32_t)a.ng;
    const int K = a.K_out;
    const uint32_t slot = blockIdx.x / K;
    const int d = (int)(blockIdx.x % K);
    if (slot >= min(a.counters[C_NSPLIT], a.g_cap)) return;
    const uint32_t roi = a.split_roi[slot];
    if (roi >= a.roi_cap) return;
    const uint32_t mw = (a.nonsym ? 5u : 4u) * ng;   // marginal words
    uint32_t *R = reinterpret_cast<uint32_t *>(smem);
    uint64_t *scratch = reinterpret_cast<uint64_t *>(smem + 4u * mw);
    for (uint32_t i = threadIdx.x; i < mw; i += blockDim.x) R[i] = 0u;
    __syncthreads();
    BlockGrp g{scratch};
    SrcSquare s{a.G + ((uint64_t)slot * K + d) * (uint64_t)ng * ng, ng, a.nonsym != 0};
    const uint64_t at = (uint64_t)roi * K + d;
    if (a.nonsym)
        dir_sums_ns<Acc>(g, s, R, R + ng, R + 2u * ng, R + 4u * ng - 1u, ng, a.dsums + at, a.dsums_y + at);
    else
        dir_sums<Acc, uint64_t>(g, s, R, R + ng, R + 3u * ng - 1u, ng, a.dsums + at);
}

// Split ROIs with symmetric matrices, first pass: one work-group per (slot,
// direction, chunk of matrix rows) visits the chunk's nonzero upper-triangle
// cells (a cell (lo < hi) with count c stands for P(lo, hi) = P(hi, lo) = c,
// a diagonal one for P = 2c), counts the marginals in LDS and adds them to
// the matrix's global marginals, and adds its exact integer cell totals; its
// sum of P log2 P goes to its own slot (added in chunk order later).
template <class Acc>
__global__ __launch_bounds__(256) void k_split_cells(StepArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ uint64_t red[4];
    const uint32_t ng = (uint32_t)a.ng, K = (uint32_t)a.K_out, chunks = a.split_chunks;
    const uint32_t sd = blockIdx.x / chunks, ch = blockIdx.x - sd * chunks;
    const uint32_t slot = sd / K;
    if (slot >= min(a.counters[C_NSPLIT], a.g_cap)) return;
    uint32_t *M = reinterpret_cast<uint32_t *>(smem);   // R [ng] | Sp [2 ng - 1] | Sm [ng]
    uint32_t *R = M, *Sp = M + ng, *Sm = M + 3u * ng - 1u;
    for (uint32_t i = threadIdx.x; i < 4u * ng; i += blockDim.x) M[i] = 0u;
    __syncthreads();
    const uint32_t rpc = (ng + chunks - 1u) / chunks, r0 = min(ch * rpc, ng), r1 = min(r0 + rpc, ng);
    const uint64_t *G = a.G + (uint64_t)sd * ng * ng;
    uint64_t T = 0, S11 = 0, sumP2 = 0, maxP = 0;
    LaneSum<Acc> plp;
    // the chunk's rows flat in row-major order (every lane busy however
    // short the rows are), upper-triangle cells only
    SquareWalk p(ng, r0, threadIdx.x, blockDim.x);
    for (uint64_t e = (uint64_t)r0 * ng + threadIdx.x; p.lo < r1; e += blockDim.x, p.next(ng)) {
        const uint32_t lo = p.lo, hi = p.hi;
        if (hi < lo) continue;
        const uint64_t cw = G[e];
        if (!cw) continue;
        const uint32_t c = (uint32_t)cw;
        atomicAdd(&R[lo], c);
        atomicAdd(&R[hi], c);
        atomicAdd(&Sp[lo + hi], 2u * c);
        atomicAdd(&Sm[hi - lo], 2u * c);
        const bool diag = lo == hi;
        const uint64_t P = diag ? 2ull * c : (uint64_t)c, Pm = diag ? P : 2u * P;
        T += 2ull * c;
        sumP2 += Pm * P;
        maxP = P > maxP ? P : maxP;
        S11 += Pm * (uint64_t)__umul24(lo + 1u, hi + 1u);
        plp.add((Acc)Pm * term_log2<Acc>((Acc)P));
    }
    __syncthreads();
    uint32_t *gm = a.smarg + (uint64_t)sd * 4u * ng;
    for (uint32_t i = threadIdx.x; i < 4u * ng; i += blockDim.x)
        if (M[i]) atomicAdd(&gm[i], M[i]);
    T = block_sum<4>(T, red);
    S11 = block_sum<4>(S11, red);
    sumP2 = block_sum<4>(sumP2, red);
    maxP = block_reduce<4>(maxP, red, OpMax());
    const double plp_t = block_sum<4>(comp_value(plp), red);
    if (threadIdx.x == 0) {
        uint64_t *tot = a.stot + (uint64_t)sd * 4u;
        atomicAdd(reinterpret_cast<unsigned long long *>(&tot[0]), (unsigned long long)T);
        atomicAdd(reinterpret_cast<unsigned long long *>(&tot[1]), (unsigned long long)S11);
        atomicAdd(reinterpret_cast<unsigned long long *>(&tot[2]), (unsigned long long)sumP2);
        atomicMax(reinterpret_cast<unsigned long long *>(&tot[3]), (unsigned long long)maxP);
        a.splp[(uint64_t)sd * chunks + ch] = plp_t;
    }
}

// Second pass: one work-group per (slot, direction) finishes the reduced sums
// from the global marginals and cell totals (the level sweeps, cluster
// moments and the mutual-information decision of dir_sums; a re-summed
// mutual information visits the matrix's cells once more).
template <class Acc>
__global__ __launch_bounds__(1024) void k_split_finish(StepArgs a) {
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t ng = (uint32_t)a.ng, K = (uint32_t)a.K_out;
    const uint32_t sd = blockIdx.x, slot = sd / K, d = sd - slot * K;
    if (slot >= min(a.counters[C_NSPLIT], a.g_cap)) return;
    const uint32_t roi = a.split_roi[slot];
    if (roi >= a.roi_cap) return;
    uint32_t *M = reinterpret_cast<uint32_t *>(smem);
    uint32_t *R = M, *Sp = M + ng, *Sm = M + 3u * ng - 1u;
    uint64_t *scratch = reinterpret_cast<uint64_t *>(smem + 16u * ng);
    const uint32_t *gm = a.smarg + (uint64_t)sd * 4u * ng;
    for (uint32_t i = threadIdx.x; i < 4u * ng; i += blockDim.x) M[i] = gm[i];
    __syncthreads();
    BlockGrp g{scratch};
    const int r0 = g.rank(), gs = g.size();
    const uint64_t *tot = a.stot + (uint64_t)sd * 4u;
    const uint64_t T = tot[0], S11t = tot[1], sumP2t = tot[2], maxPt = tot[3];
    double plp_t = 0.0;
    for (uint32_t c = 0; c < a.split_chunks; ++c) plp_t += a.splp[(uint64_t)sd * a.split_chunks + c];
    DirSums *out = a.dsums + (uint64_t)roi * K + d;
    // level sweeps over the marginals (as in dir_sums)
    uint64_t S1 = 0, S2 = 0, Sm1 = 0;
    LaneSum<Acc> rlr, slp, hom1, hom2, idmn, idn, iv, plps;
    const Acc ngf = (Acc)ng, rng = (Acc)1 / ngf, rng2 = rng * rng;
    for (uint32_t i = r0; i < ng; i += gs) {
        const uint32_t r = R[i];
        if (r) {
            const uint64_t lv = i + 1u;
            S1 += lv * r;
            S2 += lv * lv * r;
            rlr.add((Acc)r * term_log2<Acc>((Acc)r));
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
    const uint64_t S1t = g.sum(S1), S2t = g.sum(S2), Sm1t = g.sum(Sm1);
    const double rlr_t = g.sum(comp_value(rlr)), slp_t = g.sum(comp_value(slp)), plps_t = g.sum(comp_value(plps));
    const double hom1_t = g.sum(comp_value(hom1)), hom2_t = g.sum(comp_value(hom2));
    const double idmn_t = g.sum(comp_value(idmn)), idn_t = g.sum(comp_value(idn)), iv_t = g.sum(comp_value(iv));
    double CSHADE = 0.0, CPROM = 0.0, MI = __builtin_nan("");
    if (T) {
        const double Td = (double)T, invT = 1.0 / Td;
        const double two_mu = (double)(2u * S1t) / Td;   // one rounding
        double cs = 0.0, cp = 0.0;
        for (uint32_t k = r0; k < 2u * ng - 1u; k += gs) {
            const uint32_t sp = Sp[k];
            if (sp) {
                const double p = (double)sp * invT, dd = (double)(k + 2u) - two_mu, d3 = dd * dd * dd;
                cs += d3 * p;
                cp += d3 * dd * p;
            }
        }
        CSHADE = g.sum(cs);
        CPROM = g.sum(cp);
        const double mi_cf = (double)__log2f((float)Td) - (2.0 * rlr_t - plp_t) * invT;
        if (mi_cf < mi_resum_threshold<Acc>()) {
            Comp<Acc> m;
            const Acc invTa = (Acc)invT;
            SrcSquare src{a.G + (uint64_t)sd * ng * ng, ng};
            src.for_each(g, [&](uint32_t lo, uint32_t hi, uint32_t c) {
                const bool diag = lo == hi;
                const uint64_t P = diag ? 2ull * c : (uint64_t)c;
                const Acc mult = diag ? (Acc)1 : (Acc)2;
                const uint64_t A = P * T, B = (uint64_t)R[lo] * (uint64_t)R[hi];
                const Acc delta = A >= B ? (Acc)(A - B) / (Acc)B : -((Acc)(B - A) / (Acc)B);
                m.add(mult * (Acc)P * invTa * log1p_<Acc>(delta) * (Acc)1.4426950408889634);
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
    }
}

// ------------------------------------------------------------------ features
// The 30 features of every (ROI, direction) from its reduced sums, one lane
// each, then the ROI's table row: the K direction blocks and their mean over
// the non-empty directions, written as one contiguous run of the table.
// Rows [0, n) with n = min(*n_ptr, n_cap) (n_cap without n_ptr).
template <class OutT>
__global__ __launch_bounds__(128, 4) void k_features(StepArgs a, const DirSums *ds, const DirSumsY *dsy,
                                                  uint32_t n_cap, const uint32_t *n_ptr) {
    extern __shared__ __align__(16) uint8_t smem[];
    // staged in the output precision: single-precision tables take half the
    // LDS, so twice as many work-groups fit a CU; they keep cluster shade and
    // correlation in double beside (xd), for the direction mean
    constexpr bool kXd = sizeof(OutT) == 4;
    OutT *feat = reinterpret_cast<OutT *>(smem);
    const uint32_t K = (uint32_t)a.K_out;
    const uint32_t rpb = blockDim.x / K;
    double *xd = reinterpret_cast<double *>(smem + (size_t)rpb * K * kNumFeat * sizeof(OutT));
    const uint32_t n = n_ptr ? min(*n_ptr, n_cap) : n_cap;
    const uint32_t row0 = blockIdx.x * rpb;
    if (row0 >= n) return;
    uint32_t rows = min(rpb, n - row0);
    if (threadIdx.x < rows * K) {
        const uint64_t at = (uint64_t)row0 * K + threadIdx.x;
        finalize_dir<OutT>(ds[at], a.nonsym ? dsy + at : nullptr, feat + threadIdx.x * kNumFeat,
                           kXd ? xd + 2u * threadIdx.x : nullptr);
    }
    __syncthreads();
    if (row0 + rows > a.table_rows) {
        if (threadIdx.x == 0) atomicOr(&a.counters[C_ERR], (uint32_t)E_TABLE_CAP);
        rows = a.table_rows > row0 ? a.table_rows - row0 : 0u;
    }
    // K direction blocks and their mean, or the one block of the merged matrix
    const uint32_t per = (a.merged ? 1u : K + 1u) * kNumFeat;
    OutT *out = reinterpret_cast<OutT *>(a.table) + (uint64_t)row0 * per;
    // element i of the block's rows is (row rr, position q): one division for
    // the thread's first element, then stepped (no division per element)
    uint32_t rr = threadIdx.x / per, q = threadIdx.x - rr * per;
    for (uint32_t i = threadIdx.x; i < rows * per; i += blockDim.x) {
        const uint32_t blk = q / (uint32_t)kNumFeat, f = q - blk * (uint32_t)kNumFeat;
        const OutT *fr = feat + rr * K * kNumFeat;
        double v;
        if (blk < K) {
            v = fr[blk * kNumFeat + f];
        } else {
            // (cluster shade and correlation from their double copies)
            const int x = !kXd ? -1 : (f == F_CLUSHADE ? 0 : (f == F_CORR ? 1 : -1));
            const double *xr = xd + 2u * rr * K;
            double s = 0.0;
            int m = 0;
            for (uint32_t k = 0; k < K; ++k)
                if (!isnan(fr[k * kNumFeat])) {
                    s += x >= 0 ? xr[2u * k + (uint32_t)x] : (double)fr[k * kNumFeat + f];
                    ++m;
                }
            v = m ? s / (double)m : __builtin_nan("");
        }
        out[i] = (OutT)v;
        q += blockDim.x;
        while (q >= per) { q -= per; ++rr; }
    }
}

// ------------------------------------------------------------------ COO
// Nonzero upper-triangle cells of each (slot, direction) matrix.
__global__ __launch_bounds__(256) void k_coo_count(StepArgs a, uint32_t n_slots, uint64_t *counts) {
    const uint32_t ng = (uint32_t)a.ng;
    const uint32_t sd = blockIdx.x;
    if (sd >= n_slots * (uint32_t)a.K_out) return;
    const uint64_t *G = a.G + (uint64_t)sd * ng * ng;
    uint64_t c = 0;
    for (uint32_t i = 0; i < ng; ++i)
        for (uint32_t j = (a.nonsym ? 0u : i) + threadIdx.x; j < ng; j += blockDim.x) c += G[(uint64_t)i * ng + j] != 0u;
    __shared__ uint64_t part[4];
    c = wave_sum(c);
    if (lane() == 0) part[threadIdx.x / 64] = c;
    __syncthreads();
    if (threadIdx.x == 0) counts[sd] = part[0] + part[1] + part[2] + part[3];
}

// Writes each (slot, direction) matrix's nonzero cells in (i, j) order at its
// offset: keys roi << 38 | dir << 32 | i << 16 | j.
__global__ __launch_bounds__(256) void k_coo_emit(StepArgs a, uint32_t n_slots, const uint64_t *offsets,
                                                  uint64_t *keys, uint64_t *vals) {
    const uint32_t ng = (uint32_t)a.ng;
    const uint32_t sd = blockIdx.x;
    if (sd >= n_slots * (uint32_t)a.K_out) return;
    const uint32_t slot = sd / a.K_out, d = sd % a.K_out;
    const uint64_t roi = a.split_roi[slot];
    const uint64_t *G = a.G + (uint64_t)sd * ng * ng;
    __shared__ uint32_t wc[4], s_base;
    uint64_t pos = offsets[sd];
    for (uint32_t e0 = 0; e0 < ng * ng; e0 += blockDim.x) {
        uint32_t e = e0 + threadIdx.x;
        uint32_t i = e / ng, j = e - i * ng;
        uint64_t v = (e < ng * ng && (i <= j || a.nonsym)) ? G[e] : 0ull;
        uint64_t m = __ballot(v != 0ull);
        if (lane() == 0) wc[threadIdx.x / 64] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t pre = 0, tot = 0;
        for (int q = 0; q < 4; ++q) { if (q < (int)(threadIdx.x / 64)) pre += wc[q]; tot += wc[q]; }
        if (v) {
            uint64_t p = pos + pre + (uint32_t)__popcll(m & __lanemask_lt());
            keys[p] = (roi << 38) | ((uint64_t)d << 32) | ((uint64_t)i << 16) | (uint64_t)j;
            vals[p] = v;
        }
        pos += tot;
        __syncthreads();
    }
    (void)s_base;
}

// Segment start of every (roi, dir) in a sorted key list (n_rois * K + 1 entries).
__global__ void k_coo_segments_k(const uint64_t *keys, uint64_t nnz, uint32_t n_rois, int K, uint64_t *seg) {
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t n_seg = n_rois * (uint32_t)K;
    if (s > n_seg) return;
    uint64_t target = s == n_seg ? ~0ull : (((uint64_t)(s / K)) << 38) | ((uint64_t)(s % K) << 32);
    uint64_t lo = 0, hi = nnz;
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        if (keys[mid] < target) lo = mid + 1; else hi = mid;
    }
    seg[s] = s == n_seg ? nnz : lo;
}

// One work-group per (roi, direction) of a COO list.
template <class Acc>
__global__ __launch_bounds__(512) void k_coo_features(StepArgs a, const uint64_t *keys, const uint64_t *vals,
                                                      const uint64_t *seg, uint32_t n_rois, DirSums *sums,
                                                      DirSumsY *sums_y) {
    extern __shared__ __align__(16) uint8_t smem[];
    const uint32_t ng = (uint32_t)a.ng;
    const int K = a.K_out;
    const uint32_t s = blockIdx.x;
    if (s >= n_rois * (uint32_t)K) return;
    const uint32_t mw = (a.nonsym ? 5u : 4u) * ng;   // marginal words
    uint32_t *R = reinterpret_cast<uint32_t *>(smem);
    uint64_t *scr = reinterpret_cast<uint64_t *>(smem + 4u * mw);
    for (uint32_t i = threadIdx.x; i < mw; i += blockDim.x) R[i] = 0u;
    __syncthreads();
    BlockGrp g{scr};
    SrcCoo src{keys + seg[s], vals + seg[s], (uint32_t)(seg[s + 1] - seg[s]),
               ((uint64_t)(s / K) << 38) | ((uint64_t)(s % K) << 32), ng, &a.counters[C_ERR], a.nonsym != 0};
    if (a.nonsym)
        dir_sums_ns<Acc>(g, src, R, R + ng, R + 2u * ng, R + 4u * ng - 1u, ng, sums + s, sums_y + s);
    else
        dir_sums<Acc, uint64_t>(g, src, R, R + ng, R + 3u * ng - 1u, ng, sums + s);
}

// ================================================================== launchers
#define NYX_CHECK_LAUNCH() \
    do { hipError_t _e = hipGetLastError(); if (_e != hipSuccess) return _e; } while (0)

hipError_t launch_max_label(const ImgDesc *imgs, int n_images, uint32_t *out, hipStream_t st) {
    dim3 grid(256, n_images);
    hipLaunchKernelGGL(k_max_label, grid, dim3(256), 0, st, imgs, n_images, out);
    NYX_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_label_collect(const ImgDesc *imgs, int n_images, uint64_t max_vox, uint64_t *list, uint32_t cap,
                                uint32_t *count, hipStream_t st) {
    constexpr uint32_t chunk = 1u << 16;
    const uint32_t gx = (uint32_t)((max_vox + chunk - 1u) / chunk);
    if (gx == 0u || n_images <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_label_collect, dim3(gx, (uint32_t)n_images), dim3(256), 0, st, imgs, n_images, chunk, list,
                       cap, count);
    NYX_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_reset(const StepArgs &a, uint32_t n_counters, hipStream_t st) {
    uint32_t n = a.tab.total > n_counters ? a.tab.total : n_counters;
    uint32_t blocks = (n + 255) / 256;
    if (blocks > 8192) blocks = 8192;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_reset, dim3(blocks), dim3(256), 0, st, a, n_counters);
    NYX_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t n, uint64_t v, hipStream_t st) {
    if (n == 0) return hipSuccess;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_fill_u64, dim3((uint32_t)blocks), dim3(256), 0, st, p, n, v);
    NYX_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_zero_split(const StepArgs &a, hipStream_t st) {
    if (a.g_cap == 0) return hipSuccess;
    uint64_t n = (uint64_t)a.g_cap * a.K_out * (uint64_t)a.ng * a.ng;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(k_zero_split, dim3((uint32_t)blocks), dim3(256), 0, st, a);
    NYX_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_scan(const StepArgs &a, hipStream_t st) {
    if (a.total_chunks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_scan, dim3(a.total_chunks), dim3(kScanTileCols), 0, st, a);
    NYX_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_compact(const StepArgs &a, uint32_t roi_lo, uint32_t roi_hi, hipStream_t st) {
    uint32_t blocks = (a.tab.total + 1023) / 1024;
    if (blocks == 0) return hipSuccess;
    hipLaunchKernelGGL(k_compact_count, dim3(blocks), dim3(1024), 0, st, a);
    NYX_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_compact_write, dim3(blocks), dim3(1024), 0, st, a, roi_lo, roi_hi);
    NYX_CHECK_LAUNCH();
    if (a.force_split) {
        hipLaunchKernelGGL(k_set_nsplit, dim3(1), dim3(1), 0, st, a, roi_lo, roi_hi);
        NYX_CHECK_LAUNCH();
    }
    return hipSuccess;
}

hipError_t launch_bin_image(const StepArgs &a, uint16_t *bins, uint64_t total_vox, const uint64_t *img_vox_base,
                            hipStream_t st) {
    if (total_vox == 0) return hipSuccess;
    uint64_t blocks = (total_vox + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_bin_image, dim3((uint32_t)blocks), dim3(256), 0, st, a, bins, total_vox, img_vox_base);
    NYX_CHECK_LAUNCH();
    return hipSuccess;
}

template <int MODE, class OutT, bool NS, int BS>
static hipError_t launch_batch_b(const StepArgs &a, uint32_t grid, uint32_t direct_roi, hipStream_t st) {
    static bool attr_done = false;
    if (!attr_done) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_batch<MODE, OutT, NS, BS>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
        if (e != hipSuccess) return e;
        attr_done = true;
    }
    hipLaunchKernelGGL((k_batch<MODE, OutT, NS, BS>), dim3(grid), dim3(BS), a.lds.bytes, st, a, direct_roi);
    NYX_CHECK_LAUNCH();
    return hipSuccess;
}

// (work-groups of 256 or 512 threads: any other size is refused)
template <int MODE, class OutT, bool NS>
static hipError_t launch_batch_t(const StepArgs &a, uint32_t grid, uint32_t block, uint32_t direct_roi,
                                 hipStream_t st) {
    if (block == 512u) return launch_batch_b<MODE, OutT, NS, 512>(a, grid, direct_roi, st);
    if (block != 256u) return hipErrorInvalidConfiguration;
    return launch_batch_b<MODE, OutT, NS, 256>(a, grid, direct_roi, st);
}

template <int MODE, bool NS>
static hipError_t launch_batch_m(const StepArgs &a, uint32_t grid, uint32_t block, uint32_t direct_roi,
                                 hipStream_t st) {
    return a.fp64 ? launch_batch_t<MODE, double, NS>(a, grid, block, direct_roi, st)
                  : launch_batch_t<MODE, float, NS>(a, grid, block, direct_roi, st);
}

// (ordered counts never take the returning-atomic list, mode 0)
hipError_t launch_batch(const StepArgs &a, uint32_t grid, uint32_t block, uint32_t direct_roi, hipStream_t st) {
    if (grid == 0u) return hipSuccess;   // (a banded ROI has no batch tiles)
    const bool ns = a.nonsym != 0;
    switch (a.lds.mode) {
        case 0: return launch_batch_m<0, false>(a, grid, block, direct_roi, st);
        case 1: return ns ? launch_batch_m<1, true>(a, grid, block, direct_roi, st)
                          : launch_batch_m<1, false>(a, grid, block, direct_roi, st);
        case 2: return ns ? launch_batch_m<2, true>(a, grid, block, direct_roi, st)
                          : launch_batch_m<2, false>(a, grid, block, direct_roi, st);
        default: return ns ? launch_batch_m<3, true>(a, grid, block, direct_roi, st)
                           : launch_batch_m<3, false>(a, grid, block, direct_roi, st);
    }
}

template <int MODE, bool NS>
static const void *batch_kernel_m(int fp64, uint32_t block) {
    if (block == 512u)
        return fp64 ? reinterpret_cast<const void *>(&k_batch<MODE, double, NS, 512>)
                    : reinterpret_cast<const void *>(&k_batch<MODE, float, NS, 512>);
    return fp64 ? reinterpret_cast<const void *>(&k_batch<MODE, double, NS, 256>)
                : reinterpret_cast<const void *>(&k_batch<MODE, float, NS, 256>);
}

static const void *batch_kernel(int mode, int fp64, int ns, uint32_t block) {
    switch (mode) {
        case 0: return batch_kernel_m<0, false>(fp64, block);
        case 1: return ns ? batch_kernel_m<1, true>(fp64, block) : batch_kernel_m<1, false>(fp64, block);
        case 2: return ns ? batch_kernel_m<2, true>(fp64, block) : batch_kernel_m<2, false>(fp64, block);
        default: return ns ? batch_kernel_m<3, true>(fp64, block) : batch_kernel_m<3, false>(fp64, block);
    }
}

hipError_t batch_occupancy(int mode, int fp64, int ns, uint32_t block, uint32_t lds_bytes, int *blocks_per_cu) {
    if (block != 256u && block != 512u) return hipErrorInvalidConfiguration;
    const void *f = batch_kernel(mode, fp64, ns, block);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, f, (int)block, (size_t)lds_bytes);
}

hipError_t get_batch_attributes(int mode, int fp64, int ns, uint32_t block, hipFuncAttributes *attr) {
    return hipFuncGetAttributes(attr, batch_kernel(mode, fp64, ns, block));
}

static hipError_t set_feature_kernel_attrs() {
    static bool done = false;
    if (done) return hipSuccess;
    const void *fs[] = {reinterpret_cast<const void *>(&k_split_features<float>),
                        reinterpret_cast<const void *>(&k_split_features<double>),
                        reinterpret_cast<const void *>(&k_split_cells<float>),
                        reinterpret_cast<const void *>(&k_split_cells<double>),
                        reinterpret_cast<const void *>(&k_split_finish<float>),
                        reinterpret_cast<const void *>(&k_split_finish<double>),
                        reinterpret_cast<const void *>(&k_coo_features<float>),
                        reinterpret_cast<const void *>(&k_coo_features<double>)};
    for (const void *f : fs) {
        // (some of these kernels keep a few bytes of static LDS besides)
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 159 * 1024);
        if (e != hipSuccess) return e;
    }
    done = true;
    return hipSuccess;
}

hipError_t launch_band(const StepArgs &a, uint32_t grid, hipStream_t st) {
    if (a.band_vox == 0u || a.g_cap == 0u || grid == 0u) return hipSuccess;
    const uint32_t lds = (uint32_t)a.ng * a.band_w * 4u;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_band),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_band, dim3(grid), dim3(1024), lds, st, a);
    NYX_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_split_finalize(const StepArgs &a, hipStream_t st) {
    if (a.g_cap == 0) return hipSuccess;
    {
        hipError_t e = set_feature_kernel_attrs();
        if (e != hipSuccess) return e;
    }
    uint32_t grid = a.g_cap * a.K_out;
    // Enough small matrices to fill the chip: one 256-thread work-group per
    // matrix.  Few or large ones (symmetric): two passes, row chunks in
    // parallel, then one work-group per matrix.
    if (!a.nonsym && a.smarg && (a.split_chunks > 1u || a.ng > 256)) {
        const uint32_t lds1 = 16u * a.ng;
        if (a.fp64) hipLaunchKernelGGL(k_split_cells<double>, dim3(grid * a.split_chunks), dim3(256), lds1, st, a);
        else hipLaunchKernelGGL(k_split_cells<float>, dim3(grid * a.split_chunks), dim3(256), lds1, st, a);
        NYX_CHECK_LAUNCH();
        const uint32_t lds2 = 16u * a.ng + 16 * 8;
        if (a.fp64) hipLaunchKernelGGL(k_split_finish<double>, dim3(grid), dim3(1024), lds2, st, a);
        else hipLaunchKernelGGL(k_split_finish<float>, dim3(grid), dim3(1024), lds2, st, a);
        NYX_CHECK_LAUNCH();
        return hipSuccess;
    }
    uint32_t lds = (a.nonsym ? 20u : 16u) * a.ng + 16 * 8;
    const uint32_t bs = a.ng <= 256 ? 256u : 1024u;
    if (a.fp64) hipLaunchKernelGGL(k_split_features<double>, dim3(grid), dim3(bs), lds, st, a);
    else hipLaunchKernelGGL(k_split_features<float>, dim3(grid), dim3(bs), lds, st, a);
    NYX_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_features(const StepArgs &a, const DirSums *ds, const DirSumsY *dsy, uint32_t n_cap,
                           const uint32_t *n_ptr, hipStream_t st) {
    if (n_cap == 0) return hipSuccess;
    const uint32_t block = 128u, rpb = block / (uint32_t)a.K_out;
    const uint32_t grid = (n_cap + rpb - 1u) / rpb;
    const uint32_t lds = rpb * (uint32_t)a.K_out * (a.fp64 ? kNumFeat * 8u : kNumFeat * 4u + 16u);
    if (a.fp64) hipLaunchKernelGGL(k_features<double>, dim3(grid), dim3(block), lds, st, a, ds, dsy, n_cap, n_ptr);
    else hipLaunchKernelGGL(k_features<float>, dim3(grid), dim3(block), lds, st, a, ds, dsy, n_cap, n_ptr);
    NYX_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_coo_count(const StepArgs &a, uint32_t n_slots, uint64_t *counts, hipStream_t st) {
    if (n_slots == 0) return hipSuccess;
    hipLaunchKernelGGL(k_coo_count, dim3(n_slots * a.K_out), dim3(256), 0, st, a, n_slots, counts);
    NYX_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_coo_emit(const StepArgs &a, uint32_t n_slots, const uint64_t *offsets, uint64_t *keys,
                           uint64_t *vals, hipStream_t st) {
    if (n_slots == 0) return hipSuccess;
    hipLaunchKernelGGL(k_coo_emit, dim3(n_slots * a.K_out), dim3(256), 0, st, a, n_slots, offsets, keys, vals);
    NYX_CHECK_LAUNCH();
    return hipSuccess;
}

hipError_t launch_coo_features(const StepArgs &a, const uint64_t *keys, const uint64_t *vals, uint64_t nnz,
                               uint32_t n_rois, uint64_t *seg, DirSums *sums, DirSumsY *sums_y, hipStream_t st) {
    uint32_t n_seg = n_rois * (uint32_t)a.K_out;
    hipLaunchKernelGGL(k_coo_segments_k, dim3((n_seg + 1 + 255) / 256), dim3(256), 0, st, keys, nnz, n_rois,
                       a.K_out, seg);
    NYX_CHECK_LAUNCH();
    if (n_seg == 0) return hipSuccess;
    {
        hipError_t e = set_feature_kernel_attrs();
        if (e != hipSuccess) return e;
    }
    uint32_t lds = (a.nonsym ? 20u : 16u) * a.ng + 16 * 8;
    if (a.fp64)
        hipLaunchKernelGGL(k_coo_features<double>, dim3(n_seg), dim3(512), lds, st, a, keys, vals, seg, n_rois, sums,
                           sums_y);
    else
        hipLaunchKernelGGL(k_coo_features<float>, dim3(n_seg), dim3(512), lds, st, a, keys, vals, seg, n_rois, sums,
                           sums_y);
    NYX_CHECK_LAUNCH();
    return launch_features(a, sums, sums_y, n_rois, nullptr, st);
}

}  // namespace nyx
