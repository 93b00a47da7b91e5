// nyx_types.h -- plain data shared by the HIP kernels and the host runtime.
//
// Nothing here depends on torch.  Structures are passed to kernels by value
// (StepArgs) or live in device memory (ImgDesc, RoiDesc, work items).
#pragma once
#include <stdint.h>

namespace nyx {

constexpr int kWave = 64;
constexpr int kNumFeat = 30;
constexpr int kNumIntensityFeat = 37;   // first-order intensity features per ROI
constexpr int kNumNeighbourFeat = 37;   // NGLDM, NGTDM and GLDM features per ROI
constexpr int kMaxOffsets = 64;
constexpr int kClasses = 32;           // work-item size classes (log2 of voxels)
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kTicketChunk = 8;        // most queue entries taken per work ticket
constexpr uint32_t kTicketVox = 8192u; // voxels a ticket of small items aims at
constexpr uint32_t kItemBytes = 128u;  // LDS bytes of one staged work-item descriptor
constexpr int kMaxSweepPasses = 16;    // passes with a precomputed 2D sweep map

// Counter slots (u32) in the device counter block.
enum Counter : int {
    C_NROIS = 0,    // ROIs found by the last compaction
    C_NSPLIT = 1,   // ROIs split into several tiles (global-matrix slots used)
    C_ERR = 3,      // error bits (see ErrBit)
    C_NITEMS = 4,   // work items enqueued
    C_NBAND = 5,    // split ROIs accumulated by the banded kernel
    C_BAND_TICKET = 6,  // work tickets of the banded kernel
    C_CLASS = 8,    // kClasses counters: work-group items per size class
    C_TICKETS = 128,  // kTicketLanes ticket counters of the persistent kernel, kTicketStride apart
    C_BLOCKS = 128 + 32 * 32, // per-block ROI counts of the compaction (variable length)
};
// Work-group w draws tickets w mod kTicketLanes, +kTicketLanes, ... from
// its own counter: the claims spread over kTicketLanes memory lines instead
// of serialising on one.
constexpr uint32_t kTicketLanes = 32, kTicketStride = 32;
static_assert(C_TICKETS + kTicketLanes * kTicketStride <= C_BLOCKS, "ticket counters overlap");

enum ErrBit : uint32_t {
    E_LABEL_RANGE = 1u,   // a label exceeds the planned label-table capacity
    E_ROI_CAP = 2u,       // more ROIs than planned
    E_SPLIT_CAP = 4u,     // more split ROIs than planned
    E_ITEM_CAP = 8u,      // work-item bucket overflow
    E_LIST_CAP = 16u,     // LDS nonzero-list overflow (planner bug)
    E_HASH_FULL = 32u,    // LDS hash table full (planner bug)
    E_TABLE_CAP = 64u,    // output table too small
    E_BIN_RANGE = 128u,   // a caller-supplied bin image holds a value outside [1, n_bins]
    E_COO_RANGE = 256u,   // a caller-supplied COO entry is outside its matrix
};

struct ImgDesc {
    const uint16_t *I;     // intensity
    const uint32_t *L;     // labels
    const uint16_t *B;     // optional bin image (nullptr: bin on the fly)
    int32_t nz, ny, nx;
    uint32_t nvox;
    uint32_t tab_base;     // label-table index of entry 0 of this image (entry 0 is never used)
    uint32_t max_label;    // label-table entries of this image are 0..max_label
    uint32_t chunk_base;   // first scan tile of this image
    uint32_t dict_n;       // entries of dict
    const uint32_t *dict;  // the image's distinct nonzero labels, ascending (nullptr: a label is its own entry)
};

// Per-label statistics, one entry per (image, label), struct of arrays.
struct LabelTab {
    uint32_t *cnt, *mn, *mx;
    int32_t *x0, *y0, *z0, *x1, *y1, *z1;
    uint32_t *row;         // ROI row of a present label
    uint32_t total;        // entries over all images
};

struct RoiDesc {
    uint32_t label, image, n, n_tiles;
    uint32_t vmin, vmax, gslot, rows;   // rows = bbox rows (z * y extent)
    int32_t x0, y0, z0, x1, y1, z1;
    uint32_t tcols;                      // column blocks per tile row (n_tiles = row blocks * tcols)
    uint32_t pad1;
};

// Layout of the persistent kernel's dynamic LDS (byte offsets).
// Reduced sums of one (ROI, direction), written by the accumulation kernels
// and turned into the 30 features by the feature kernel.  Slots 0..15 come
// out of one batched reduction (slot i = 8-byte word i); the integer sums are
// exact.  The floating sums are raw (unnormalised) totals over the counts:
//   plp  = sum over both orders of P log2 P     rlr  = sum_i R(i) log2 R(i)
//   slp  = sum_k Sm(k) log2 Sm(k)               plps = sum_k Sp(k) log2 Sp(k)
//   hom1, hom2, idmn, idn, iv = sum_k Sm(k) w(k) with the feature's weight w
// with R, Sp, Sm the row, sum and difference marginals of P (Sm over |i-j|
// counting both orders).  CSHADE / CPROM are already normalised; MI is the
// cell-by-cell re-summed mutual information (bits) or NaN when the closed
// form 2 HX - JE is accurate enough.
struct DirSums {
    uint64_t T, S1, S2, Sm1, S11, sumP2;                              // slots 0-5
    double plp, rlr, slp, plps, hom1, hom2, idmn, idn, iv, spare;     // slots 6-15
    uint64_t maxP;
    double CSHADE, CPROM, MI;
};
static_assert(sizeof(DirSums) == 160, "DirSums layout");
// The column-marginal sums of a non-symmetric matrix (for a symmetric one
// they equal the row-marginal sums S1, S2, rlr of DirSums):
//   S1y = sum_j j C(j), S2y = sum_j j^2 C(j), clc = sum_j C(j) log2 C(j)
// with C the column marginal.
struct DirSumsY {
    uint64_t S1y, S2y;
    double clc, spare;
};
static_assert(sizeof(DirSumsY) == 32, "DirSumsY layout");
constexpr int kSumSlots = 16;
// ROI discovery tiles: rows (of all z-planes, flattened) x columns; one
// work-group of kScanTileCols threads per tile.
constexpr uint32_t kScanTileRows = 32;
constexpr uint32_t kScanTileCols = 256;
// Compaction buffer entries (u32 cell indices) per lane of an ordered
// triangle scan (one 16-byte read: at most 8 packed counters).
constexpr int kScanCells = 8;
// First-pass rounds of the two-level triangle scan per block: the nonzero
// 16-byte runs of kChunkRounds x 64 runs are listed (u16 entries) before
// their cells are.
constexpr int kChunkRounds = 5;
// u16 entries per wavefront of the scan buffer: cell indices (64 x cells per
// read), then the run list (64 x kChunkRounds).
__host__ __device__ constexpr uint32_t scan_buf_entries(uint32_t cells_per_read) {
    return 64u * cells_per_read + 64u * (uint32_t)kChunkRounds;
}

struct LdsLayout {
    uint32_t mode;        // 0 = dense triangles, 1 = hash table
    uint32_t kp;          // directions accumulated per pass
    uint32_t tri_pad;     // u32 words per dense triangle (dense mode)
    uint32_t list_cap;    // entries per direction list
    uint32_t hash_cap;    // slots (power of two, hash mode)
    uint32_t u_off, list_off, lcnt_off, marg_off, feat_off, sums_off, misc_off, hkey_off, hcnt_off, buf_off;
    uint32_t item_off;    // staged descriptors of the current ticket (work-group kernel)
    uint32_t ring_off, ring_bytes;   // level ring of the staged accumulation (0 bytes: none)
    uint32_t ro_off;      // triangle row offsets of the levels 0..ng (dense symmetric modes; 0: none)
    uint32_t bytes;       // total dynamic LDS
    uint32_t nwaves;      // waves per work-group
    uint32_t marg_sets;   // marginal sets at marg_off (one per wave that reduces a matrix)
    uint32_t n_tri;       // dense matrices at u_off (kp, or 1 when the offsets' matrices are merged)
    uint32_t copies;      // privatised copies of each dense triangle (1, 2 or 4): lane l adds to copy
                          // l mod copies; copy c of matrix m starts (m * copies + c) * tri_pad words in
};

struct StepArgs {
    const ImgDesc *imgs;
    int32_t n_images;
    uint32_t total_chunks;      // scan tiles over all images
    LabelTab tab;
    RoiDesc *rois;
    uint32_t roi_cap;
    uint32_t *counters;
    uint2 *buckets;             // kClasses buckets of bucket_cap items
    uint32_t bucket_cap;
    uint64_t *G;                // split-ROI dense matrices: g_cap slots of K * ng * ng
    uint32_t g_cap;
    DirSums *dsums;             // roi_cap * K reduced sums, row-major by ROI
    DirSumsY *dsums_y;          // roi_cap * K column-marginal sums (non-symmetric matrices only)
    int32_t nonsym;             // 1: ordered counts P = C (full ng x ng squares), 0: symmetric P = C + C^T
    uint32_t *split_roi;        // g_cap: ROI row of each split slot
    // Banded accumulation of large split ROIs whose triangle does not fit LDS:
    // ROIs above band_vox voxels (0: none) are counted by k_band, one
    // (ROI, direction, block of bbox rows of about band_tile voxels) per work
    // item, into an LDS band of ng x band_w cells (|i - j| < band_w, a power
    // of two) merged once into the ROI's global matrix.
    uint32_t band_vox, band_w, band_tile;
    uint32_t *band_roi;         // g_cap: ROI rows of the banded ROIs
    // Reduced sums of split ROIs (symmetric matrices) in two passes: chunks
    // of rows of each global matrix in parallel (marginals and cell totals),
    // then one work-group per matrix.  smarg: 4 ng u32 per (slot, direction)
    // (row, sum, difference marginals); stot: T, S11, sum P^2, max P (u64);
    // splp: the chunks' sums of P log2 P, added in chunk order.
    uint32_t *smarg;
    uint64_t *stot;
    double *splp;
    uint32_t split_chunks;
    int32_t off[kMaxOffsets][3];
    int32_t K;                  // offsets
    int32_t K_out;              // matrices per ROI: K, or 1 when the offsets' matrices are merged
    int32_t merged;             // 1: features of the sum of the K matrices (dense scan modes only)
    int32_t ng;
    uint32_t split_vox;         // ROIs above this many voxels are split
    uint32_t tile_vox;          // target voxels per tile of a split ROI
    int32_t force_split;        // 1: every ROI goes through the global matrices
    int32_t enqueue;            // 0: compaction builds the ROI table only
    int32_t fp64;               // feature table element type
    void *table;
    uint32_t table_rows;
    // optional ROI-table outputs
    uint32_t *o_label, *o_image;
    uint64_t *o_n;
    uint16_t *o_min, *o_max;
    int32_t *o_bbox;
    LdsLayout lds;
    // 2D distance-1 row-sweep accumulation: per pass, the local direction slot
    // of the H, V, D45, D135 neighbour classes (-1 = absent)
    int32_t sweep_ok;
    int8_t sweep[kMaxSweepPasses][4];
};

// Deterministic split rule shared by host planning and device enqueueing:
// a ROI above split_vox voxels is cut into about n / tile_vox tiles, first
// into blocks of bbox rows, then each row block into column blocks.
struct Tiling { uint32_t row_blocks, col_blocks; };

#ifdef __HIPCC__
__host__ __device__
#endif
inline Tiling tiles_for(uint32_t n, uint32_t rows, uint32_t width, uint32_t split_vox, uint32_t tile_vox) {
    Tiling t{1u, 1u};
    if (n <= split_vox || tile_vox == 0u) return t;
    uint32_t nt = (n + tile_vox - 1u) / tile_vox;
    t.row_blocks = nt < rows ? nt : rows;
    uint32_t nc = (nt + t.row_blocks - 1u) / t.row_blocks;
    t.col_blocks = nc < width ? nc : width;
    if (t.col_blocks < 1u) t.col_blocks = 1u;
    return t;
}

// Bounds of tile `tile` of a ROI: bbox rows [ra, rb) and columns [ca, cb).
#ifdef __HIPCC__
__host__ __device__
#endif
inline void tile_bounds(uint32_t rows, uint32_t width, uint32_t n_tiles, uint32_t tcols, uint32_t tile,
                        uint32_t *ra, uint32_t *rb, uint32_t *ca, uint32_t *cb) {
    uint32_t nrb = n_tiles / tcols;
    uint32_t rpt = (rows + nrb - 1u) / nrb;
    uint32_t cpt = (width + tcols - 1u) / tcols;
    uint32_t r = tile / tcols, c = tile - r * tcols;
    *ra = r * rpt;
    *rb = *ra + rpt < rows ? *ra + rpt : rows;
    *ca = c * cpt;
    *cb = *ca + cpt < width ? *ca + cpt : width;
    if (*ra > rows) *ra = rows;
    if (*ca > width) *ca = width;
}

// Work tickets.  The queue is the concatenation of the size-class buckets,
// largest class first; a ticket hands out up to ticket_chunk(cl) consecutive
// entries of one class (several small items per ticket, one item per ticket
// from the classes whose items alone keep a work-group busy).
#ifdef __HIPCC__
__host__ __device__
#endif
inline uint32_t ticket_chunk(int cl) {
    const uint32_t c = kTicketVox >> cl;
    return c < 1u ? 1u : (c > (uint32_t)kTicketChunk ? (uint32_t)kTicketChunk : c);
}

#ifdef __HIPCC__
__host__ __device__
#endif
inline uint32_t class_tickets(uint32_t entries, int cl) {
    const uint32_t ch = ticket_chunk(cl);
    return (entries + ch - 1u) / ch;
}

// first[cl] = tickets of all larger classes (entries[cl]: queue entries of
// class cl); returns the number of tickets.
#ifdef __HIPCC__
__host__ __device__
#endif
inline uint32_t ticket_offsets(const uint32_t *entries, uint32_t *first) {
    uint32_t acc = 0;
    for (int cl = kClasses - 1; cl >= 0; --cl) {
        first[cl] = acc;
        acc += class_tickets(entries[cl], cl);
    }
    return acc;
}

// Class and entry range [*e0, *e1) of ticket t < total (as ticket_offsets
// laid them out).
#ifdef __HIPCC__
__host__ __device__
#endif
inline void ticket_range(uint32_t t, const uint32_t *entries, const uint32_t *first, int *cl_out, uint32_t *e0,
                         uint32_t *e1) {
    int cl = kClasses - 1;
    while (cl > 0 && t >= first[cl] + class_tickets(entries[cl], cl)) --cl;
    const uint32_t ch = ticket_chunk(cl);
    *cl_out = cl;
    *e0 = (t - first[cl]) * ch;
    const uint32_t end = *e0 + ch;
    *e1 = end < entries[cl] ? end : entries[cl];
}

// Row blocks a banded ROI of `rows` bbox rows of width W is cut into: about
// tile voxels each, at most one block per row.
#ifdef __HIPCC__
__host__ __device__
#endif
inline uint32_t band_blocks(uint32_t rows, uint32_t W, uint32_t tile) {
    const uint64_t vox = (uint64_t)rows * W;
    uint64_t nb = tile ? (vox + tile - 1u) / tile : 1u;
    if (nb < 1u) nb = 1u;
    return (uint32_t)(nb < rows ? nb : rows);
}

#ifdef __HIPCC__
__host__ __device__
#endif
inline uint32_t size_class(uint32_t vox) {
    uint32_t c = 0;
    while ((vox >> c) > 1u && c < 31u) ++c;
    return c;
}

// Label-table entry (within its image) of label l, 0 when l has none.  With
// no dictionary a label is its own entry (labels up to max_label); with one,
// the entry is 1 + the rank of l among the image's distinct labels, found by
// binary search (labels absent from the dictionary have none).
__host__ __device__
inline uint32_t label_entry(const uint32_t *dict, uint32_t dict_n, uint32_t max_label, uint32_t l) {
    if (l == 0u) return 0u;
    if (!dict) return l <= max_label ? l : 0u;
    uint32_t lo = 0u, hi = dict_n;   // first index with dict[i] >= l lies in [lo, hi]
    while (lo < hi) {
        const uint32_t mid = lo + ((hi - lo) >> 1);
        if (dict[mid] < l) lo = mid + 1u; else hi = mid;
    }
    return lo < dict_n && dict[lo] == l ? lo + 1u : 0u;
}

// Fixed-bin-number level 1 + floor(ng (I - vmin) / Dm), clamped to [1, ng]
// (Dm = max(vmax - vmin, 1); a constant ROI has every I = vmin, level 1),
// from a double-precision reciprocal rounded up: rcp_up = (1 / Dm)(1 + delta)
// with 0 <= delta <= 2^-51.  num = ng (I - vmin) is exact in double and
// num / Dm <= ng < 2^13, so the rounded product never falls below num / Dm
// (an integral quotient stays integral) and stays below the next integer by
// more than 1 / Dm - 2^-38 > 0: truncation gives floor(num / Dm) with no
// correction step.  Values outside the ROI's range give some level in
// [1, ng] (callers mask them by label).
__host__ __device__
inline uint32_t fbn_level_rd(uint32_t I, uint32_t vmin, double rcp_up, uint32_t ng) {
#ifdef __HIP_DEVICE_COMPILE__
    const uint32_t num = __umul24(ng, I - vmin);   // 24-bit operands, low 32 bits of the product
#else
    const uint32_t num = (uint32_t)((uint64_t)(ng & 0xFFFFFFu) * ((I - vmin) & 0xFFFFFFu));
#endif
    const double q = __builtin_fmin((double)num * rcp_up, (double)(ng - 1u));
    return (uint32_t)q + 1u;
}

// rcp_up for fbn_level_rd: the rounded reciprocal of Dm plus one unit in the
// last place (at least 1 / Dm, at most 1.5 units above it).
__host__ __device__
inline double fbn_rcp_up(uint32_t Dm) {
    return __builtin_bit_cast(double, __builtin_bit_cast(uint64_t, 1.0 / (double)Dm) + 1ull);
}

}  // namespace nyx
