// nyx_runtime.hip -- host runtime and C ABI (include/nyx.h).
//
// Planning discovers the ROIs once, chooses the LDS accumulation mode and the
// split of large ROIs, sizes the work queue and scratch, and captures the
// whole step (discovery, binning, accumulation, features) in a HIP graph
// replayed by nyx_plan_execute.  nyx_plan_execute_per_roi runs the same step
// with one accumulation launch per ROI instead of the persistent queue.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/nyx.h"
#include "nyx_launch.h"
#include "nyx_types.h"

using namespace nyx;

namespace {

const char *const kFeatureNames[kNumFeat] = {
    "ASM", "ACOR", "CLUPROM", "CLUSHADE", "CLUTEND", "CONTRAST", "CORR", "DIFAVE", "DIFENTRO", "DIFVAR",
    "DIS", "ENERGY", "ENTROPY", "HOM1", "HOM2", "IDM", "INFOMEAS1", "INFOMEAS2", "IDMN", "ID",
    "IDN", "IV", "JAVE", "JE", "JMAX", "SUMAVE", "SUMENT", "JVAR", "SUMVAR", "VARIANCE"};

const char *const kIntensityNames[kNumIntensityFeat] = {
    "MEAN", "MIN", "MAX", "RANGE", "INTEGRATED_INTENSITY", "ENERGY", "RMS", "VARIANCE", "STDDEV",
    "STANDARD_ERROR", "SKEWNESS", "KURTOSIS", "HYPERSKEWNESS", "HYPERFLATNESS", "MEAN_ABSOLUTE_DEVIATION",
    "MEDIAN", "MEDIAN_ABSOLUTE_DEVIATION", "P01", "P10", "P25", "P75", "P90", "P99", "INTERQUARTILE_RANGE",
    "ROBUST_MEAN_ABSOLUTE_DEVIATION", "MODE", "ENTROPY", "UNIFORMITY", "UNIFORMITY_PIU", "WEIGHTED_CENTROID_X",
    "WEIGHTED_CENTROID_Y", "WEIGHTED_CENTROID_Z", "EDGE_INTEGRATED_INTENSITY", "EDGE_MIN", "EDGE_MAX",
    "EDGE_MEAN", "EDGE_STDDEV"};

const char *const kNeighbourNames[kNumNeighbourFeat] = {
    "NGLDM_DCENRG", "NGLDM_DCENT", "NGLDM_DCNU", "NGLDM_DCNUN", "NGLDM_DCM", "NGLDM_DCV", "NGLDM_GLNU",
    "NGLDM_GLNUN", "NGLDM_GLM", "NGLDM_GLV", "NGLDM_HDE", "NGLDM_HDHGLE", "NGLDM_HDLGLE", "NGLDM_HGLCE",
    "NGLDM_LDE", "NGLDM_LDHGLE", "NGLDM_LDLGLE", "NGLDM_LGLCE", "NGTDM_BUSYNESS", "NGTDM_COARSENESS",
    "NGTDM_COMPLEXITY", "NGTDM_CONTRAST", "NGTDM_STRENGTH", "GLDM_SDE", "GLDM_LDE", "GLDM_GLN", "GLDM_DN",
    "GLDM_DNN", "GLDM_GLV", "GLDM_DV", "GLDM_DE", "GLDM_LGLE", "GLDM_HGLE", "GLDM_SDLGLE", "GLDM_SDHGLE",
    "GLDM_LDLGLE", "GLDM_LDHGLE"};

constexpr uint32_t kLdsBudget = 160u * 1024u;   // LDS per CU on gfx950
constexpr uint32_t kRingMin = 2048u, kRingMax = 32768u;   // staged-accumulation level ring (bytes)
constexpr uint32_t kMaxGroupsPerCu = 5u;                  // k_batch, single precision: 5 waves per SIMD
constexpr uint32_t kMaxNgFused = 8191u;         // hash keys carry 13-bit levels
constexpr uint64_t kMaxLabelEntries = 1ull << 26;
// Banded accumulation (hash mode, symmetric matrices): ROIs above
// kBandMinVox voxels (and above the split size), LDS band of at most
// kBandLds bytes, work items of about kBandTile bbox voxels.
constexpr uint32_t kBandMinVox = 32768u, kBandLds = 128u * 1024u, kBandTile = 256u * 1024u, kBandMinW = 8u;

int log_level() {
    static int lvl = -1;
    if (lvl < 0) {
        const char *s = getenv("NYX_LOG");
        lvl = s ? atoi(s) : 0;
    }
    return lvl;
}

// A bump allocator over a fixed device region (the no-allocation entry
// point's scratch): carving never calls the HIP allocator, and the region is
// reused from its start by the next call.
struct Arena {
    uint8_t *base = nullptr;
    size_t cap = 0, used = 0;
    size_t wanted = 0;   // bytes the failed request would have needed in total
    void *carve(size_t n) {
        const size_t at = (used + 255u) & ~(size_t)255u;
        if (at + n > cap) {
            wanted = at + n;
            return nullptr;
        }
        used = at + n;
        return base + at;
    }
};

// Device buffer: owned (hipMalloc / hipFree), or carved from an Arena when
// one is given (never freed by the buffer).
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool owned = false;
    Arena *arena = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p && owned) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        owned = false;
    }
    hipError_t alloc(size_t n) {
        release();
        if (n == 0) n = 16;
        if (arena) {
            p = arena->carve(n);
            if (!p) return hipErrorOutOfMemory;
            bytes = n;
            return hipSuccess;
        }
        hipError_t e = hipMalloc(&p, n);
        if (e == hipSuccess) {
            bytes = n;
            owned = true;
        } else {
            p = nullptr;
        }
        return e;
    }
    template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};


uint32_t next_pow2(uint32_t v) {
    uint32_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

}  // namespace

// Device memory of the no-allocation entry point: one array per GPU for the
// life of the process, shared by every call on that GPU.  Host code never
// uses the symbol itself (on the host it only names a stand-in): the device
// address is taken once per device with hipGetSymbolAddress and kept below.
constexpr size_t kScratchBytes = NYX_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint8_t *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on `device` (current); nullptr on failure.
uint8_t *scratch_address(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_scratch_ptr[device] = static_cast<uint8_t *>(ptr);
    }
    return g_scratch_ptr[device];
}
}  // namespace

struct nyx_ctx {
    int device = 0;
    int n_cu = 0;
    std::string err;
    hipStream_t capture_stream = nullptr;
    uint8_t *scratch = nullptr;   // this device's no-allocation scratch (device address)
};

// All device state of one discovery/step over a batch of images.
struct Work {
    std::vector<ImgDesc> h_imgs;
    DevBuf imgs, tab[10], counters, rois, buckets, G, dsums, dsums_y, split_roi, band_roi, smarg, stot, splp, vox_base,
        dict;
    uint32_t tab_total = 0, n_blocks = 0, n_counters = 0, total_chunks = 0;
    uint32_t n_rois = 0;
    uint64_t total_vox = 0;
    std::vector<RoiDesc> h_rois;
    StepArgs args{};
    // Carve every buffer from `ar` (nullptr: hipMalloc).
    void use_arena(Arena *ar) {
        for (DevBuf *b : {&imgs, &counters, &rois, &buckets, &G, &dsums, &dsums_y, &split_roi, &band_roi, &smarg, &stot,
                          &splp, &vox_base, &dict})
            b->arena = ar;
        for (DevBuf &b : tab) b.arena = ar;
    }
};

struct nyx_plan {
    nyx_ctx *ctx = nullptr;
    Work w;
    std::vector<nyx_image> imgs;
    int K = 0, ng = 0;
    nyx_precision prec = NYX_FP32;
    uint32_t grid = 0, block = 256;
    std::vector<uint32_t> roi_tiles;   // per-ROI tile count for the per-ROI path
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void *graph_table = nullptr;
    nyx_roi_table graph_rois{};
    std::string desc;
    int64_t workspace_bytes = 0;
    float tuned_ms = 0.f;
    struct Cfg { int mode; uint32_t kp, block, split_vox, tile_vox, list_cap, hash_cap; int force_split; };
    Cfg cfg{};
};

namespace {

nyx_status fail(nyx_ctx *c, nyx_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c) c->err = buf;
    if (log_level() > 0) fprintf(stderr, "[nyx] error: %s\n", buf);
    return s;
}

#define HIPC(ctx, x)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (x);                                                                      \
        if (e_ != hipSuccess)                                                                     \
            return fail(ctx, e_ == hipErrorOutOfMemory ? NYX_ERR_OOM : NYX_ERR_DEVICE, "%s: %s", #x, \
                        hipGetErrorString(e_));                                                   \
    } while (0)

nyx_status validate_images(nyx_ctx *ctx, const nyx_image *imgs, int32_t n) {
    if (!imgs || n <= 0) return fail(ctx, NYX_ERR_INVALID, "no images");
    for (int i = 0; i < n; ++i) {
        const nyx_image &m = imgs[i];
        if (!m.intensity || !m.labels) return fail(ctx, NYX_ERR_INVALID, "image %d: NULL array", i);
        if (m.nz <= 0 || m.ny <= 0 || m.nx <= 0) return fail(ctx, NYX_ERR_INVALID, "image %d: dimension <= 0", i);
        if (m.nz > 65535 || m.ny > 65535 || m.nx > 65535)
            return fail(ctx, NYX_ERR_INVALID, "image %d: dimension above 65535", i);
        if (m.nz * m.ny * m.nx >= (1ll << 31)) return fail(ctx, NYX_ERR_INVALID, "image %d: 2^31 voxels or more", i);
    }
    return NYX_OK;
}

nyx_status validate_offsets(nyx_ctx *ctx, const nyx_image *imgs, int32_t n_images, const nyx_offset *off,
                            int32_t K) {
    if (!off) return fail(ctx, NYX_ERR_INVALID, "offsets are NULL");
    if (K < 1 || K > kMaxOffsets) return fail(ctx, NYX_ERR_INVALID, "n_offsets must be in [1, 64]");
    bool any3d = false;
    for (int i = 0; i < n_images; ++i) any3d |= imgs[i].nz > 1;
    for (int k = 0; k < K; ++k) {
        if (off[k].dz == 0 && off[k].dy == 0 && off[k].dx == 0)
            return fail(ctx, NYX_ERR_INVALID, "offset %d is (0,0,0)", k);
        if (!any3d && off[k].dz != 0) return fail(ctx, NYX_ERR_INVALID, "offset %d has dz != 0 on 2D images", k);
        if (abs(off[k].dz) > 65535 || abs(off[k].dy) > 65535 || abs(off[k].dx) > 65535)
            return fail(ctx, NYX_ERR_INVALID, "offset %d out of range", k);
    }
    return NYX_OK;
}

nyx_status validate_bins(nyx_ctx *ctx, int32_t ng) {
    if (ng < 2 || ng > 65535) return fail(ctx, NYX_ERR_INVALID, "n_bins must be in [2, 65535]");
    if ((uint32_t)ng > kMaxNgFused)
        return fail(ctx, NYX_ERR_UNSUPPORTED, "n_bins above %u is not supported", kMaxNgFused);
    return NYX_OK;
}

// Distinct nonzero labels of every image, ascending, uploaded to w.dict;
// sets dict, dict_n and max_label (= dict_n) of w.h_imgs.  Labels present in
// a later execution but absent here have no table entry (E_LABEL_RANGE).
nyx_status build_label_dict(nyx_ctx *ctx, Work &w, int32_t n, hipStream_t st) {
    uint64_t max_vox = 0;
    for (int i = 0; i < n; ++i) max_vox = std::max<uint64_t>(max_vox, w.h_imgs[i].nvox);
    DevBuf list, cnt;
    list.arena = cnt.arena = w.imgs.arena;
    HIPC(ctx, cnt.alloc(sizeof(uint32_t)));
    uint32_t cap = 1u << 16, got = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        HIPC(ctx, list.alloc(sizeof(uint64_t) * cap));
        const uint32_t zero = 0u;
        HIPC(ctx, hipMemcpyAsync(cnt.p, &zero, sizeof zero, hipMemcpyHostToDevice, st));
        HIPC(ctx, launch_label_collect(w.imgs.as<ImgDesc>(), n, max_vox, list.as<uint64_t>(), cap, cnt.as<uint32_t>(),
                                       st));
        HIPC(ctx, hipMemcpyAsync(&got, cnt.p, sizeof got, hipMemcpyDeviceToHost, st));
        HIPC(ctx, hipStreamSynchronize(st));
        if (got <= cap) break;
        cap = got;   // every entry fits the second time (same images)
    }
    if (got > cap) return fail(ctx, NYX_ERR_INTERNAL, "label collection did not converge");
    std::vector<uint64_t> h(got);
    if (got) HIPC(ctx, hipMemcpyAsync(h.data(), list.p, sizeof(uint64_t) * got, hipMemcpyDeviceToHost, st));
    HIPC(ctx, hipStreamSynchronize(st));
    std::sort(h.begin(), h.end());
    h.erase(std::unique(h.begin(), h.end()), h.end());
    std::vector<uint32_t> labels(h.size());
    std::vector<uint64_t> first(n + 1, 0);
    for (size_t k = 0; k < h.size(); ++k) {
        labels[k] = (uint32_t)h[k];
        first[(size_t)(h[k] >> 32) + 1u]++;
    }
    for (int i = 0; i < n; ++i) first[i + 1] += first[i];
    HIPC(ctx, w.dict.alloc(sizeof(uint32_t) * std::max<size_t>(labels.size(), 1)));
    if (!labels.empty())
        HIPC(ctx, hipMemcpyAsync(w.dict.p, labels.data(), sizeof(uint32_t) * labels.size(), hipMemcpyHostToDevice, st));
    HIPC(ctx, hipStreamSynchronize(st));
    for (int i = 0; i < n; ++i) {
        w.h_imgs[i].dict = w.dict.as<uint32_t>() + first[i];
        w.h_imgs[i].dict_n = (uint32_t)(first[i + 1] - first[i]);
        w.h_imgs[i].max_label = w.h_imgs[i].dict_n;
    }
    return NYX_OK;
}

// Label tables, ROI discovery and the ROI table (no work items).
nyx_status discover(nyx_ctx *ctx, const nyx_image *imgs, int32_t n, Work &w, hipStream_t st) {
    w.h_imgs.resize(n);
    uint32_t chunk = 0;
    uint64_t tv = 0;
    std::vector<uint64_t> vbase(n);
    for (int i = 0; i < n; ++i) {
        ImgDesc &d = w.h_imgs[i];
        memset(&d, 0, sizeof d);
        d.I = imgs[i].intensity;
        d.L = imgs[i].labels;
        d.B = nullptr;
        d.nz = (int32_t)imgs[i].nz;
        d.ny = (int32_t)imgs[i].ny;
        d.nx = (int32_t)imgs[i].nx;
        d.nvox = (uint32_t)(imgs[i].nz * imgs[i].ny * imgs[i].nx);
        d.chunk_base = chunk;
        {
            // discovery tiles: kScanTileRows rows (all planes flattened) by kScanTileCols columns
            uint64_t rows = (uint64_t)d.nz * (uint64_t)d.ny;
            chunk += (uint32_t)(((rows + kScanTileRows - 1u) / kScanTileRows) *
                                (((uint64_t)d.nx + kScanTileCols - 1u) / kScanTileCols));
        }
        vbase[i] = tv;
        tv += d.nvox;
    }
    w.total_chunks = chunk;
    w.total_vox = tv;
    HIPC(ctx, w.imgs.alloc(sizeof(ImgDesc) * n));
    HIPC(ctx, hipMemcpyAsync(w.imgs.p, w.h_imgs.data(), sizeof(ImgDesc) * n, hipMemcpyHostToDevice, st));
    HIPC(ctx, w.vox_base.alloc(sizeof(uint64_t) * n));
    HIPC(ctx, hipMemcpyAsync(w.vox_base.p, vbase.data(), sizeof(uint64_t) * n, hipMemcpyHostToDevice, st));
    // largest label per image sizes the label tables
    DevBuf dmax;
    dmax.arena = w.imgs.arena;
    HIPC(ctx, dmax.alloc(sizeof(uint32_t) * n));
    std::vector<uint32_t> zeros(n, 0u), hmax(n);
    HIPC(ctx, hipMemcpyAsync(dmax.p, zeros.data(), sizeof(uint32_t) * n, hipMemcpyHostToDevice, st));
    HIPC(ctx, launch_max_label(w.imgs.as<ImgDesc>(), n, dmax.as<uint32_t>(), st));
    HIPC(ctx, hipMemcpyAsync(hmax.data(), dmax.p, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, st));
    HIPC(ctx, hipStreamSynchronize(st));
    uint64_t total = 0;
    for (int i = 0; i < n; ++i) total += (uint64_t)hmax[i] + 1u;
    if (total > kMaxLabelEntries || total > tv + (uint64_t)n) {
        // Label values too large (or too sparse) to index the table: the
        // table gets one entry per distinct label of each image instead.
        nyx_status s = build_label_dict(ctx, w, n, st);
        if (s != NYX_OK) return s;
        total = 0;
        for (int i = 0; i < n; ++i) total += (uint64_t)w.h_imgs[i].dict_n + 1u;
        if (total > kMaxLabelEntries)
            return fail(ctx, NYX_ERR_UNSUPPORTED, "%llu distinct labels (limit %llu)", (unsigned long long)total,
                        (unsigned long long)kMaxLabelEntries);
    } else {
        for (int i = 0; i < n; ++i) {
            w.h_imgs[i].dict = nullptr;
            w.h_imgs[i].dict_n = 0u;
            w.h_imgs[i].max_label = hmax[i];
        }
    }
    total = 0;
    for (int i = 0; i < n; ++i) {
        w.h_imgs[i].tab_base = (uint32_t)total;
        total += (uint64_t)w.h_imgs[i].max_label + 1u;
    }
    w.tab_total = (uint32_t)total;
    HIPC(ctx, hipMemcpyAsync(w.imgs.p, w.h_imgs.data(), sizeof(ImgDesc) * n, hipMemcpyHostToDevice, st));
    for (auto &b : w.tab) HIPC(ctx, b.alloc(sizeof(uint32_t) * (size_t)total));
    w.n_blocks = (w.tab_total + 1023u) / 1024u;
    w.n_counters = C_BLOCKS + w.n_blocks;
    HIPC(ctx, w.counters.alloc(sizeof(uint32_t) * w.n_counters));

    StepArgs &a = w.args;
    memset(&a, 0, sizeof a);
    a.imgs = w.imgs.as<ImgDesc>();
    a.n_images = n;
    a.total_chunks = w.total_chunks;
    a.tab.cnt = w.tab[0].as<uint32_t>();
    a.tab.mn = w.tab[1].as<uint32_t>();
    a.tab.mx = w.tab[2].as<uint32_t>();
    a.tab.x0 = w.tab[3].as<int32_t>();
    a.tab.y0 = w.tab[4].as<int32_t>();
    a.tab.z0 = w.tab[5].as<int32_t>();
    a.tab.x1 = w.tab[6].as<int32_t>();
    a.tab.y1 = w.tab[7].as<int32_t>();
    a.tab.z1 = w.tab[8].as<int32_t>();
    a.tab.row = w.tab[9].as<uint32_t>();
    a.tab.total = w.tab_total;
    a.counters = w.counters.as<uint32_t>();
    HIPC(ctx, launch_reset(a, w.n_counters, st));
    HIPC(ctx, launch_scan(a, st));
    // ROI count from the per-block counts
    StepArgs a0 = a;
    if (w.n_blocks) {
        // count kernel only (compaction with zero ROI capacity writes nothing)
        a0.roi_cap = 0;
        a0.enqueue = 0;
        HIPC(ctx, launch_compact(a0, 0u, 0u, st));
    }
    std::vector<uint32_t> hc(w.n_counters);
    HIPC(ctx, hipMemcpyAsync(hc.data(), w.counters.p, sizeof(uint32_t) * w.n_counters, hipMemcpyDeviceToHost, st));
    HIPC(ctx, hipStreamSynchronize(st));
    if (hc[C_ERR] & E_LABEL_RANGE) return fail(ctx, NYX_ERR_INTERNAL, "label range check failed during discovery");
    w.n_rois = hc[C_NROIS];
    HIPC(ctx, w.rois.alloc(sizeof(RoiDesc) * std::max<uint32_t>(w.n_rois, 1u)));
    a.rois = w.rois.as<RoiDesc>();
    a.roi_cap = w.n_rois;
    return NYX_OK;
}

// Re-runs the compaction to fill the ROI descriptors and fetches them.
nyx_status fetch_rois(nyx_ctx *ctx, Work &w, hipStream_t st) {
    StepArgs a = w.args;
    a.enqueue = 0;
    HIPC(ctx, launch_reset(a, w.n_counters, st));
    HIPC(ctx, launch_scan(a, st));
    HIPC(ctx, launch_compact(a, 0u, 0u, st));
    w.h_rois.resize(w.n_rois);
    if (w.n_rois)
        HIPC(ctx, hipMemcpyAsync(w.h_rois.data(), w.rois.p, sizeof(RoiDesc) * w.n_rois, hipMemcpyDeviceToHost, st));
    HIPC(ctx, hipStreamSynchronize(st));
    return NYX_OK;
}

struct Config {
    int mode = 0;            // 0 dense + list, 1 hash, 2 dense + scan, 3 packed dense + scan
    uint32_t kp = 1;
    uint32_t block = 256;
    uint32_t split_vox = 0, tile_vox = 0;
    uint32_t list_cap = 0, hash_cap = 0;
    int force_split = 0;
    int merged = 0;          // one matrix per ROI: the sum of the K offsets' matrices
    uint32_t copies = 1;     // privatised copies of each dense triangle (scan modes)
    float tile_scale = 1.f;  // split ROIs above tile_scale x the load-balance share
    int nonsym = 0;          // ordered counts: full squares (dense modes 2 and 3, or the hash)
    uint32_t band_vox = 0;   // ROIs above this go to the banded kernel (0: none)
    uint32_t band_w = 0;     // band width (power of two)
};

// The banded kernel takes the large ROIs of hash-mode plans (triangle larger
// than LDS) with symmetric matrices: band width = the largest power of two
// whose ng x width 32-bit cells fit kBandLds.
void set_band(Config &c, uint32_t ng) {
    c.band_vox = 0u;
    c.band_w = 0u;
    if (c.mode != 1 || c.nonsym) return;
    uint32_t w = 1u;
    while (w * 2u <= ng && (uint64_t)ng * (w * 2u) * 4u <= kBandLds) w *= 2u;
    if (w < kBandMinW) return;
    c.band_w = w;
    c.band_vox = std::max(c.split_vox, kBandMinVox);
}

const char *mode_name(int m) {
    switch (m) {
        case 0: return "dense-list";
        case 1: return "hash";
        case 2: return "dense-scan";
        default: return "dense16-scan";
    }
}

// Compaction entries (u32 cell indices) per lane of a scan chunk: one
// 16-byte read holds 8 packed 16-bit or 4 32-bit counters.
uint32_t scan_cells(int mode) { return mode == 3 ? (uint32_t)kScanCells : (uint32_t)kScanCells / 2u; }

// Cells of one dense matrix: the upper triangle, or the full square of
// ordered counts.
uint32_t mat_cells(uint32_t ng, bool nonsym) { return nonsym ? ng * ng : ng * (ng + 1u) / 2u; }

uint32_t u_words(int mode, uint32_t ng, bool nonsym = false) {
    uint32_t tri = mat_cells(ng, nonsym);
    uint32_t w = mode == 3 ? (tri + 1u) / 2u : tri;
    return (w + 3u) & ~3u;
}

// Marginal words per reducing wave: row, sum and difference marginals, plus
// the column marginal of an ordered matrix.
uint32_t marg_words(uint32_t ng, bool nonsym) { return (nonsym ? 5u : 4u) * ng; }

// ring: reserve an LDS level ring for the staged accumulation, sized to the
// LDS the work-group can take without lowering its occupancy.
LdsLayout make_layout(const Config &c, uint32_t ng, int K, bool ring) {
    LdsLayout L;
    memset(&L, 0, sizeof L);
    L.mode = (uint32_t)c.mode;
    L.kp = c.kp;
    L.nwaves = c.block / kWave;
    L.tri_pad = u_words(c.mode, ng, c.nonsym != 0);
    L.copies = (c.mode == 2 || c.mode == 3) ? c.copies : 1u;
    L.list_cap = c.list_cap;
    L.hash_cap = c.hash_cap;
    uint32_t off = 0;
    auto take = [&](uint32_t bytes) {
        uint32_t o = off;
        off += (bytes + 15u) & ~15u;
        return o;
    };
    if (c.mode != 1) {
        L.n_tri = c.merged ? 1u : c.kp;   // merged: one triangle for all offsets
        L.u_off = take(L.n_tri * L.copies * L.tri_pad * 4u);
    } else {
        L.hkey_off = take(c.hash_cap * 4u);
        L.hcnt_off = take(c.hash_cap * 4u);
    }
    L.list_off = take(c.kp * c.list_cap * 4u);
    L.lcnt_off = take(c.kp * 4u);
    L.buf_off = take((c.mode == 2 || c.mode == 3) ? L.nwaves * scan_buf_entries(scan_cells(c.mode)) * 2u : 0u);
    L.marg_sets = std::min(L.nwaves, c.merged ? 1u : c.kp);   // one set per wave that reduces a matrix
    L.marg_off = take(L.marg_sets * marg_words(ng, c.nonsym != 0) * 4u);
    L.misc_off = take(128u * 4u);
    if ((c.mode == 2 || c.mode == 3) && !c.nonsym) L.ro_off = take((ng + 1u) * 4u);
    L.item_off = take((uint32_t)kTicketChunk * kItemBytes);
    if (ring && ng <= 255u && c.mode != 1 && !c.nonsym) {
        // work-groups per CU: LDS-bound, and at most kMaxGroupsPerCu (the
        // single-precision kernel's register bound)
        const uint32_t per_group = kLdsBudget / std::max(1u, std::min(kMaxGroupsPerCu, kLdsBudget / off));
        const uint32_t bytes = off < per_group ? std::min(kRingMax, (per_group - off) & ~15u) : 0u;
        if (bytes >= kRingMin) {
            L.ring_off = take(bytes);
            L.ring_bytes = bytes;
        }
    }
    L.bytes = off;
    return L;
}

// Largest voxel count any work item can hold under a split rule.
uint64_t max_item_vox(const std::vector<RoiDesc> &rois, uint32_t split_vox, uint32_t tile_vox) {
    uint64_t m = 0;
    for (const RoiDesc &r : rois) {
        uint32_t W = (uint32_t)(r.x1 - r.x0 + 1);
        Tiling t = tiles_for(r.n, r.rows, W, split_vox, tile_vox);
        if (t.row_blocks * t.col_blocks == 1u) { m = std::max<uint64_t>(m, r.n); continue; }
        uint32_t rpt = (r.rows + t.row_blocks - 1u) / t.row_blocks;
        uint32_t cpt = (W + t.col_blocks - 1u) / t.col_blocks;
        m = std::max<uint64_t>(m, std::min<uint64_t>((uint64_t)rpt * cpt, r.n));
    }
    return m;
}

// Feasible LDS configurations for this workload, one per accumulation mode,
// each with as many directions per pass as fit.  Dense triangles first; the
// hash table only when no dense triangle fits.
// Work-groups of the persistent kernel per CU for a given LDS footprint.
uint32_t groups_per_cu(uint64_t lds_bytes) {
    return (uint32_t)std::min<uint64_t>(kMaxGroupsPerCu, kLdsBudget / std::max<uint64_t>(lds_bytes, 1u));
}

// merged: every offset counts into one LDS triangle in one pass, so only the
// dense scan modes qualify, and packed 16-bit counters need K x (voxels of an
// item) < 65536 (offered only when that bound leaves the load-balance tile
// size alone; 32-bit counters otherwise).  copies: privatised copies of each
// dense scan triangle (list and hash modes keep one); tile_scale scales the
// load-balance share above which ROIs are split.
std::vector<Config> candidate_configs(const nyx_ctx *ctx, const Work &w, uint32_t ng, int K, int force_split,
                                      uint32_t block, bool merged = false, uint32_t copies = 1u,
                                      float tile_scale = 1.f, bool nonsym = false) {
    std::vector<Config> out;
    const uint32_t nw = block / kWave;
    const uint32_t tri = mat_cells(ng, nonsym);
    // LDS besides triangles / hash / lists: marginals for up to nw directions
    // at a time, misc, alignment slack
    auto fixed_for = [&](uint32_t kp) {
        // (marginal sets, misc words, staged item descriptors, row-offset table, alignment slack)
        return (std::min(nw, kp) * marg_words(ng, nonsym) * 4u + 15u) / 16u * 16u + 128u * 4u +
               (uint32_t)kTicketChunk * kItemBytes + ((ng + 1u) * 4u + 15u) / 16u * 16u + 64u * 4u + 64;
    };
    const uint32_t fixed = fixed_for(1u);
    uint64_t total_vox = 0;
    for (const RoiDesc &r : w.h_rois) total_vox += r.n;
    // load balance: split ROIs that would take more than ~1/4 of one
    // work-group's share of the voxels
    uint64_t share = (uint64_t)((double)(total_vox / ((uint64_t)std::max(ctx->n_cu, 1) * 4u) + 1u) * tile_scale);
    const uint32_t lb = (uint32_t)std::min<uint64_t>(std::max<uint64_t>(share, 4096u), 1u << 20);
    std::vector<Config> later;
    for (int mode : {3, 2, 0}) {
        if ((merged || nonsym) && mode == 0) continue;   // the returning-atomic list keeps triangles only
        if (copies > 1u && mode == 0) continue;   // the returning-atomic list keeps one triangle
        const uint32_t cell_max = merged ? 65535u / (uint32_t)K : 65535u;   // 16-bit counters
        uint32_t split = mode == 3 ? std::min<uint32_t>(lb, cell_max) : lb;
        uint64_t mi = max_item_vox(w.h_rois, split, split);
        while (mode == 3 && mi > cell_max && split > 64u) {
            split /= 2u;
            mi = max_item_vox(w.h_rois, split, split);
        }
        if (mode == 3 && mi > cell_max) continue;
        if (merged && mode == 3 && split < std::min<uint32_t>(lb, 65535u)) continue;
        const bool scan = mode == 2 || mode == 3;
        const uint32_t list_cap = scan ? 0u : (uint32_t)std::min<uint64_t>(tri, std::max<uint64_t>(mi, 1u));
        const uint64_t scan_buf = scan ? (uint64_t)nw * scan_buf_entries(scan_cells(mode)) * 2u : 0u;
        const uint32_t cp = scan ? copies : 1u;
        for (uint32_t kp = (uint32_t)K; kp >= (merged ? (uint32_t)K : 1u); --kp) {
            const uint32_t n_tri = merged ? 1u : kp;
            uint64_t bytes = (uint64_t)n_tri * cp * u_words(mode, ng, nonsym) * 4u + (uint64_t)kp * list_cap * 4u + kp * 4u +
                             fixed_for(n_tri) + scan_buf;
            if (bytes <= kLdsBudget) {
                Config c;
                c.mode = mode; c.kp = kp; c.block = block; c.split_vox = split; c.tile_vox = split;
                c.list_cap = list_cap; c.force_split = force_split; c.merged = merged ? 1 : 0;
                c.copies = cp; c.tile_scale = tile_scale; c.nonsym = nonsym ? 1 : 0;
                out.push_back(c);
                if (merged) break;
                // many offsets: fewer directions per pass cost another pass
                // over the voxels but leave LDS for more work-groups per CU
                // (timed by the autotuner, never the default)
                if (mode == 3 && (K > 4 || groups_per_cu(bytes) < 3u))
                    for (uint32_t parts : {2u, 3u, 4u}) {
                        Config f = c;
                        f.kp = ((uint32_t)K + parts - 1u) / parts;
                        if (f.kp < kp && (later.empty() || later.back().kp != f.kp)) later.push_back(f);
                    }
                break;
            }
        }
    }
    out.insert(out.end(), later.begin(), later.end());
    if (!out.empty() || fixed >= kLdsBudget || merged || copies > 1u) return out;
    // hash mode: items small enough that kp directions of pairs fill at most
    // half the table
    for (uint32_t kp = (uint32_t)K; kp >= 1u; --kp) {
        for (uint32_t hc = 1u << 14; hc >= 512u; hc >>= 1) {
            uint32_t per_dir = hc / (2u * kp);
            if (per_dir < 64u) continue;
            uint32_t split = std::min<uint32_t>(per_dir, lb);
            uint64_t mi = max_item_vox(w.h_rois, split, split);
            while (mi > per_dir && split > 16u) {
                split /= 2u;
                mi = max_item_vox(w.h_rois, split, split);
            }
            if (mi > per_dir) continue;
            uint32_t list_cap = (uint32_t)std::max<uint64_t>(mi, 1u);
            uint64_t bytes = (uint64_t)hc * 8u + (uint64_t)kp * list_cap * 4u + kp * 4u + fixed_for(kp);
            if (bytes <= kLdsBudget) {
                Config c;
                c.mode = 1; c.kp = kp; c.block = block; c.hash_cap = hc; c.split_vox = split; c.tile_vox = split;
                c.list_cap = list_cap; c.force_split = force_split; c.tile_scale = tile_scale;
                c.nonsym = nonsym ? 1 : 0;
                set_band(c, ng);
                out.push_back(c);
                return out;
            }
        }
    }
    return out;
}

// Default choice without timing: an ordered scan of the triangle costs
// O(Ng^2) per direction and item, a returning-atomic list costs O(pairs);
// scan while the triangle is small next to the average item.
Config default_config(const std::vector<Config> &cands, const Work &w, uint32_t ng, int K) {
    uint64_t total_vox = 0;
    for (const RoiDesc &r : w.h_rois) total_vox += r.n;
    const uint64_t avg = w.h_rois.empty() ? 1u : std::max<uint64_t>(1u, total_vox / w.h_rois.size());
    const uint64_t tri = (uint64_t)ng * (ng + 1u) / 2u;
    const bool prefer_scan = tri <= 8u * avg;
    // among the candidates of the preferred kind: fewest passes over the
    // voxels per work-group slot (passes / work-groups per CU); ties keep the
    // earlier candidate (more directions per pass)
    const Config *best = nullptr;
    double best_score = 0.0;
    for (const Config &c : cands) {
        const bool scan = c.mode == 2 || c.mode == 3;
        if (!(prefer_scan == scan || c.mode == 1)) continue;
        const uint32_t passes = ((uint32_t)K + c.kp - 1u) / c.kp;
        const double score = (double)passes / (double)std::max(1u, groups_per_cu(make_layout(c, ng, K, false).bytes));
        if (!best || score < best_score) { best = &c; best_score = score; }
    }
    return best ? *best : cands.front();
}

// A configuration whose LDS leaves room for one 256-thread work-group per CU
// runs with 512 threads instead when its layout (a scan buffer and a set of
// marginals per reducing wave) still fits: eight waves then share the CU's
// latency instead of four.
Config widen_block(const Config &c, uint32_t ng, int K) {
    if (c.block != 256u || groups_per_cu(make_layout(c, ng, K, false).bytes) != 1u) return c;
    Config w = c;
    w.block = 512u;
    return make_layout(w, ng, K, false).bytes <= kLdsBudget ? w : c;
}

nyx_status choose_config(nyx_ctx *ctx, const Work &w, uint32_t ng, int K, int force_split, uint32_t block,
                         Config &cfg, bool nonsym = false) {
    std::vector<Config> c = candidate_configs(ctx, w, ng, K, force_split, block, false, 1u, 1.f, nonsym);
    if (c.empty()) return fail(ctx, NYX_ERR_UNSUPPORTED, "no LDS configuration fits n_bins=%u with %d offsets", ng, K);
    cfg = default_config(c, w, ng, K);
    return NYX_OK;
}

// Item and split-slot counts implied by a configuration.
void count_items(const std::vector<RoiDesc> &rois, const Config &c, uint64_t *items, uint32_t *n_split,
                 std::vector<uint32_t> *tiles) {
    uint64_t it = 0;
    uint32_t ns = 0;
    if (tiles) tiles->resize(rois.size());
    for (size_t i = 0; i < rois.size(); ++i) {
        const RoiDesc &r = rois[i];
        const bool band = c.band_vox && r.n > c.band_vox;
        Tiling t = tiles_for(r.n, r.rows, (uint32_t)(r.x1 - r.x0 + 1), c.split_vox, c.tile_vox);
        uint32_t nt = band ? 0u : t.row_blocks * t.col_blocks;
        it += nt;
        if (nt > 1u || band || c.force_split) ++ns;
        if (tiles) (*tiles)[i] = nt;
    }
    *items = it;
    *n_split = ns;
}

// Row-sweep eligibility: all images 2D and every offset of each pass one of
// the four distance-1 in-plane classes, each class at most once per pass.
bool sweep_table(const std::vector<ImgDesc> &imgs, const nyx_offset *off, int K, uint32_t kp,
                 int8_t (*sweep)[4], int max_passes) {
    memset(sweep, -1, sizeof(int8_t[4]) * max_passes);
    for (const ImgDesc &d : imgs)
        if (d.nz != 1) return false;
    int pass = 0;
    for (int d0 = 0; d0 < K; d0 += (int)kp, ++pass) {
        if (pass >= max_passes) return false;
        for (int d = d0; d < std::min(K, d0 + (int)kp); ++d) {
            const nyx_offset &o = off[d];
            if (o.dz != 0 || abs(o.dy) > 1 || abs(o.dx) > 1) return false;
            int cls;
            if (o.dy == 0) cls = 0;
            else if (o.dx == 0) cls = 1;
            else if (o.dy * o.dx < 0) cls = 2;   // (-1, +1) or (+1, -1)
            else cls = 3;                        // (-1, -1) or (+1, +1)
            if (sweep[pass][cls] >= 0) return false; // the same class twice in a pass
            sweep[pass][cls] = (int8_t)(d - d0);
        }
    }
    return true;
}

void set_sweep(StepArgs &a, const std::vector<ImgDesc> &imgs, const nyx_offset *off, int K, uint32_t kp) {
    a.sweep_ok = sweep_table(imgs, off, K, kp, a.sweep, kMaxSweepPasses) ? 1 : 0;
}

// Allocates queue, split matrices and fills the step arguments.
nyx_status setup_step(nyx_ctx *ctx, Work &w, const Config &cfg, const nyx_offset *off, int K, uint32_t ng,
                      int fp64, uint32_t g_cap_override, int64_t cap_bytes, int64_t *ws_bytes) {
    StepArgs &a = w.args;
    uint64_t items;
    uint32_t n_split;
    count_items(w.h_rois, cfg, &items, &n_split, nullptr);
    if (g_cap_override) n_split = g_cap_override;
    if (items >= (1ull << 31)) return fail(ctx, NYX_ERR_UNSUPPORTED, "too many work items");
    uint32_t bucket_cap = (uint32_t)std::max<uint64_t>(items, 1u);
    const int K_out = cfg.merged ? 1 : K;
    uint64_t g_bytes = (uint64_t)n_split * K_out * (uint64_t)ng * ng * 8u;
    const uint64_t sums_bytes = (uint64_t)std::max<uint32_t>(w.n_rois, 1u) * K_out * sizeof(DirSums);
    const uint64_t sums_y_bytes =
        cfg.nonsym ? (uint64_t)std::max<uint32_t>(w.n_rois, 1u) * K_out * sizeof(DirSumsY) : 16u;
    const uint64_t mats0 = (uint64_t)std::max<uint32_t>(n_split, 1u) * K_out;
    uint64_t need = (uint64_t)kClasses * bucket_cap * 8u + g_bytes + sums_bytes + sums_y_bytes + n_split * 8u +
                    mats0 * (16u * ng + 32u + 8u * std::max(1u, ng / 8u));
    for (auto &b : w.tab) need += b.bytes;
    need += w.rois.bytes + w.counters.bytes;
    if (ws_bytes) *ws_bytes = (int64_t)need;
    if (cap_bytes > 0 && (int64_t)need > cap_bytes)
        return fail(ctx, NYX_ERR_OOM, "workspace needs %llu bytes, cap is %lld", (unsigned long long)need,
                    (long long)cap_bytes);
    HIPC(ctx, w.buckets.alloc((size_t)kClasses * bucket_cap * sizeof(uint2)));
    HIPC(ctx, w.G.alloc(std::max<uint64_t>(g_bytes, 16u)));
    HIPC(ctx, w.dsums.alloc(sums_bytes));
    HIPC(ctx, w.dsums_y.alloc(sums_y_bytes));
    HIPC(ctx, w.split_roi.alloc((size_t)std::max<uint32_t>(n_split, 1u) * 4u));
    HIPC(ctx, w.band_roi.alloc((size_t)std::max<uint32_t>(n_split, 1u) * 4u));
    // two-pass reduction of split matrices: enough row chunks to fill the chip
    const uint64_t mats = (uint64_t)std::max<uint32_t>(n_split, 1u) * K_out;
    const uint32_t chunks = (uint32_t)std::max<uint64_t>(
        1u, std::min<uint64_t>(std::max(1u, ng / 8u), (2u * (uint64_t)std::max(ctx->n_cu, 1) + mats - 1u) / mats));
    HIPC(ctx, w.smarg.alloc((size_t)mats * 4u * ng * 4u));
    HIPC(ctx, w.stot.alloc((size_t)mats * 4u * 8u));
    HIPC(ctx, w.splp.alloc((size_t)mats * chunks * 8u));
    a.buckets = w.buckets.as<uint2>();
    a.bucket_cap = bucket_cap;
    a.G = w.G.as<uint64_t>();
    a.g_cap = n_split;
    a.dsums = w.dsums.as<DirSums>();
    a.dsums_y = w.dsums_y.as<DirSumsY>();
    a.nonsym = cfg.nonsym;
    a.split_roi = w.split_roi.as<uint32_t>();
    a.band_roi = w.band_roi.as<uint32_t>();
    a.smarg = w.smarg.as<uint32_t>();
    a.stot = w.stot.as<uint64_t>();
    a.splp = w.splp.as<double>();
    a.split_chunks = chunks;
    a.band_vox = cfg.band_vox;
    a.band_w = cfg.band_w;
    a.band_tile = kBandTile;
    for (int k = 0; k < K; ++k) {
        a.off[k][0] = off[k].dz;
        a.off[k][1] = off[k].dy;
        a.off[k][2] = off[k].dx;
    }
    a.K = K;
    a.K_out = K_out;
    a.merged = cfg.merged;
    a.ng = (int32_t)ng;
    a.split_vox = cfg.split_vox;
    a.tile_vox = cfg.tile_vox;
    a.force_split = cfg.force_split;
    a.enqueue = 1;
    a.fp64 = fp64;
    // ordered counts take the gather accumulation (no sweep, no staged ring)
    if (cfg.nonsym) a.sweep_ok = 0;
    else set_sweep(a, w.h_imgs, off, K, cfg.kp);
    a.lds = make_layout(cfg, ng, K, !a.sweep_ok);
    return NYX_OK;
}

nyx_status set_outputs(nyx_ctx *ctx, StepArgs &a, nyx_roi_table *rois, void *table, uint32_t table_rows) {
    a.table = table;
    a.table_rows = table_rows;
    a.o_label = rois ? rois->label : nullptr;
    a.o_image = rois ? rois->image : nullptr;
    a.o_n = rois ? rois->n_vox : nullptr;
    a.o_min = rois ? rois->vmin : nullptr;
    a.o_max = rois ? rois->vmax : nullptr;
    a.o_bbox = rois ? rois->bbox : nullptr;
    (void)ctx;
    return NYX_OK;
}

// The full step on a stream.  per_roi: one accumulation launch per ROI.
nyx_status enqueue_step(nyx_plan *p, hipStream_t st, bool per_roi) {
    nyx_ctx *ctx = p->ctx;
    const StepArgs &a = p->w.args;
    HIPC(ctx, launch_reset(a, p->w.n_counters, st));
    HIPC(ctx, launch_scan(a, st));
    HIPC(ctx, launch_compact(a, 0u, 0xFFFFFFFFu, st));
    HIPC(ctx, launch_zero_split(a, st));
    if (!per_roi) {
        HIPC(ctx, launch_batch(a, p->grid, p->block, kNone, st));
    } else {
        for (uint32_t r = 0; r < p->w.n_rois; ++r) HIPC(ctx, launch_batch(a, p->roi_tiles[r], p->block, r, st));
    }
    HIPC(ctx, launch_band(a, (uint32_t)ctx->n_cu, st));
    HIPC(ctx, launch_split_finalize(a, st));
    HIPC(ctx, launch_features(a, a.dsums, a.dsums_y, a.roi_cap, a.counters + C_NROIS, st));
    return NYX_OK;
}

nyx_status check_counters(nyx_ctx *ctx, Work &w, hipStream_t st) {
    uint32_t h[8];
    HIPC(ctx, hipMemcpyAsync(h, w.counters.p, sizeof h, hipMemcpyDeviceToHost, st));
    HIPC(ctx, hipStreamSynchronize(st));
    uint32_t e = h[C_ERR];
    if (e & E_LABEL_RANGE) return fail(ctx, NYX_ERR_CAPACITY, "a label exceeds the planned label range");
    if (e & E_ROI_CAP) return fail(ctx, NYX_ERR_CAPACITY, "more ROIs than planned");
    if (e & E_SPLIT_CAP) return fail(ctx, NYX_ERR_CAPACITY, "more split ROIs than planned");
    if (e & E_ITEM_CAP) return fail(ctx, NYX_ERR_CAPACITY, "more work items than planned");
    if (e & E_TABLE_CAP) return fail(ctx, NYX_ERR_CAPACITY, "feature table too small");
    if (e & E_BIN_RANGE) return fail(ctx, NYX_ERR_INVALID, "bin image holds a value outside [1, n_bins]");
    if (e & E_COO_RANGE) return fail(ctx, NYX_ERR_INVALID, "COO entry outside its matrix");
    if (e & (E_LIST_CAP | E_HASH_FULL)) return fail(ctx, NYX_ERR_INTERNAL, "LDS capacity exceeded (error bits %u)", e);
    return NYX_OK;
}

std::string describe(const Config &c, const nyx_plan *p, uint64_t items, uint32_t n_split) {
    uint64_t band_voxels = 0;
    for (const RoiDesc &r : p->w.h_rois)
        if (c.band_vox && r.n > c.band_vox) band_voxels += r.n;
    char buf[640];
    snprintf(buf, sizeof buf,
             "mode=%s kp=%u copies=%u symmetric=%d block=%u grid=%u lds=%uB split_vox=%u tile_vox=%u tile_scale=%g "
             "list_cap=%u hash_cap=%u band_vox=%u band_w=%u band_voxels=%llu rois=%u items=%llu split_rois=%u ng=%d K=%d "
             "tuned_ms=%.4f",
             mode_name(c.mode), c.kp, p->w.args.lds.copies, c.nonsym ? 0 : 1, c.block, p->grid, p->w.args.lds.bytes, c.split_vox,
             c.tile_vox, (double)c.tile_scale, c.list_cap, c.hash_cap, c.band_vox, c.band_w,
             (unsigned long long)band_voxels, p->w.n_rois,
             (unsigned long long)items,
             n_split, p->ng, p->K, (double)p->tuned_ms);
    return buf;
}

// Applies a configuration to a plan: scratch, step arguments, grid.
nyx_status configure(nyx_plan *p, const Config &cfg, const nyx_extract_opts *opts) {
    nyx_ctx *ctx = p->ctx;
    nyx_status s = setup_step(ctx, p->w, cfg, opts->offsets_host, p->K, (uint32_t)p->ng, p->prec == NYX_FP64, 0,
                              opts->workspace_cap_bytes, &p->workspace_bytes);
    if (s != NYX_OK) return s;
    if (p->w.args.lds.bytes > kLdsBudget)
        return fail(ctx, NYX_ERR_UNSUPPORTED, "LDS layout of %u bytes exceeds the %u available", p->w.args.lds.bytes,
                    kLdsBudget);
    p->block = cfg.block;
    int occ = 0;
    HIPC(ctx, batch_occupancy(cfg.mode, p->prec == NYX_FP64, cfg.nonsym, cfg.block, p->w.args.lds.bytes, &occ));
    p->grid = (uint32_t)ctx->n_cu * (uint32_t)std::max(occ, 1);
    uint64_t items;
    uint32_t n_split;
    count_items(p->w.h_rois, cfg, &items, &n_split, &p->roi_tiles);
    p->cfg = nyx_plan::Cfg{cfg.mode, cfg.kp, cfg.block, cfg.split_vox, cfg.tile_vox, cfg.list_cap, cfg.hash_cap,
                           cfg.force_split};
    p->desc = describe(cfg, p, items, n_split);
    return NYX_OK;
}

}  // namespace

// ======================================================================= ABI
extern "C" {

const char *nyx_status_string(nyx_status s) {
    switch (s) {
        case NYX_OK: return "ok";
        case NYX_ERR_INVALID: return "invalid argument";
        case NYX_ERR_OOM: return "out of memory";
        case NYX_ERR_DEVICE: return "device error";
        case NYX_ERR_CAPACITY: return "capacity too small";
        case NYX_ERR_UNSUPPORTED: return "unsupported";
        case NYX_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

nyx_status nyx_create(nyx_ctx **out, int device_ordinal) {
    if (!out) return NYX_ERR_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return NYX_ERR_DEVICE;
    if (device_ordinal < 0 || device_ordinal >= n) return NYX_ERR_DEVICE;
    if (hipSetDevice(device_ordinal) != hipSuccess) return NYX_ERR_DEVICE;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device_ordinal) != hipSuccess) return NYX_ERR_DEVICE;
    uint8_t *scr = scratch_address(device_ordinal);
    if (!scr) return NYX_ERR_DEVICE;
    nyx_ctx *c = new nyx_ctx();
    c->device = device_ordinal;
    c->n_cu = prop.multiProcessorCount;
    c->scratch = scr;
    if (hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return NYX_ERR_DEVICE;
    }
    *out = c;
    return NYX_OK;
}

void nyx_destroy(nyx_ctx *ctx) {
    if (!ctx) return;
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
    delete ctx;
}

const char *nyx_last_error(const nyx_ctx *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

nyx_status nyx_offsets_default(int32_t dims, int32_t distance, nyx_offset *out_host, int32_t *n) {
    static const int32_t two[4][3] = {{0, 0, 1}, {0, -1, 1}, {0, -1, 0}, {0, -1, -1}};
    static const int32_t three[13][3] = {{0, 0, 1},  {0, 1, 0},  {1, 0, 0},   {0, 1, 1},  {0, 1, -1},
                                         {1, 0, 1},  {1, 0, -1}, {1, 1, 0},   {1, -1, 0}, {1, 1, 1},
                                         {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};
    if (!out_host || !n || distance < 1 || (dims != 2 && dims != 3)) return NYX_ERR_INVALID;
    int k = dims == 2 ? 4 : 13;
    for (int i = 0; i < k; ++i) {
        const int32_t *o = dims == 2 ? two[i] : three[i];
        out_host[i].dz = o[0] * distance;
        out_host[i].dy = o[1] * distance;
        out_host[i].dx = o[2] * distance;
    }
    *n = k;
    return NYX_OK;
}

int32_t nyx_feature_count(void) { return kNumFeat; }

const char *nyx_feature_name(int32_t f) { return (f >= 0 && f < kNumFeat) ? kFeatureNames[f] : nullptr; }

nyx_status nyx_bin_rois(nyx_ctx *ctx, const nyx_image *imgs, int32_t n_images, int32_t n_bins, nyx_roi_table *rois,
                        uint16_t *bins_out, nyx_stream stream) {
    if (!ctx) return NYX_ERR_INVALID;
    if (!rois) return fail(ctx, NYX_ERR_INVALID, "rois is NULL");
    nyx_status s = validate_images(ctx, imgs, n_images);
    if (s != NYX_OK) return s;
    if (n_bins < 2 || n_bins > 65535) return fail(ctx, NYX_ERR_INVALID, "n_bins must be in [2, 65535]");
    hipStream_t st = (hipStream_t)stream;
    HIPC(ctx, hipSetDevice(ctx->device));
    Work w;
    s = discover(ctx, imgs, n_images, w, st);
    if (s != NYX_OK) return s;
    if (rois->n_rois_host) *rois->n_rois_host = w.n_rois;
    if (rois->capacity < (int64_t)w.n_rois)
        return fail(ctx, NYX_ERR_CAPACITY, "ROI table capacity %lld < %u ROIs", (long long)rois->capacity, w.n_rois);
    StepArgs a = w.args;
    a.ng = n_bins;
    a.enqueue = 0;
    set_outputs(ctx, a, rois, nullptr, 0);
    HIPC(ctx, launch_reset(a, w.n_counters, st));
    HIPC(ctx, launch_scan(a, st));
    HIPC(ctx, launch_compact(a, 0u, 0u, st));
    if (bins_out) HIPC(ctx, launch_bin_image(a, bins_out, w.total_vox, w.vox_base.as<uint64_t>(), st));
    HIPC(ctx, hipStreamSynchronize(st));
    return NYX_OK;
}

nyx_status nyx_glcm_accumulate(nyx_ctx *ctx, const nyx_image *imgs, int32_t n_images, const nyx_roi_table *rois,
                               const uint16_t *bins, const nyx_offset *offsets, int32_t K, int32_t symmetric,
                               int32_t n_bins, nyx_glcm *out, nyx_stream stream) {
    if (!ctx) return NYX_ERR_INVALID;
    if (!out) return fail(ctx, NYX_ERR_INVALID, "out is NULL");
    nyx_status s = validate_images(ctx, imgs, n_images);
    if (s != NYX_OK) return s;
    if ((s = validate_offsets(ctx, imgs, n_images, offsets, K)) != NYX_OK) return s;
    if (n_bins < 2 || n_bins > 65535) return fail(ctx, NYX_ERR_INVALID, "n_bins must be in [2, 65535]");
    if ((s = validate_bins(ctx, n_bins)) != NYX_OK) return s;
    if (symmetric != 0 && symmetric != 1) return fail(ctx, NYX_ERR_INVALID, "symmetric must be 0 or 1");
    const bool nonsym = symmetric == 0;
    hipStream_t st = (hipStream_t)stream;
    HIPC(ctx, hipSetDevice(ctx->device));
    Work w;
    if ((s = discover(ctx, imgs, n_images, w, st)) != NYX_OK) return s;
    if (rois && rois->n_rois_host && *rois->n_rois_host != (int64_t)w.n_rois)
        return fail(ctx, NYX_ERR_INVALID, "ROI table has %lld rows, images have %u ROIs",
                    (long long)*rois->n_rois_host, w.n_rois);
    if (bins) {
        uint64_t off = 0;
        for (auto &d : w.h_imgs) { d.B = bins + off; off += d.nvox; }
        HIPC(ctx, hipMemcpyAsync(w.imgs.p, w.h_imgs.data(), sizeof(ImgDesc) * n_images, hipMemcpyHostToDevice, st));
    }
    if ((s = fetch_rois(ctx, w, st)) != NYX_OK) return s;
    const uint32_t ng = (uint32_t)n_bins;
    Config cfg;
    if ((s = choose_config(ctx, w, ng, K, 1, 256, cfg, nonsym)) != NYX_OK) return s;
    // ROIs in batches whose global matrices fit a fixed budget
    const uint64_t per_roi = (uint64_t)K * ng * ng * 8u;
    const uint64_t budget = 2ull << 30;
    uint32_t batch = (uint32_t)std::max<uint64_t>(1u, std::min<uint64_t>(w.n_rois ? w.n_rois : 1u, budget / per_roi));
    if ((s = setup_step(ctx, w, cfg, offsets, K, ng, 0, batch, 0, nullptr)) != NYX_OK) return s;
    StepArgs &a = w.args;
    set_outputs(ctx, a, nullptr, nullptr, 0);
    int occ = 0;
    {
        hipFuncAttributes fa;
        HIPC(ctx, get_batch_attributes(a.lds.mode, 0, a.nonsym, cfg.block, &fa));
        occ = 1;
    }
    const uint32_t grid = (uint32_t)ctx->n_cu * (uint32_t)std::max(occ, 1) * 2u;
    DevBuf dcount, doff;
    HIPC(ctx, dcount.alloc((size_t)batch * K * 8u));
    HIPC(ctx, doff.alloc((size_t)batch * K * 8u));
    std::vector<uint64_t> hcount((size_t)batch * K), hoff((size_t)batch * K);
    uint64_t nnz_total = 0;
    for (int phase = 0; phase < 2; ++phase) {
        uint64_t written = 0;
        for (uint32_t lo = 0; lo < w.n_rois; lo += batch) {
            uint32_t hi = std::min(w.n_rois, lo + batch);
            uint32_t ns = hi - lo;
            HIPC(ctx, launch_reset(a, w.n_counters, st));
            HIPC(ctx, launch_scan(a, st));
            HIPC(ctx, launch_compact(a, lo, hi, st));
            HIPC(ctx, launch_zero_split(a, st));
            HIPC(ctx, launch_batch(a, grid, cfg.block, kNone, st));
            HIPC(ctx, launch_band(a, (uint32_t)ctx->n_cu, st));
            HIPC(ctx, launch_coo_count(a, ns, dcount.as<uint64_t>(), st));
            HIPC(ctx, hipMemcpyAsync(hcount.data(), dcount.p, (size_t)ns * K * 8u, hipMemcpyDeviceToHost, st));
            HIPC(ctx, hipStreamSynchronize(st));
            if ((s = check_counters(ctx, w, st)) != NYX_OK) return s;
            uint64_t acc = written;
            for (size_t i = 0; i < (size_t)ns * K; ++i) { hoff[i] = acc; acc += hcount[i]; }
            if (phase == 1) {
                HIPC(ctx, hipMemcpyAsync(doff.p, hoff.data(), (size_t)ns * K * 8u, hipMemcpyHostToDevice, st));
                HIPC(ctx, launch_coo_emit(a, ns, doff.as<uint64_t>(), out->key, out->count, st));
                HIPC(ctx, hipStreamSynchronize(st));
            }
            written = acc;
        }
        if (phase == 0) {
            nnz_total = written;
            if (out->nnz_host) *out->nnz_host = (int64_t)nnz_total;
            out->n_bins = n_bins;
            out->n_offsets = K;
            out->symmetric = symmetric;
            out->n_rois = w.n_rois;
            if (out->capacity < (int64_t)nnz_total)
                return fail(ctx, NYX_ERR_CAPACITY, "COO capacity %lld < %llu nonzero cells", (long long)out->capacity,
                            (unsigned long long)nnz_total);
            if (nnz_total && (!out->key || !out->count)) return fail(ctx, NYX_ERR_INVALID, "COO arrays are NULL");
        }
    }
    return NYX_OK;
}

int32_t nyx_intensity_feature_count(void) { return kNumIntensityFeat; }

const char *nyx_intensity_feature_name(int32_t f) {
    return (f >= 0 && f < kNumIntensityFeat) ? kIntensityNames[f] : nullptr;
}

nyx_status nyx_intensity_features(nyx_ctx *ctx, const nyx_image *imgs, int32_t n_images, int32_t n_bins,
                                  nyx_precision prec, nyx_roi_table *rois, void *table, int64_t table_capacity_rows,
                                  nyx_stream stream) {
    if (!ctx) return NYX_ERR_INVALID;
    nyx_status s = validate_images(ctx, imgs, n_images);
    if (s != NYX_OK) return s;
    if (n_bins < 2 || n_bins > 65535) return fail(ctx, NYX_ERR_INVALID, "n_bins must be in [2, 65535]");
    if ((s = validate_bins(ctx, n_bins)) != NYX_OK) return s;
    if (prec != NYX_FP32 && prec != NYX_FP64) return fail(ctx, NYX_ERR_INVALID, "bad precision");
    hipStream_t st = (hipStream_t)stream;
    HIPC(ctx, hipSetDevice(ctx->device));
    Work w;
    if ((s = discover(ctx, imgs, n_images, w, st)) != NYX_OK) return s;
    const int64_t n = w.n_rois;
    if (rois && rois->n_rois_host) *rois->n_rois_host = n;
    if (rois && rois->capacity < n)
        return fail(ctx, NYX_ERR_CAPACITY, "ROI table capacity %lld < %lld ROIs", (long long)rois->capacity, (long long)n);
    if (table_capacity_rows < n)
        return fail(ctx, NYX_ERR_CAPACITY, "table capacity %lld < %lld rows", (long long)table_capacity_rows, (long long)n);
    if (n > 0 && !table) return fail(ctx, NYX_ERR_INVALID, "table is NULL");
    StepArgs a = w.args;
    a.ng = n_bins;
    a.enqueue = 0;
    set_outputs(ctx, a, rois, nullptr, 0);
    HIPC(ctx, launch_reset(a, w.n_counters, st));
    HIPC(ctx, launch_scan(a, st));
    HIPC(ctx, launch_compact(a, 0u, 0u, st));
    HIPC(ctx, launch_intensity(a, (uint32_t)n, prec == NYX_FP64, table,
                               (uint32_t)std::min<int64_t>(table_capacity_rows, 0xFFFFFFFFll), st));
    return check_counters(ctx, w, st);
}

int32_t nyx_neighbourhood_feature_count(void) { return kNumNeighbourFeat; }

const char *nyx_neighbourhood_feature_name(int32_t f) {
    return (f >= 0 && f < kNumNeighbourFeat) ? kNeighbourNames[f] : nullptr;
}

nyx_status nyx_neighbourhood_features(nyx_ctx *ctx, const nyx_image *imgs, int32_t n_images, int32_t n_bins,
                                      int32_t alpha, nyx_precision prec, nyx_roi_table *rois, void *table,
                                      int64_t table_capacity_rows, nyx_stream stream) {
    if (!ctx) return NYX_ERR_INVALID;
    nyx_status s = validate_images(ctx, imgs, n_images);
    if (s != NYX_OK) return s;
    if (n_bins < 2 || n_bins > 65535) return fail(ctx, NYX_ERR_INVALID, "n_bins must be in [2, 65535]");
    if (alpha < 0) return fail(ctx, NYX_ERR_INVALID, "alpha must be >= 0");
    if (prec != NYX_FP32 && prec != NYX_FP64) return fail(ctx, NYX_ERR_INVALID, "bad precision");
    int any_volume = 0;
    for (int i = 0; i < n_images; ++i) any_volume |= imgs[i].nz > 1;
    if (neighbourhood_lds_bytes((uint32_t)n_bins, any_volume) > kLdsBudget - 1024u)
        return fail(ctx, NYX_ERR_UNSUPPORTED, "n_bins=%d: the per-ROI %s neighbourhood tables exceed LDS", n_bins,
                    any_volume ? "3D" : "2D");
    hipStream_t st = (hipStream_t)stream;
    HIPC(ctx, hipSetDevice(ctx->device));
    Work w;
    if ((s = discover(ctx, imgs, n_images, w, st)) != NYX_OK) return s;
    const int64_t n = w.n_rois;
    if (rois && rois->n_rois_host) *rois->n_rois_host = n;
    if (rois && rois->capacity < n)
        return fail(ctx, NYX_ERR_CAPACITY, "ROI table capacity %lld < %lld ROIs", (long long)rois->capacity, (long long)n);
    if (table_capacity_rows < n)
        return fail(ctx, NYX_ERR_CAPACITY, "table capacity %lld < %lld rows", (long long)table_capacity_rows, (long long)n);
    if (n > 0 && !table) return fail(ctx, NYX_ERR_INVALID, "table is NULL");
    StepArgs a = w.args;
    a.ng = n_bins;
    a.enqueue = 0;
    set_outputs(ctx, a, rois, nullptr, 0);
    HIPC(ctx, launch_reset(a, w.n_counters, st));
    HIPC(ctx, launch_scan(a, st));
    HIPC(ctx, launch_compact(a, 0u, 0u, st));
    HIPC(ctx, launch_neighbourhood(a, (uint32_t)n, prec == NYX_FP64, (uint32_t)alpha, any_volume, table,
                                   (uint32_t)std::min<int64_t>(table_capacity_rows, 0xFFFFFFFFll), st));
    return check_counters(ctx, w, st);
}

nyx_status nyx_glcm_features(nyx_ctx *ctx, const nyx_glcm *glcm, const nyx_roi_table *rois, nyx_precision prec,
                             void *table, int64_t table_capacity_rows, nyx_stream stream) {
    if (!ctx) return NYX_ERR_INVALID;
    if (!glcm || !table) return fail(ctx, NYX_ERR_INVALID, "NULL argument");
    if (rois && rois->n_rois_host && *rois->n_rois_host != glcm->n_rois)
        return fail(ctx, NYX_ERR_INVALID, "ROI table has %lld rows, the COO list %lld ROIs",
                    (long long)*rois->n_rois_host, (long long)glcm->n_rois);
    if (glcm->n_offsets < 1 || glcm->n_offsets > kMaxOffsets) return fail(ctx, NYX_ERR_INVALID, "bad n_offsets");
    nyx_status s = validate_bins(ctx, glcm->n_bins);
    if (s != NYX_OK) return s;
    if (glcm->n_rois < 0 || glcm->n_rois >= (1ll << 26)) return fail(ctx, NYX_ERR_INVALID, "bad n_rois");
    if (table_capacity_rows < glcm->n_rois)
        return fail(ctx, NYX_ERR_CAPACITY, "table capacity %lld < %lld rows", (long long)table_capacity_rows,
                    (long long)glcm->n_rois);
    uint64_t nnz = glcm->nnz_host ? (uint64_t)*glcm->nnz_host : 0u;
    if (nnz && (!glcm->key || !glcm->count)) return fail(ctx, NYX_ERR_INVALID, "COO arrays are NULL");
    if (prec != NYX_FP32 && prec != NYX_FP64) return fail(ctx, NYX_ERR_INVALID, "bad precision");
    if (glcm->symmetric != 0 && glcm->symmetric != 1) return fail(ctx, NYX_ERR_INVALID, "symmetric must be 0 or 1");
    hipStream_t st = (hipStream_t)stream;
    HIPC(ctx, hipSetDevice(ctx->device));
    const uint32_t n_rois = (uint32_t)glcm->n_rois;
    const int K = glcm->n_offsets;
    if (n_rois == 0) return NYX_OK;
    DevBuf seg, scratch, scratch_y, counters;
    HIPC(ctx, seg.alloc(((size_t)n_rois * K + 1) * 8u));
    HIPC(ctx, scratch.alloc((size_t)n_rois * K * sizeof(DirSums)));
    HIPC(ctx, scratch_y.alloc((size_t)n_rois * K * sizeof(DirSumsY)));
    HIPC(ctx, counters.alloc(256));
    HIPC(ctx, hipMemsetAsync(counters.p, 0, 256, st));
    StepArgs a;
    memset(&a, 0, sizeof a);
    a.K = K;
    a.K_out = K;
    a.ng = glcm->n_bins;
    a.fp64 = prec == NYX_FP64;
    a.table = table;
    a.table_rows = (uint32_t)std::min<int64_t>(table_capacity_rows, 0xFFFFFFFFll);
    a.counters = counters.as<uint32_t>();
    a.nonsym = glcm->symmetric == 0;
    HIPC(ctx, launch_coo_features(a, glcm->key, glcm->count, nnz, n_rois, seg.as<uint64_t>(), scratch.as<DirSums>(),
                                  scratch_y.as<DirSumsY>(), st));
    uint32_t herr = 0;
    HIPC(ctx, hipMemcpyAsync(&herr, counters.as<uint32_t>() + C_ERR, 4, hipMemcpyDeviceToHost, st));
    HIPC(ctx, hipStreamSynchronize(st));
    if (herr & E_COO_RANGE) return fail(ctx, NYX_ERR_INVALID, "COO entry outside its matrix");
    if (herr & E_TABLE_CAP) return fail(ctx, NYX_ERR_CAPACITY, "feature table too small");
    return NYX_OK;
}

}  // extern "C"

namespace {

// Validation, ROI discovery and the untimed default configuration of a plan
// (shared by nyx_plan_create and the no-allocation entry point).
nyx_status plan_init(nyx_ctx *ctx, const nyx_image *imgs, int32_t n_images, const nyx_extract_opts *opts,
                     nyx_plan *p, hipStream_t st, std::vector<Config> &cands, Config &cfg) {
    nyx_status s = validate_images(ctx, imgs, n_images);
    if (s != NYX_OK) return s;
    if ((s = validate_offsets(ctx, imgs, n_images, opts->offsets_host, opts->n_offsets)) != NYX_OK) return s;
    if (opts->n_bins < 2 || opts->n_bins > 65535) return fail(ctx, NYX_ERR_INVALID, "n_bins must be in [2, 65535]");
    if ((s = validate_bins(ctx, opts->n_bins)) != NYX_OK) return s;
    if (opts->symmetric != 0 && opts->symmetric != 1) return fail(ctx, NYX_ERR_INVALID, "symmetric must be 0 or 1");
    if (opts->precision != NYX_FP32 && opts->precision != NYX_FP64) return fail(ctx, NYX_ERR_INVALID, "bad precision");
    if (opts->aggregate != NYX_AGG_PER_OFFSET && opts->aggregate != NYX_AGG_MERGED)
        return fail(ctx, NYX_ERR_INVALID, "aggregate must be NYX_AGG_PER_OFFSET or NYX_AGG_MERGED");
    if (opts->copies != 0 && opts->copies != 1 && opts->copies != 2 && opts->copies != 4)
        return fail(ctx, NYX_ERR_INVALID, "copies must be 0, 1, 2 or 4");
    HIPC(ctx, hipSetDevice(ctx->device));
    p->ctx = ctx;
    p->imgs.assign(imgs, imgs + n_images);
    p->K = opts->n_offsets;
    p->ng = opts->n_bins;
    p->prec = opts->precision;
    if ((s = discover(ctx, imgs, n_images, p->w, st)) != NYX_OK) return s;
    if ((s = fetch_rois(ctx, p->w, st)) != NYX_OK) return s;
    const bool merged = opts->aggregate == NYX_AGG_MERGED;
    // the default plan: one copy (or the forced count) at the load-balance tile size
    const uint32_t copies0 = opts->copies > 0 ? (uint32_t)opts->copies : 1u;
    const bool nonsym = opts->symmetric == 0;
    cands = candidate_configs(ctx, p->w, (uint32_t)p->ng, p->K, 0, 256, merged, copies0, 1.f, nonsym);
    if (cands.empty())
        return fail(ctx, NYX_ERR_UNSUPPORTED, "no LDS configuration fits n_bins=%d with %d offsets%s%s", p->ng, p->K,
                    merged ? " merged in one pass" : "", copies0 > 1u ? " with privatised copies" : "");
    cfg = default_config(cands, p->w, (uint32_t)p->ng, p->K);
    if (opts->accum_mode >= 0) {
        bool found = false;
        for (const Config &c : cands)
            if (c.mode == opts->accum_mode) { cfg = c; found = true; break; }
        if (!found) return fail(ctx, NYX_ERR_UNSUPPORTED, "accumulation mode %d does not fit this workload", opts->accum_mode);
    }
    cfg = widen_block(cfg, (uint32_t)p->ng, p->K);
    return NYX_OK;
}

}  // namespace

extern "C" {

nyx_status nyx_plan_create(nyx_ctx *ctx, const nyx_image *imgs, int32_t n_images, const nyx_extract_opts *opts,
                           nyx_plan **out, int64_t *n_rois_host) {
    if (!ctx) return NYX_ERR_INVALID;
    if (!out || !opts) return fail(ctx, NYX_ERR_INVALID, "NULL argument");
    *out = nullptr;
    hipStream_t st = ctx->capture_stream;
    std::unique_ptr<nyx_plan> p(new nyx_plan());
    std::vector<Config> cands;
    Config cfg;
    nyx_status s = plan_init(ctx, imgs, n_images, opts, p.get(), st, cands, cfg);
    if (s != NYX_OK) return s;
    const bool merged = opts->aggregate == NYX_AGG_MERGED;
    const uint32_t copies0 = opts->copies > 0 ? (uint32_t)opts->copies : 1u;
    if (opts->autotune) {
        // further axes: privatised copies (when not forced) and the tile size of split ROIs
        for (uint32_t cp : {1u, 2u, 4u}) {
            if (opts->copies > 0 && cp != copies0) continue;
            for (float ts : {0.5f, 1.f, 2.f}) {
                if (cp == copies0 && ts == 1.f) continue;
                for (const Config &c :
                     candidate_configs(ctx, p->w, (uint32_t)p->ng, p->K, 0, 256, merged, cp, ts, opts->symmetric == 0))
                    if (cp == 1u || c.copies == cp) cands.push_back(c);
            }
        }
        // and the work-group size: 512 threads where 256 leave one group per CU
        const size_t n256 = cands.size();
        for (size_t i = 0; i < n256; ++i) {
            const Config c = widen_block(cands[i], (uint32_t)p->ng, p->K);
            if (c.block != cands[i].block) cands.push_back(c);
        }
    }
    if (opts->autotune && cands.size() > 1) {
        // every candidate: one warm-up step, then the median of kTuneSteps timed steps
        constexpr int kTuneSteps = 5;
        DevBuf tmp;
        size_t row_bytes = (size_t)(merged ? 1 : p->K + 1) * kNumFeat * (p->prec == NYX_FP64 ? 8u : 4u);
        HIPC(ctx, tmp.alloc(std::max<size_t>(p->w.n_rois, 1u) * row_bytes));
        hipEvent_t ev[kTuneSteps + 1];
        for (auto &e : ev) HIPC(ctx, hipEventCreate(&e));
        float best = 1e30f;
        for (const Config &c : cands) {
            if (opts->accum_mode >= 0 && c.mode != opts->accum_mode) continue;
            if ((s = configure(p.get(), c, opts)) != NYX_OK) continue;
            set_outputs(ctx, p->w.args, nullptr, tmp.p, p->w.n_rois);
            if ((s = enqueue_step(p.get(), st, false)) != NYX_OK) break;
            hipError_t he = hipEventRecord(ev[0], st);
            for (int k = 0; k < kTuneSteps && he == hipSuccess && s == NYX_OK; ++k) {
                s = enqueue_step(p.get(), st, false);
                he = hipEventRecord(ev[k + 1], st);
            }
            if (s != NYX_OK) break;
            HIPC(ctx, he);
            HIPC(ctx, hipEventSynchronize(ev[kTuneSteps]));
            float t[kTuneSteps];
            for (int k = 0; k < kTuneSteps; ++k) HIPC(ctx, hipEventElapsedTime(&t[k], ev[k], ev[k + 1]));
            std::sort(t, t + kTuneSteps);
            const float ms = t[kTuneSteps / 2];
            if (log_level() > 0)
                fprintf(stderr, "[nyx] autotune %s kp=%u copies=%u tile_scale=%g block=%u: %.3f ms\n", mode_name(c.mode),
                        c.kp, c.copies, (double)c.tile_scale, c.block, ms);
            if (ms < best) { best = ms; cfg = c; }
        }
        for (auto &e : ev) (void)hipEventDestroy(e);
        if (s != NYX_OK) return s;
        p->tuned_ms = best;
    }
    if ((s = configure(p.get(), cfg, opts)) != NYX_OK) return s;
    if (log_level() > 0) fprintf(stderr, "[nyx] plan: %s\n", p->desc.c_str());
    if (n_rois_host) *n_rois_host = p->w.n_rois;
    *out = p.release();
    return NYX_OK;
}

nyx_status nyx_plan_execute(nyx_plan *p, nyx_roi_table *rois, void *table, nyx_stream stream) {
    if (!p) return NYX_ERR_INVALID;
    nyx_ctx *ctx = p->ctx;
    if (!table) return fail(ctx, NYX_ERR_INVALID, "table is NULL");
    if (rois && rois->capacity < (int64_t)p->w.n_rois)
        return fail(ctx, NYX_ERR_CAPACITY, "ROI table capacity too small");
    HIPC(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    nyx_roi_table key{};
    if (rois) key = *rois;
    key.n_rois_host = nullptr;
    bool same = p->exec && p->graph_table == table && memcmp(&key, &p->graph_rois, sizeof key) == 0;
    if (!same) {
        if (p->exec) { (void)hipGraphExecDestroy(p->exec); p->exec = nullptr; }
        if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
        set_outputs(ctx, p->w.args, rois, table, p->w.n_rois);
        hipStream_t cs = ctx->capture_stream;
        HIPC(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        nyx_status s = enqueue_step(p, cs, false);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(cs, &g);
        if (s != NYX_OK) { if (g) (void)hipGraphDestroy(g); return s; }
        if (e != hipSuccess) return fail(ctx, NYX_ERR_DEVICE, "graph capture: %s", hipGetErrorString(e));
        p->graph = g;
        HIPC(ctx, hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0));
        p->graph_table = table;
        p->graph_rois = key;
    }
    HIPC(ctx, hipGraphLaunch(p->exec, st));
    if (rois && rois->n_rois_host) *rois->n_rois_host = p->w.n_rois;
    return NYX_OK;
}

nyx_status nyx_plan_execute_per_roi(nyx_plan *p, nyx_roi_table *rois, void *table, nyx_stream stream) {
    if (!p) return NYX_ERR_INVALID;
    nyx_ctx *ctx = p->ctx;
    if (!table) return fail(ctx, NYX_ERR_INVALID, "table is NULL");
    if (rois && rois->capacity < (int64_t)p->w.n_rois)
        return fail(ctx, NYX_ERR_CAPACITY, "ROI table capacity too small");
    HIPC(ctx, hipSetDevice(ctx->device));
    set_outputs(ctx, p->w.args, rois, table, p->w.n_rois);
    nyx_status s = enqueue_step(p, (hipStream_t)stream, true);
    if (rois && rois->n_rois_host) *rois->n_rois_host = p->w.n_rois;
    return s;
}

nyx_status nyx_plan_profile(nyx_plan *p, void *table, float *ms_host, nyx_stream stream) {
    if (!p) return NYX_ERR_INVALID;
    nyx_ctx *ctx = p->ctx;
    if (!table || !ms_host) return fail(ctx, NYX_ERR_INVALID, "NULL argument");
    HIPC(ctx, hipSetDevice(ctx->device));
    hipStream_t st = (hipStream_t)stream;
    set_outputs(ctx, p->w.args, nullptr, table, p->w.n_rois);
    // the graph (if any) was captured with other outputs; drop it
    if (p->exec) { (void)hipGraphExecDestroy(p->exec); p->exec = nullptr; }
    if (p->graph) { (void)hipGraphDestroy(p->graph); p->graph = nullptr; }
    p->graph_table = nullptr;
    static_assert(NYX_PHASE_COUNT == 8, "one event interval per phase");
    hipEvent_t ev[NYX_PHASE_COUNT + 1];
    for (auto &e : ev) HIPC(ctx, hipEventCreate(&e));
    const StepArgs &a = p->w.args;
    nyx_status s = NYX_OK;
    hipError_t he = hipSuccess;
    he = hipEventRecord(ev[0], st);
    if (he == hipSuccess) he = launch_reset(a, p->w.n_counters, st);
    if (he == hipSuccess) he = hipEventRecord(ev[1], st);
    if (he == hipSuccess) he = launch_scan(a, st);
    if (he == hipSuccess) he = hipEventRecord(ev[2], st);
    if (he == hipSuccess) he = launch_compact(a, 0u, 0xFFFFFFFFu, st);
    if (he == hipSuccess) he = hipEventRecord(ev[3], st);
    if (he == hipSuccess) he = launch_zero_split(a, st);
    if (he == hipSuccess) he = hipEventRecord(ev[4], st);
    if (he == hipSuccess) he = launch_batch(a, p->grid, p->block, kNone, st);
    if (he == hipSuccess) he = hipEventRecord(ev[5], st);
    if (he == hipSuccess) he = launch_band(a, (uint32_t)ctx->n_cu, st);
    if (he == hipSuccess) he = hipEventRecord(ev[6], st);
    if (he == hipSuccess) he = launch_split_finalize(a, st);
    if (he == hipSuccess) he = hipEventRecord(ev[7], st);
    if (he == hipSuccess) he = launch_features(a, a.dsums, a.dsums_y, a.roi_cap, a.counters + C_NROIS, st);
    if (he == hipSuccess) he = hipEventRecord(ev[8], st);
    if (he == hipSuccess) he = hipEventSynchronize(ev[8]);
    if (he == hipSuccess)
        for (int i = 0; i < NYX_PHASE_COUNT; ++i) {
            he = hipEventElapsedTime(&ms_host[i], ev[i], ev[i + 1]);
            if (he != hipSuccess) break;
        }
    for (auto &e : ev) (void)hipEventDestroy(e);
    if (he != hipSuccess) s = fail(ctx, NYX_ERR_DEVICE, "profile: %s", hipGetErrorString(he));
    return s;
}

nyx_status nyx_plan_check(nyx_plan *p, nyx_stream stream) {
    if (!p) return NYX_ERR_INVALID;
    return check_counters(p->ctx, p->w, (hipStream_t)stream);
}

const char *nyx_plan_describe(const nyx_plan *p) { return p ? p->desc.c_str() : ""; }

void nyx_plan_destroy(nyx_plan *p) {
    if (!p) return;
    (void)hipSetDevice(p->ctx->device);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    delete p;
}

nyx_status nyx_extract_batch(nyx_ctx *ctx, const nyx_image *imgs, int32_t n_images, const nyx_extract_opts *opts,
                             nyx_roi_table *rois, void *table, int64_t table_capacity_rows, nyx_stream stream) {
    if (!ctx) return NYX_ERR_INVALID;
    nyx_plan *p = nullptr;
    int64_t n = 0;
    nyx_status s = nyx_plan_create(ctx, imgs, n_images, opts, &p, &n);
    if (s != NYX_OK) return s;
    if (rois && rois->n_rois_host) *rois->n_rois_host = n;
    if (table_capacity_rows < n) {
        nyx_plan_destroy(p);
        return fail(ctx, NYX_ERR_CAPACITY, "table capacity %lld < %lld rows", (long long)table_capacity_rows, (long long)n);
    }
    if (rois && rois->capacity < n) {
        nyx_plan_destroy(p);
        return fail(ctx, NYX_ERR_CAPACITY, "ROI table capacity %lld < %lld", (long long)rois->capacity, (long long)n);
    }
    set_outputs(ctx, p->w.args, rois, table, (uint32_t)n);
    s = enqueue_step(p, (hipStream_t)stream, false);
    if (s == NYX_OK) s = check_counters(ctx, p->w, (hipStream_t)stream);
    else (void)hipStreamSynchronize((hipStream_t)stream);
    nyx_plan_destroy(p);
    return s;
}

nyx_status nyx_extract_batch_noalloc(nyx_ctx *ctx, const nyx_image *imgs, int32_t n_images,
                                     const nyx_extract_opts *opts, nyx_roi_table *rois, void *table,
                                     int64_t table_capacity_rows, nyx_stream stream) {
    if (!ctx) return NYX_ERR_INVALID;
    if (!opts) return fail(ctx, NYX_ERR_INVALID, "NULL argument");
    if (!ctx->scratch) return fail(ctx, NYX_ERR_DEVICE, "no scratch address for device %d", ctx->device);
    hipStream_t st = (hipStream_t)stream;
    // every device buffer of the step is carved from this device's scratch
    Arena ar;
    ar.base = ctx->scratch;
    ar.cap = kScratchBytes;
    nyx_plan p;
    p.w.use_arena(&ar);
    std::vector<Config> cands;
    Config cfg;
    nyx_status s = plan_init(ctx, imgs, n_images, opts, &p, st, cands, cfg);
    if (s == NYX_OK) s = configure(&p, cfg, opts);
    if (s != NYX_OK) {
        if (ar.wanted > ar.cap)
            return fail(ctx, NYX_ERR_CAPACITY,
                        "batch needs more than the %zu bytes of no-allocation scratch (at least %zu)", ar.cap,
                        ar.wanted);
        return s;
    }
    const int64_t n = p.w.n_rois;
    if (rois && rois->n_rois_host) *rois->n_rois_host = n;
    if (table_capacity_rows < n)
        return fail(ctx, NYX_ERR_CAPACITY, "table capacity %lld < %lld rows", (long long)table_capacity_rows, (long long)n);
    if (rois && rois->capacity < n)
        return fail(ctx, NYX_ERR_CAPACITY, "ROI table capacity %lld < %lld", (long long)rois->capacity, (long long)n);
    if (n > 0 && !table) return fail(ctx, NYX_ERR_INVALID, "table is NULL");
    set_outputs(ctx, p.w.args, rois, table, (uint32_t)n);
    s = enqueue_step(&p, st, false);
    if (s == NYX_OK) s = check_counters(ctx, p.w, st);
    else (void)hipStreamSynchronize(st);
    return s;
}

}  // extern "C"
