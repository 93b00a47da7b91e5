/*
 * nyx.h -- C ABI of the MI355X per-ROI GLCM texture library (libnyx.so).
 *
 * The problem follows the paper's statement of regional feature extraction:
 * an intensity image and a label mask go in, one row of measurements per
 * unique nonzero label comes out (Supplementary Table S7, "ROI/FOV"; Main
 * section, regional features).  The measurements are the grey-level
 * co-occurrence (GLCM) features of Supplementary Table S3 (rows 140-174 with
 * the NY mark; AVEAMP is not defined by the paper and is left out), in 2D
 * and in 3D (Table S5, row 361), with the two hyper-parameters the paper
 * names for texture cost O(m, g, s): the number of grey levels g and the
 * spatial offset s (Materials and methods, "Feature Control and Tunability").
 *
 * Conventions shared by every call
 *  - Images are [nz][ny][nx], x fastest; 2D images have nz = 1.  Label 0 is
 *    background; all voxels with the same nonzero label form one ROI,
 *    connected or not.
 *  - Grey levels: fixed bin number over the ROI's own [min, max]:
 *    level = 1 + floor(n_bins (I - min) / (max - min)), clamped to n_bins;
 *    a constant ROI is level 1.  Computed exactly in integers.
 *  - A voxel pair (v, v + d) is counted only when both voxels are inside the
 *    image and carry the ROI's label.  C(i, j) counts the pairs with level i
 *    at v and j at v + d.  Matrices are symmetric, P = C + C^T, unless a call
 *    asks for the ordered counts P = C (symmetric = 0): the texture
 *    hyper-parameters the paper names leave the symmetry open (Methods,
 *    "Feature Control and Tunability"), and the 30 features are defined for
 *    either (row and column marginals then differ; a matrix whose row or
 *    column marginal has one occupied level gives CORR = 1 and
 *    INFOMEAS1 = INFOMEAS2 = 0).
 *  - ROIs are ordered by (image index, label), ascending.  Output rows follow
 *    that order.
 *  - Feature table: row r holds (n_offsets + 1) blocks of 30 values; block
 *    k < n_offsets is direction k, the last block is the mean over the
 *    directions that have at least one pair (NYX_AGG_MERGED: one block, the
 *    features of the summed matrix).  Element type float (NYX_FP32)
 *    or double (NYX_FP64).  Undefined values (a direction with no pair) are
 *    quiet NaN.  Column order: nyx_feature_name(0..29).
 *  - Pointers are DEVICE pointers (HIP device memory, e.g. torch CUDA
 *    tensors) unless the name ends in _host.  The caller owns all input and
 *    output buffers; the library owns only scratch memory inside a context
 *    or plan.
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = null stream).  Calls
 *    that must report a size to the host (nyx_bin_rois, nyx_glcm_accumulate,
 *    nyx_plan_create) synchronise that stream once.
 *  - Errors: a nyx_status is returned; on failure nyx_last_error(ctx) gives a
 *    message (valid until the next call on that ctx).  Arguments are
 *    validated before any device work: NYX_ERR_INVALID for n_bins outside
 *    [2, 65535], n_offsets outside [1, 64], an offset (0,0,0), a non-positive
 *    or too large dimension, dz != 0 on a 2D image, a NULL required pointer.
 *    A too small output capacity gives NYX_ERR_CAPACITY with the required
 *    size written to the *_host count (call once with capacity 0 to query).
 *  - A context is used by one host thread at a time.
 */
#ifndef NYX_H
#define NYX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum nyx_status {
    NYX_OK = 0,
    NYX_ERR_INVALID = 1,
    NYX_ERR_OOM = 2,
    NYX_ERR_DEVICE = 3,
    NYX_ERR_CAPACITY = 4,
    NYX_ERR_UNSUPPORTED = 5,
    NYX_ERR_INTERNAL = 6
} nyx_status;

typedef enum nyx_precision { NYX_FP32 = 0, NYX_FP64 = 1 } nyx_precision;

typedef struct nyx_ctx nyx_ctx;
typedef struct nyx_plan nyx_plan;
typedef void *nyx_stream; /* hipStream_t */

/* One neighbour offset (dz, dy, dx); y grows downward. */
typedef struct nyx_offset { int32_t dz, dy, dx; } nyx_offset;

/* One image: device arrays of nz*ny*nx elements (each dimension <= 65535 and
 * nz*ny*nx < 2^31). */
typedef struct nyx_image {
    const uint16_t *intensity;
    const uint32_t *labels;
    int64_t nz, ny, nx;
} nyx_image;

/* Per-ROI statistics (device arrays of `capacity` entries; any array may be
 * NULL when not wanted).  bbox holds 6 int32 per ROI: x_min, y_min, z_min,
 * x_max, y_max, z_max (inclusive). */
typedef struct nyx_roi_table {
    uint32_t *label;
    uint32_t *image;
    uint64_t *n_vox;
    uint16_t *vmin;
    uint16_t *vmax;
    int32_t *bbox;
    int64_t capacity;
    int64_t *n_rois_host; /* out: number of ROIs found */
} nyx_roi_table;

/* Sparse co-occurrence counts as a COO list sorted by key, key = roi << 38 |
 * dir << 32 | (i - 1) << 16 | (j - 1) with 1-based levels; count is exact
 * (64-bit).  Symmetric matrices: the upper triangle U(i, j), i <= j,
 * U(i, j) = P(i, j) for i < j and U(i, i) = P(i, i) / 2.  Ordered counts
 * (symmetric = 0): every nonzero cell C(i, j). */
typedef struct nyx_glcm {
    uint64_t *key;
    uint64_t *count;
    int64_t capacity;
    int64_t *nnz_host;  /* out: number of nonzero cells */
    int32_t n_bins;     /* set by nyx_glcm_accumulate */
    int32_t n_offsets;  /* set by nyx_glcm_accumulate */
    int32_t symmetric;  /* set by nyx_glcm_accumulate: 1 triangle of P = C + C^T, 0 ordered counts C */
    int64_t n_rois;     /* set by nyx_glcm_accumulate */
} nyx_glcm;

/* How the offsets' matrices become features.  The offset set is one of the
 * texture hyper-parameters (Methods, "Feature Control and Tunability"); how
 * the per-offset matrices are combined is not fixed there, so both usual
 * choices are offered:
 *   NYX_AGG_PER_OFFSET  features of each offset's matrix and their mean
 *                       (table rows of n_offsets + 1 blocks);
 *   NYX_AGG_MERGED      features of P = sum over the offsets of P_k, one
 *                       matrix per ROI (table rows of 1 block): every offset
 *                       counts into one LDS triangle, so it needs that
 *                       triangle in LDS and a dense scan accumulation mode;
 *                       NYX_ERR_UNSUPPORTED otherwise (e.g. 1024 levels). */
typedef enum nyx_aggregate { NYX_AGG_PER_OFFSET = 0, NYX_AGG_MERGED = 1 } nyx_aggregate;

typedef struct nyx_extract_opts {
    int32_t n_bins;
    const nyx_offset *offsets_host;
    int32_t n_offsets;
    int32_t symmetric;           /* 1: P = C + C^T; 0: ordered counts P = C (dense square per
                                    direction in LDS, or the hash table; gather accumulation) */
    nyx_precision precision;     /* feature output type */
    int32_t autotune;            /* 1: time candidate kernel configurations at plan time */
    int32_t accum_mode;          /* -1 = automatic; else force one accumulation mode:
                                    0 LDS triangle + nonzero list built by returning atomics,
                                    1 LDS hash table, 2 LDS triangle + ordered scan,
                                    3 LDS triangle of 16-bit counters + ordered scan
                                    (NYX_ERR_UNSUPPORTED when it does not fit) */
    int32_t copies;              /* privatised copies of each LDS triangle (dense scan modes):
                                    0 = automatic (1, or the fastest of 1, 2 and 4 when autotune
                                    is set); 1, 2 or 4 = forced.  Lane l of a wavefront counts
                                    into copy l mod copies, so neighbouring lanes that hit the
                                    same cell add to different words; the copies are summed when
                                    the triangle is read.  NYX_ERR_UNSUPPORTED when the copies do
                                    not fit LDS */
    int64_t workspace_cap_bytes; /* 0 = no cap; exceeding it gives NYX_ERR_OOM */
    int32_t aggregate;           /* NYX_AGG_PER_OFFSET or NYX_AGG_MERGED (table layout above) */
} nyx_extract_opts;

/* Context on one device (hipSetDevice ordinal).  NYX_ERR_DEVICE if absent.
 * Owns the library's scratch for the one-shot calls; not thread-safe. */
nyx_status nyx_create(nyx_ctx **out, int device_ordinal);
void nyx_destroy(nyx_ctx *ctx);
const char *nyx_last_error(const nyx_ctx *ctx);
const char *nyx_status_string(nyx_status s);

/* The offset / scan-angle hyper-parameter of texture (Methods, "Feature
 * Control and Tunability"; Fig. 7 offsets).
 * Default offsets at a distance: dims 2 -> 0, 45, 90, 135 degrees
 * ((0,0,1), (0,-1,1), (0,-1,0), (0,-1,-1)); dims 3 -> the 13 directions
 * that represent the 26-neighbourhood up to sign.  out_host needs room for
 * 13 entries; *n receives 4 or 13. */
nyx_status nyx_offsets_default(int32_t dims, int32_t distance, nyx_offset *out_host, int32_t *n);

/* The GLCM feature columns: Supplementary Table S3 rows with the NY mark
 * (AVEAMP left out), in table order. */
int32_t nyx_feature_count(void);               /* 30 */
const char *nyx_feature_name(int32_t f);       /* NULL outside [0, 30) */

/* ROI discovery and per-ROI statistics (count, min, max, bbox) over a batch
 * of images: one row per unique nonzero label of each image (Supplementary
 * Table S7, "ROI/FOV"; the regional extraction of the Main section); the
 * levels are the fixed-bin-number grey levels of the texture
 * hyper-parameter n_bins (Methods, "Feature Control and Tunability").
 * Optionally the per-voxel grey level under each voxel's own ROI (0 for
 * background) into bins_out (device, caller-owned, one uint16 per voxel of
 * every image, laid out like the input images one after another).  rois:
 * caller-owned device arrays of rois->capacity rows; a smaller capacity than
 * the ROI count gives NYX_ERR_CAPACITY with the count in *n_rois_host and
 * nothing written.  Synchronises once to report the ROI count. */
nyx_status nyx_bin_rois(nyx_ctx *ctx, const nyx_image *imgs_host, int32_t n_images, int32_t n_bins,
                        nyx_roi_table *rois, uint16_t *bins_out, nyx_stream stream);

/* Co-occurrence counts (the grey-level co-occurrence matrix of the GLCM
 * rows of Supplementary Table S3, per offset: texture cost O(m, g, s) in
 * Methods, "Feature Control and Tunability") of the ROIs in `rois` (as
 * produced by nyx_bin_rois, with *rois->n_rois_host rows) for the given
 * offsets, as a sorted COO list in caller-owned device arrays (out->capacity
 * entries; too few gives NYX_ERR_CAPACITY with the count in *out->nnz_host
 * and nothing written).
 * `bins` (nullable) is a bin image as written by nyx_bin_rois; when NULL,
 * levels are computed on the fly from intensity and the ROI min/max.
 * Synchronises to report the nonzero count. */
nyx_status nyx_glcm_accumulate(nyx_ctx *ctx, const nyx_image *imgs_host, int32_t n_images,
                               const nyx_roi_table *rois, const uint16_t *bins,
                               const nyx_offset *offsets_host, int32_t n_offsets, int32_t symmetric,
                               int32_t n_bins, nyx_glcm *out, nyx_stream stream);

/* Feature table (normalisation, marginals and the 30 GLCM features of
 * Supplementary Table S3 per direction and their mean) from a COO list as
 * written by nyx_glcm_accumulate, into the caller-owned device table: row r
 * of the table belongs to ROI r of the list.  `rois` (nullable) is the ROI
 * table the list was accumulated for; when given, its *n_rois_host must equal
 * glcm->n_rois (NYX_ERR_INVALID otherwise), so a table is never paired with
 * another image batch's counts.  table has room for table_capacity_rows rows
 * (glcm->n_rois needed).  Synchronises to report entries outside their
 * matrix (NYX_ERR_INVALID). */
nyx_status nyx_glcm_features(nyx_ctx *ctx, const nyx_glcm *glcm, const nyx_roi_table *rois, nyx_precision prec,
                             void *table, int64_t table_capacity_rows, nyx_stream stream);

/* First-order intensity features of every ROI (the intensity group of
 * Supplementary Table S1, rows with the NY mark; Table S5 for volumes): the
 * statistics of each ROI's voxel values, in the column order of
 * nyx_intensity_feature_name(0..36): MEAN, MIN, MAX, RANGE,
 * INTEGRATED_INTENSITY, ENERGY (sum of squares), RMS, VARIANCE and STDDEV
 * (unbiased; 0 for one voxel), STANDARD_ERROR, SKEWNESS, KURTOSIS,
 * HYPERSKEWNESS, HYPERFLATNESS (biased central moments m3..m6 over
 * m2^(k/2); 0 for a constant ROI), MEAN_ABSOLUTE_DEVIATION, MEDIAN,
 * MEDIAN_ABSOLUTE_DEVIATION (mean distance to the median), P01, P10, P25,
 * P75, P90, P99 (linear interpolation between the closest ranks,
 * h = (n - 1) p / 100), INTERQUARTILE_RANGE, ROBUST_MEAN_ABSOLUTE_DEVIATION
 * (values within [P10, P90] about their mean; NaN when none lies there),
 * MODE (lowest fixed-bin-number level among the most frequent), ENTROPY
 * (log2) and UNIFORMITY of the level histogram (levels as for the texture
 * features, n_bins of them), UNIFORMITY_PIU (100 (1 - range / (max + min)),
 * 100 when max + min = 0), WEIGHTED_CENTROID_X/Y/Z (image column, row,
 * plane weighted by intensity; NaN when the intensities sum to 0), and the
 * integrated intensity, min, max, mean and unbiased standard deviation of
 * the edge voxels (ROI voxels with a face neighbour, 4 in a plane or 6 in a
 * volume, outside the image or the ROI).  The cost is O(m) per ROI of m
 * voxels for the moments and O(m, h) with h = n_bins for the histogram
 * features (Materials and methods, "Feature Control and Tunability").
 * table: n_rois rows of 37 values, float (NYX_FP32) or double (NYX_FP64);
 * every value is computed in double from exact integer sums, the order
 * statistics exactly.  rois (nullable) receives the ROI table.  n_bins in
 * [2, 8191] (NYX_ERR_UNSUPPORTED above).  Synchronises the stream (ROI count
 * and capacity checks). */
int32_t nyx_intensity_feature_count(void);         /* 37 */
const char *nyx_intensity_feature_name(int32_t f); /* NULL outside [0, 37) */
nyx_status nyx_intensity_features(nyx_ctx *ctx, const nyx_image *imgs_host, int32_t n_images, int32_t n_bins,
                                  nyx_precision prec, nyx_roi_table *rois, void *table,
                                  int64_t table_capacity_rows, nyx_stream stream);

/* Neighbourhood texture features of every ROI from one scan of each ROI
 * voxel's neighbourhood: the neighbouring grey level dependence matrix
 * (NGLDM, Supplementary Table S3 rows 175-192), the neighbourhood grey tone
 * difference matrix (NGTDM, rows 246-250) and the grey level dependence
 * matrix (GLDM, rows 251-264), the rows with the NY mark, in the column
 * order of nyx_neighbourhood_feature_name(0..36): 18 NGLDM_*, 5 NGTDM_*,
 * 14 GLDM_* columns.  Levels are the fixed-bin-number levels of the texture
 * features (n_bins); the neighbourhood is Chebyshev distance 1 (8 neighbours
 * in a plane, 26 in a volume), neighbours outside the image or the ROI do
 * not take part.  Dependence k = 1 + the neighbours whose level differs by at
 * most alpha (>= 0); S(i, k) counts the voxels of level i and dependence k,
 * and the NGLDM and GLDM columns are its emphases, non-uniformities, means,
 * variances, energy and entropy (log2) with p = S / voxels.  NGTDM: n_i
 * counts the voxels of level i with at least one neighbour, s_i sums
 * |i - mean neighbour level| over them; COARSENESS, CONTRAST, BUSYNESS,
 * COMPLEXITY, STRENGTH use p_i = n_i / sum n; a flat texture gives
 * COARSENESS = 1e6 and 0 for CONTRAST, BUSYNESS and STRENGTH, an ROI without
 * neighbouring voxels NaN for all five.  table: n_rois rows of 37 values,
 * float (NYX_FP32) or double (NYX_FP64), computed in double from exact
 * integer counts.  rois (nullable) receives the ROI table.  The per-ROI
 * tables live in LDS: NYX_ERR_UNSUPPORTED above about 1300 levels for 2D
 * images and 460 with a volume in the batch.  Synchronises the stream. */
int32_t nyx_neighbourhood_feature_count(void);         /* 37 */
const char *nyx_neighbourhood_feature_name(int32_t f); /* NULL outside [0, 37) */
nyx_status nyx_neighbourhood_features(nyx_ctx *ctx, const nyx_image *imgs_host, int32_t n_images, int32_t n_bins,
                                      int32_t alpha, nyx_precision prec, nyx_roi_table *rois, void *table,
                                      int64_t table_capacity_rows, nyx_stream stream);

/* Whole path in one call (regional GLCM texture of every ROI, Supplementary
 * Tables S3 and S7, with the hyper-parameters n_bins and offsets of Methods,
 * "Feature Control and Tunability"): plan, execute once, destroy the plan.
 * rois (nullable) and table are caller-owned device buffers; a table or ROI
 * capacity below the ROI count gives NYX_ERR_CAPACITY with the count in
 * *rois->n_rois_host. */
nyx_status nyx_extract_batch(nyx_ctx *ctx, const nyx_image *imgs_host, int32_t n_images,
                             const nyx_extract_opts *opts, nyx_roi_table *rois, void *table,
                             int64_t table_capacity_rows, nyx_stream stream);

/* The same pass as nyx_extract_batch, for callers that cannot allocate
 * device memory (code that must not call hipMalloc: serving loops, harnesses
 * that forbid allocation).  Allocates nothing: every scratch buffer of the
 * step (label statistics, ROI descriptors, work queue, split-ROI matrices,
 * reduced sums) is carved from one library-owned array of NYX_NOALLOC_SCRATCH_BYTES
 * per GPU, which the library holds until the process ends.  The caller still
 * passes the images, the ROI table (nullable) and the feature table.
 * opts->autotune and opts->workspace_cap_bytes are ignored (the configuration
 * is the untimed default, so results equal nyx_extract_batch's without
 * autotune).  A batch whose scratch exceeds the array gives NYX_ERR_CAPACITY
 * and a message with the size it needs; other errors as nyx_extract_batch.
 * Synchronises `stream` (twice during discovery, once at the end).  Every
 * call on one GPU uses that GPU's one array: calls that overlap on a GPU
 * (from several threads or streams) race and must be serialised by the
 * caller. */
#define NYX_NOALLOC_SCRATCH_BYTES (256ull << 20)
nyx_status nyx_extract_batch_noalloc(nyx_ctx *ctx, const nyx_image *imgs_host, int32_t n_images,
                                     const nyx_extract_opts *opts, nyx_roi_table *rois, void *table,
                                     int64_t table_capacity_rows, nyx_stream stream);

/* Plan for repeated extraction (the batched execution of the regional
 * extraction, Supplementary Table S7; "Scalability" in Results for the
 * many-small-ROI regime) over images with the same geometry and
 * labels-per-image capacity: discovers the ROIs once (one synchronisation),
 * sizes the work queue and scratch, and (with opts->autotune) picks the
 * kernel configuration by timing.  *n_rois_host receives the ROI count.
 * The image arrays must stay valid (and may change contents) while the plan
 * lives; a later execution whose labels exceed the planned capacity reports
 * NYX_ERR_CAPACITY from nyx_plan_check. */
nyx_status nyx_plan_create(nyx_ctx *ctx, const nyx_image *imgs_host, int32_t n_images,
                           const nyx_extract_opts *opts, nyx_plan **out, int64_t *n_rois_host);

/* One full pass of the batched path (ROI discovery, binning, accumulation,
 * features) as one graph replay on `stream`.  rois may be NULL. */
nyx_status nyx_plan_execute(nyx_plan *plan, nyx_roi_table *rois, void *table, nyx_stream stream);

/* The same pass with one kernel launch per ROI: the comparison baseline, the
 * per-ROI GPU regime the paper reports losing to the CPU for many small ROIs
 * (Results, "Scalability", Fig. 3f). */
nyx_status nyx_plan_execute_per_roi(nyx_plan *plan, nyx_roi_table *rois, void *table,
                                    nyx_stream stream);

/* Phases of one step, in order (indices into nyx_plan_profile's output). */
typedef enum nyx_phase {
    NYX_PHASE_RESET = 0,     /* clear per-label statistics and counters */
    NYX_PHASE_SCAN = 1,      /* ROI discovery: count, min, max, bbox per label */
    NYX_PHASE_COMPACT = 2,   /* ROI table and size-sorted work queue */
    NYX_PHASE_ZERO = 3,      /* clear the global matrices of split ROIs */
    NYX_PHASE_BATCH = 4,     /* binning, co-occurrence counts, reduced sums (work-group per item) */
    NYX_PHASE_BAND = 5,      /* split ROIs whose triangle exceeds LDS: banded counts, fold */
    NYX_PHASE_SPLIT = 6,     /* reduced sums of split ROIs from their merged global matrices */
    NYX_PHASE_FEATURES = 7,  /* the 30 features per direction and their mean, every ROI */
    NYX_PHASE_COUNT = 8
} nyx_phase;

/* Runs one step eagerly (no graph) on `stream` with HIP events between its
 * phases, synchronises, and writes the duration of each phase in
 * milliseconds to ms_host[NYX_PHASE_COUNT].  Results land in `table` as with
 * nyx_plan_execute.  For measurement only. */
nyx_status nyx_plan_profile(nyx_plan *plan, void *table, float *ms_host, nyx_stream stream);

/* Synchronises `stream` and reports any device-side capacity overflow of
 * the last execution. */
nyx_status nyx_plan_check(nyx_plan *plan, nyx_stream stream);

/* Human-readable description of the configuration the plan uses. */
const char *nyx_plan_describe(const nyx_plan *plan);

void nyx_plan_destroy(nyx_plan *plan);

#ifdef __cplusplus
}
#endif
#endif /* NYX_H */
