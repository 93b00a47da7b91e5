/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU reference for per-ROI grey-level
 * co-occurrence (GLCM) texture, written from the method's definitions in
 * double precision.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load this library; the product (the HIP library)
 * never links or calls it, and the two share no code, tables or headers.
 *
 * What is computed, and where it is defined:
 *  - The problem: an intensity image plus a label mask in, one row of
 *    measurements per unique nonzero label out (paper, Supplementary
 *    Table S7, "ROI/FOV" criterion; Main section, regional vs image features).
 *  - Hyper-parameters: number of grey levels and the spatial offset / scan
 *    angle (paper, Materials and methods, "Feature Control and Tunability":
 *    texture cost O(m, g, s) in voxels m, grey scale g and offset s).
 *  - The GLCM feature list: Supplementary Table S3, GLCM rows 140-174 with
 *    an NY (Nyxus) mark; 3D GLCM is Table S5 row 361.  The paper prints no
 *    formulas and defers to the IBSI standard it cites (Results, "Accuracy and
 *    Reproducibility"); the formulas below are the standard IBSI/Haralick
 *    definitions.  Readings of points the paper leaves open are marked [A#]
 *    where they are applied (the same labels name them in the design notes).
 *
 * Conventions:
 *  - Image layout [nz][ny][nx], x fastest.  Label 0 is background; voxels
 *    carrying the same nonzero label form one ROI, connected or not [A1].
 *  - Fixed-bin-number discretisation over the ROI's own [min, max] with
 *    1-based levels 1..Ng, computed in exact integer arithmetic [A2, A3].
 *  - A pair (v, v+d) counts only if both voxels are inside the image and
 *    carry the ROI's label [A5]; the matrix is symmetrised P = C + C^T [A6]
 *    by default, or kept as the ordered counts P = C on request [A16].
 *  - Logarithms are base 2; 0 log 0 = 0 [A7].
 *  - Sums use Neumaier compensation; all arithmetic is binary64.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NFEAT 30

/* ------------------------------------------------------------------ sums */
typedef struct { double s, c; } nsum;

static void nadd(nsum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else                       a->c += (x - t) + a->s;
    a->s = t;
}
static double nval(const nsum *a) { return a->s + a->c; }

/* -------------------------------------------------------------- features */
/* Column order of the feature table: Table S3 GLCM rows with the NY mark, in
 * the table's order, without AVEAMP (#142), which the paper never defines [A8]. */
static const char *const ORACLE_NAMES[NFEAT] = {
    "ASM", "ACOR", "CLUPROM", "CLUSHADE", "CLUTEND", "CONTRAST", "CORR",
    "DIFAVE", "DIFENTRO", "DIFVAR", "DIS", "ENERGY", "ENTROPY", "HOM1",
    "HOM2", "IDM", "INFOMEAS1", "INFOMEAS2", "IDMN", "ID", "IDN", "IV",
    "JAVE", "JE", "JMAX", "SUMAVE", "SUMENT", "JVAR", "SUMVAR", "VARIANCE"};

int32_t oracle_feature_count(void) { return NFEAT; }
const char *oracle_feature_name(int32_t f) {
    return (f >= 0 && f < NFEAT) ? ORACLE_NAMES[f] : (const char *)0;
}

/* ------------------------------------------------------------- binning */
/* Fixed bin number over the ROI's own range [A2]: level 1 + floor(Ng (I-min)
 * / (max-min)), clamped to Ng (the clamp only fires at I = max); a constant
 * ROI maps to level 1.  Exact: the numerator is below 2^32. */
uint32_t oracle_bin(uint32_t intensity, uint32_t vmin, uint32_t vmax, int32_t n_bins) {
    if (vmax == vmin) return 1u;
    uint64_t num = (uint64_t)(uint32_t)n_bins * (uint64_t)(intensity - vmin);
    uint64_t q = num / (uint64_t)(vmax - vmin);
    uint64_t b = 1u + q;
    if (b > (uint64_t)n_bins) b = (uint64_t)n_bins;
    return (uint32_t)b;
}

/* --------------------------------------------------------- ROI discovery */
static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* Number of distinct nonzero labels in one image. */
int64_t oracle_roi_count(const uint32_t *labels, int64_t nvox) {
    uint32_t *tmp = (uint32_t *)malloc((size_t)(nvox > 0 ? nvox : 1) * sizeof(uint32_t));
    if (!tmp) return -1;
    int64_t m = 0;
    for (int64_t v = 0; v < nvox; ++v) if (labels[v] != 0) tmp[m++] = labels[v];
    qsort(tmp, (size_t)m, sizeof(uint32_t), cmp_u32);
    int64_t u = 0;
    for (int64_t i = 0; i < m; ++i) if (i == 0 || tmp[i] != tmp[i - 1]) ++u;
    free(tmp);
    return u;
}

/* Per-ROI statistics for one image, ROIs in ascending label order.
 * bbox holds 6 int32 per ROI: x_min, y_min, z_min, x_max, y_max, z_max
 * (inclusive).  Returns the number of ROIs, or -1 if it exceeds cap / on
 * allocation failure. */
int64_t oracle_roi_stats(const uint16_t *intensity, const uint32_t *labels,
                         int64_t nz, int64_t ny, int64_t nx, int64_t cap,
                         uint32_t *label_out, uint64_t *count_out,
                         uint16_t *vmin_out, uint16_t *vmax_out, int32_t *bbox_out) {
    int64_t nvox = nz * ny * nx;
    uint32_t *tmp = (uint32_t *)malloc((size_t)(nvox > 0 ? nvox : 1) * sizeof(uint32_t));
    if (!tmp) return -1;
    int64_t m = 0;
    for (int64_t v = 0; v < nvox; ++v) if (labels[v] != 0) tmp[m++] = labels[v];
    qsort(tmp, (size_t)m, sizeof(uint32_t), cmp_u32);
    int64_t u = 0;
    for (int64_t i = 0; i < m; ++i)
        if (i == 0 || tmp[i] != tmp[i - 1]) tmp[u++] = tmp[i];
    if (u > cap) { free(tmp); return -1; }
    for (int64_t r = 0; r < u; ++r) {
        label_out[r] = tmp[r];
        count_out[r] = 0;
        vmin_out[r] = 0xFFFF;
        vmax_out[r] = 0;
        bbox_out[6 * r + 0] = bbox_out[6 * r + 1] = bbox_out[6 * r + 2] = INT32_MAX;
        bbox_out[6 * r + 3] = bbox_out[6 * r + 4] = bbox_out[6 * r + 5] = -1;
    }
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t v = (z * ny + y) * nx + x;
                uint32_t l = labels[v];
                if (l == 0) continue;
                /* binary search of l in the sorted unique label list */
                int64_t lo = 0, hi = u - 1, r = -1;
                while (lo <= hi) {
                    int64_t mid = (lo + hi) / 2;
                    if (tmp[mid] == l) { r = mid; break; }
                    if (tmp[mid] < l) lo = mid + 1; else hi = mid - 1;
                }
                count_out[r] += 1;
                if (intensity[v] < vmin_out[r]) vmin_out[r] = intensity[v];
                if (intensity[v] > vmax_out[r]) vmax_out[r] = intensity[v];
                int32_t *b = bbox_out + 6 * r;
                if (x < b[0]) b[0] = (int32_t)x;
                if (y < b[1]) b[1] = (int32_t)y;
                if (z < b[2]) b[2] = (int32_t)z;
                if (x > b[3]) b[3] = (int32_t)x;
                if (y > b[4]) b[4] = (int32_t)y;
                if (z > b[5]) b[5] = (int32_t)z;
            }
    free(tmp);
    return u;
}

/* Bin image: the level of every ROI voxel under its own ROI's range, 0 for
 * background.  The ROI statistics come from oracle_roi_stats. */
int oracle_bin_image(const uint16_t *intensity, const uint32_t *labels, int64_t nvox,
                     int64_t n_rois, const uint32_t *roi_label, const uint16_t *roi_min,
                     const uint16_t *roi_max, int32_t n_bins, uint16_t *bins_out) {
    for (int64_t v = 0; v < nvox; ++v) {
        uint32_t l = labels[v];
        if (l == 0) { bins_out[v] = 0; continue; }
        int64_t lo = 0, hi = n_rois - 1, r = -1;
        while (lo <= hi) {
            int64_t mid = (lo + hi) / 2;
            if (roi_label[mid] == l) { r = mid; break; }
            if (roi_label[mid] < l) lo = mid + 1; else hi = mid - 1;
        }
        if (r < 0) return -1;
        bins_out[v] = (uint16_t)oracle_bin(intensity[v], roi_min[r], roi_max[r], n_bins);
    }
    return 0;
}

/* ------------------------------------------------------------ matrices */
/* Co-occurrence matrices of one ROI, one per offset: P[k][i][j] (Ng x Ng,
 * 0-based level indices).  For each ROI voxel v and offset d_k, the pair
 * (v, v + d_k) counts when v + d_k is inside the image and carries the same
 * label [A5]; C(i, j) is the number of such pairs with level i at v and j at
 * v + d_k.  symmetric != 0: P = C + C^T [A6]; symmetric == 0: P = C, the
 * ordered counts [A16]. */
int oracle_glcm_roi(const uint16_t *intensity, const uint32_t *labels,
                    int64_t nz, int64_t ny, int64_t nx, uint32_t label,
                    uint16_t vmin, uint16_t vmax, const int32_t *bbox,
                    int32_t n_bins, const int32_t *offsets, int32_t n_offsets,
                    int32_t symmetric, uint64_t *P) {
    int64_t ng = n_bins;
    memset(P, 0, (size_t)n_offsets * (size_t)(ng * ng) * sizeof(uint64_t));
    for (int32_t k = 0; k < n_offsets; ++k) {
        int64_t dz = offsets[3 * k + 0], dy = offsets[3 * k + 1], dx = offsets[3 * k + 2];
        uint64_t *Pk = P + (size_t)k * (size_t)(ng * ng);
        for (int64_t z = bbox[2]; z <= bbox[5]; ++z)
            for (int64_t y = bbox[1]; y <= bbox[4]; ++y)
                for (int64_t x = bbox[0]; x <= bbox[3]; ++x) {
                    int64_t v = (z * ny + y) * nx + x;
                    if (labels[v] != label) continue;
                    int64_t wz = z + dz, wy = y + dy, wx = x + dx;
                    if (wz < 0 || wz >= nz || wy < 0 || wy >= ny || wx < 0 || wx >= nx) continue;
                    int64_t w = (wz * ny + wy) * nx + wx;
                    if (labels[w] != label) continue;
                    int64_t i = (int64_t)oracle_bin(intensity[v], vmin, vmax, n_bins) - 1;
                    int64_t j = (int64_t)oracle_bin(intensity[w], vmin, vmax, n_bins) - 1;
                    Pk[i * ng + j] += 1;                 /* C(i, j) */
                    if (symmetric) Pk[j * ng + i] += 1;  /* C^T contributes C(i, j) at (j, i) */
                }
    }
    return 0;
}

/* ------------------------------------------------------------ features */
/* The 30 GLCM features of one matrix P (Ng x Ng counts, symmetric or not), written to
 * out[0..29] in ORACLE_NAMES order.  Every feature is its own plain loop over
 * the normalised matrix p = P / T, following the standard definitions. */
void oracle_features(const uint64_t *P, int32_t n_bins, double *out) {
    const int64_t ng = n_bins;
    uint64_t T = 0;
    for (int64_t c = 0; c < ng * ng; ++c) T += P[c];
    if (T == 0) { /* no pair in this direction: every feature undefined */
        for (int f = 0; f < NFEAT; ++f) out[f] = NAN;
        return;
    }
    const double Td = (double)T;
#define PIJ(i, j) ((double)P[(i) * ng + (j)] / Td)
    /* levels are 1-based: level of index i is (i + 1) [A3] */

    /* marginals p_x(i) = sum_j p_ij and p_y(j) = sum_i p_ij */
    double *px = (double *)calloc((size_t)ng, sizeof(double));
    double *py = (double *)calloc((size_t)ng, sizeof(double));
    double *psum = (double *)calloc((size_t)(2 * ng + 1), sizeof(double)); /* k = 2..2Ng */
    double *pdif = (double *)calloc((size_t)ng, sizeof(double));           /* k = 0..Ng-1 */
    for (int64_t i = 0; i < ng; ++i) {
        nsum a = {0, 0};
        for (int64_t j = 0; j < ng; ++j) nadd(&a, PIJ(i, j));
        px[i] = nval(&a);
    }
    for (int64_t j = 0; j < ng; ++j) {
        nsum a = {0, 0};
        for (int64_t i = 0; i < ng; ++i) nadd(&a, PIJ(i, j));
        py[j] = nval(&a);
    }
    for (int64_t k = 2; k <= 2 * ng; ++k) {
        nsum a = {0, 0};
        for (int64_t i = 0; i < ng; ++i) {
            int64_t j = k - (i + 1) - 1; /* level(j) = k - level(i) */
            if (j >= 0 && j < ng) nadd(&a, PIJ(i, j));
        }
        psum[k] = nval(&a);
    }
    for (int64_t k = 0; k < ng; ++k) { /* cells with |i - j| = k: j = i + k and j = i - k */
        nsum a = {0, 0};
        for (int64_t i = 0; i < ng; ++i) {
            if (i + k < ng) nadd(&a, PIJ(i, i + k));
            if (k > 0 && i - k >= 0) nadd(&a, PIJ(i, i - k));
        }
        pdif[k] = nval(&a);
    }

    /* means and standard deviations of the marginals */
    nsum a;
    a = (nsum){0, 0}; for (int64_t i = 0; i < ng; ++i) nadd(&a, (double)(i + 1) * px[i]);
    const double mux = nval(&a);
    a = (nsum){0, 0}; for (int64_t j = 0; j < ng; ++j) nadd(&a, (double)(j + 1) * py[j]);
    const double muy = nval(&a);
    a = (nsum){0, 0}; for (int64_t i = 0; i < ng; ++i) { double d = (double)(i + 1) - mux; nadd(&a, d * d * px[i]); }
    const double sx = sqrt(nval(&a));
    a = (nsum){0, 0}; for (int64_t j = 0; j < ng; ++j) { double d = (double)(j + 1) - muy; nadd(&a, d * d * py[j]); }
    const double sy = sqrt(nval(&a));

    /* single-level test on integers [A11, A16]: exactly one level has a
     * nonzero row, or exactly one level has a nonzero column (the same test
     * for a symmetric matrix).  Then p_ij = p_x(i) p_y(j), so the correlation
     * is 0/0 and the mutual information is exactly 0. */
    int64_t nonzero_rows = 0, nonzero_cols = 0;
    for (int64_t i = 0; i < ng; ++i) {
        uint64_t row = 0, col = 0;
        for (int64_t j = 0; j < ng; ++j) { row += P[i * ng + j]; col += P[j * ng + i]; }
        if (row) ++nonzero_rows;
        if (col) ++nonzero_cols;
    }
    const int single_level = (nonzero_rows == 1 || nonzero_cols == 1);
    /* occupied levels of the sum and difference marginals, on integers [A17] */
    int64_t nonzero_sums = 0, nonzero_difs = 0;
    for (int64_t k = 0; k <= 2 * ng - 2; ++k) {
        uint64_t c = 0;
        for (int64_t i = 0; i < ng; ++i) if (k - i >= 0 && k - i < ng) c += P[i * ng + (k - i)];
        if (c) ++nonzero_sums;
    }
    for (int64_t k = 0; k < ng; ++k) {
        uint64_t c = 0;
        for (int64_t i = 0; i < ng; ++i) {
            if (i + k < ng) c += P[i * ng + i + k];
            if (k > 0 && i - k >= 0) c += P[i * ng + i - k];
        }
        if (c) ++nonzero_difs;
    }

    double f[NFEAT];
    /* 1 ASM: sum p^2 */
    a = (nsum){0, 0};
    for (int64_t i = 0; i < ng; ++i) for (int64_t j = 0; j < ng; ++j) { double p = PIJ(i, j); nadd(&a, p * p); }
    f[0] = nval(&a);
    /* 2 ACOR: sum i j p */
    a = (nsum){0, 0};
    for (int64_t i = 0; i < ng; ++i) for (int64_t j = 0; j < ng; ++j) nadd(&a, (double)(i + 1) * (double)(j + 1) * PIJ(i, j));
    f[1] = nval(&a);
    /* 3-5 cluster prominence / shade / tendency: powers of (i + j - mux - muy) */
    {
        nsum a4 = {0, 0}, a3 = {0, 0}, a2 = {0, 0};
        for (int64_t i = 0; i < ng; ++i)
            for (int64_t j = 0; j < ng; ++j) {
                double p = PIJ(i, j);
                double d = (double)(i + 1) + (double)(j + 1) - mux - muy;
                nadd(&a4, d * d * d * d * p);
                nadd(&a3, d * d * d * p);
                nadd(&a2, d * d * p);
            }
        f[2] = nval(&a4);
        f[3] = nval(&a3);
        f[4] = nval(&a2);
    }
    /* 6 CONTRAST: sum (i - j)^2 p */
    a = (nsum){0, 0};
    for (int64_t i = 0; i < ng; ++i) for (int64_t j = 0; j < ng; ++j) { double d = (double)(i - j); nadd(&a, d * d * PIJ(i, j)); }
    f[5] = nval(&a);
    /* 7 CORR: sum (i - mux)(j - muy) p / (sx sy); 1 on a single-level matrix [A11] */
    if (single_level) f[6] = 1.0;
    else {
        a = (nsum){0, 0};
        for (int64_t i = 0; i < ng; ++i) for (int64_t j = 0; j < ng; ++j)
            nadd(&a, ((double)(i + 1) - mux) * ((double)(j + 1) - muy) * PIJ(i, j));
        f[6] = nval(&a) / (sx * sy);
    }
    /* 8 DIFAVE: sum k p_{x-y}(k) */
    a = (nsum){0, 0}; for (int64_t k = 0; k < ng; ++k) nadd(&a, (double)k * pdif[k]);
    const double difave = nval(&a);
    f[7] = difave;
    /* 9 DIFENTRO: -sum p_{x-y} log2 p_{x-y} */
    a = (nsum){0, 0}; for (int64_t k = 0; k < ng; ++k) if (pdif[k] > 0) nadd(&a, -pdif[k] * log2(pdif[k]));
    f[8] = nval(&a);
    /* 10 DIFVAR: sum (k - DIFAVE)^2 p_{x-y}(k), centred on DIFAVE [A12] */
    a = (nsum){0, 0}; for (int64_t k = 0; k < ng; ++k) { double d = (double)k - difave; nadd(&a, d * d * pdif[k]); }
    f[9] = nval(&a);
    /* 11 DIS: sum |i - j| p */
    a = (nsum){0, 0};
    for (int64_t i = 0; i < ng; ++i) for (int64_t j = 0; j < ng; ++j) nadd(&a, fabs((double)(i - j)) * PIJ(i, j));
    f[10] = nval(&a);
    /* 12 ENERGY: sum p^2 (the same quantity as ASM under the common reading) [A9] */
    a = (nsum){0, 0};
    for (int64_t i = 0; i < ng; ++i) for (int64_t j = 0; j < ng; ++j) { double p = PIJ(i, j); nadd(&a, p * p); }
    f[11] = nval(&a);
    /* 13 ENTROPY and 24 JE: -sum p log2 p [A9] */
    a = (nsum){0, 0};
    for (int64_t i = 0; i < ng; ++i) for (int64_t j = 0; j < ng; ++j) { double p = PIJ(i, j); if (p > 0) nadd(&a, -p * log2(p)); }
    const double hxy = nval(&a);
    f[12] = hxy;
    f[23] = hxy;
    /* 14 HOM1 and 20 ID: sum p / (1 + |i - j|) */
    a = (nsum){0, 0};
    for (int64_t i = 0; i < ng; ++i) for (int64_t j = 0; j < ng; ++j) nadd(&a, PIJ(i, j) / (1.0 + fabs((double)(i - j))));
    f[13] = nval(&a);
    f[19] = f[13];
    /* 15 HOM2 and 16 IDM: sum p / (1 + (i - j)^2) */
    a = (nsum){0, 0};
    for (int64_t i = 0; i < ng; ++i) for (int64_t j = 0; j < ng; ++j) { double d = (double)(i - j); nadd(&a, PIJ(i, j) / (1.0 + d * d)); }
    f[14] = nval(&a);
    f[15] = f[14];
    /* 17, 18 information measures of correlation from HX, HY, HXY, HXY1, HXY2 */
    {
        nsum hx = {0, 0}, hy = {0, 0}, h1 = {0, 0}, h2 = {0, 0};
        for (int64_t i = 0; i < ng; ++i) if (px[i] > 0) nadd(&hx, -px[i] * log2(px[i]));
        for (int64_t j = 0; j < ng; ++j) if (py[j] > 0) nadd(&hy, -py[j] * log2(py[j]));
        for (int64_t i = 0; i < ng; ++i)
            for (int64_t j = 0; j < ng; ++j) {
                double p = PIJ(i, j);
                double q = px[i] * py[j];
                if (p > 0) nadd(&h1, -p * log2(q));
                if (q > 0) nadd(&h2, -q * log2(q));
            }
        double HX = nval(&hx), HY = nval(&hy), HXY1 = nval(&h1), HXY2 = nval(&h2);
        double hmax = HX > HY ? HX : HY;
        f[16] = single_level ? 0.0 : (hxy - HXY1) / hmax;           /* 0/0 -> 0 [A11] */
        double arg = HXY2 - hxy;
        if (arg < 0) arg = 0;                                      /* [A7] */
        f[17] = single_level ? 0.0 : sqrt(1.0 - exp(-2.0 * arg));  /* MI = 0 exactly [A16] */
    }
    /* 19 IDMN: sum p / (1 + (i - j)^2 / Ng^2) */
    a = (nsum){0, 0};
    for (int64_t i = 0; i < ng; ++i) for (int64_t j = 0; j < ng; ++j) {
        double d = (double)(i - j);
        nadd(&a, PIJ(i, j) / (1.0 + d * d / ((double)ng * (double)ng)));
    }
    f[18] = nval(&a);
    /* 21 IDN: sum p / (1 + |i - j| / Ng) */
    a = (nsum){0, 0};
    for (int64_t i = 0; i < ng; ++i) for (int64_t j = 0; j < ng; ++j)
        nadd(&a, PIJ(i, j) / (1.0 + fabs((double)(i - j)) / (double)ng));
    f[20] = nval(&a);
    /* 22 IV: sum over i != j of p / (i - j)^2 */
    a = (nsum){0, 0};
    for (int64_t i = 0; i < ng; ++i) for (int64_t j = 0; j < ng; ++j)
        if (i != j) { double d = (double)(i - j); nadd(&a, PIJ(i, j) / (d * d)); }
    f[21] = nval(&a);
    /* 23 JAVE: mu = sum i p */
    a = (nsum){0, 0};
    for (int64_t i = 0; i < ng; ++i) for (int64_t j = 0; j < ng; ++j) nadd(&a, (double)(i + 1) * PIJ(i, j));
    const double mu = nval(&a);
    f[22] = mu;
    /* 25 JMAX: max p */
    {
        uint64_t m = 0;
        for (int64_t c = 0; c < ng * ng; ++c) if (P[c] > m) m = P[c];
        f[24] = (double)m / Td;
    }
    /* 26 SUMAVE: sum k p_{x+y}(k) */
    a = (nsum){0, 0}; for (int64_t k = 2; k <= 2 * ng; ++k) nadd(&a, (double)k * psum[k]);
    const double sumave = nval(&a);
    f[25] = sumave;
    /* 27 SUMENT: -sum p_{x+y} log2 p_{x+y} */
    a = (nsum){0, 0}; for (int64_t k = 2; k <= 2 * ng; ++k) if (psum[k] > 0) nadd(&a, -psum[k] * log2(psum[k]));
    f[26] = nval(&a);
    /* 28 JVAR and 30 VARIANCE: sum (i - mu)^2 p [A9] */
    a = (nsum){0, 0};
    for (int64_t i = 0; i < ng; ++i) for (int64_t j = 0; j < ng; ++j) { double d = (double)(i + 1) - mu; nadd(&a, d * d * PIJ(i, j)); }
    f[27] = nval(&a);
    f[29] = f[27];
    /* 29 SUMVAR: sum (k - SUMAVE)^2 p_{x+y}(k), centred on SUMAVE [A12] */
    a = (nsum){0, 0}; for (int64_t k = 2; k <= 2 * ng; ++k) { double d = (double)k - sumave; nadd(&a, d * d * psum[k]); }
    f[28] = nval(&a);
#undef PIJ
    /* A centred moment of a distribution on one value is exactly 0; the sums
     * above leave the rounding of the computed mean instead [A17]. */
    if (nonzero_rows == 1) f[27] = f[29] = 0.0;                  /* JVAR, VARIANCE */
    if (nonzero_sums == 1) f[2] = f[3] = f[4] = f[28] = 0.0;     /* CLUPROM, CLUSHADE, CLUTEND, SUMVAR */
    if (nonzero_difs == 1) f[9] = 0.0;                           /* DIFVAR */
    for (int q = 0; q < NFEAT; ++q) out[q] = f[q];
    free(px); free(py); free(psum); free(pdif);
}

/* Per-direction features then the arithmetic mean over directions whose
 * matrix is non-empty [A10]; out holds (n_offsets + 1) blocks of 30. */
void oracle_features_roi(const uint64_t *P, int32_t n_bins, int32_t n_offsets, double *out) {
    const int64_t cells = (int64_t)n_bins * n_bins;
    double *mean = out + (size_t)n_offsets * NFEAT;
    for (int q = 0; q < NFEAT; ++q) mean[q] = 0.0;
    int used = 0;
    for (int32_t k = 0; k < n_offsets; ++k) {
        double *blk = out + (size_t)k * NFEAT;
        oracle_features(P + (size_t)k * (size_t)cells, n_bins, blk);
        if (!isnan(blk[0])) {
            for (int q = 0; q < NFEAT; ++q) mean[q] += blk[q];
            ++used;
        }
    }
    for (int q = 0; q < NFEAT; ++q) mean[q] = used ? mean[q] / (double)used : NAN;
}

/* ------------------------------------------------------- error scale */
/* Magnitude the cluster-shade sum is formed from: sum |i + j - mux - muy|^3 p
 * over the normalised matrix (the same centring as CLUSHADE).  Not a
 * feature: the error measure of the parity tests divides a cluster-shade
 * difference by it, because a signed sum of cubes can cancel to near zero
 * while its rounding error scales with the magnitudes summed.  NaN for an
 * empty matrix. */
double oracle_shade_magnitude(const uint64_t *P, int32_t n_bins) {
    const int64_t ng = n_bins;
    uint64_t T = 0;
    for (int64_t c = 0; c < ng * ng; ++c) T += P[c];
    if (T == 0) return NAN;
    const double Td = (double)T;
    nsum mx = {0, 0}, my = {0, 0};
    for (int64_t i = 0; i < ng; ++i)
        for (int64_t j = 0; j < ng; ++j) {
            double p = (double)P[i * ng + j] / Td;
            nadd(&mx, (double)(i + 1) * p);
            nadd(&my, (double)(j + 1) * p);
        }
    const double mux = nval(&mx), muy = nval(&my);
    nsum a = {0, 0};
    for (int64_t i = 0; i < ng; ++i)
        for (int64_t j = 0; j < ng; ++j) {
            double d = fabs((double)(i + 1) + (double)(j + 1) - mux - muy);
            nadd(&a, d * d * d * (double)P[i * ng + j] / Td);
        }
    return nval(&a);
}

/* ------------------------------------------------------------- pipeline */
/* Feature table for a list of ROIs of one image (ROI statistics as produced
 * by oracle_roi_stats): table[r][blk][f] with blk = 0..n_offsets-1 the
 * directions and blk = n_offsets the direction mean; shade_mag (nullable)
 * receives oracle_shade_magnitude of every (ROI, direction); symmetric as for
 * oracle_glcm_roi.  n_threads > 1 runs
 * independent ROIs on OpenMP threads (timing only; results do not depend on
 * it).  Returns 0, or -1 on allocation failure. */
int oracle_extract(const uint16_t *intensity, const uint32_t *labels,
                   int64_t nz, int64_t ny, int64_t nx, int32_t n_bins,
                   const int32_t *offsets, int32_t n_offsets, int64_t n_rois,
                   const uint32_t *roi_label, const uint16_t *roi_min,
                   const uint16_t *roi_max, const int32_t *roi_bbox,
                   double *table, double *shade_mag, int32_t symmetric, int32_t n_threads) {
    const size_t cells = (size_t)n_bins * (size_t)n_bins * (size_t)n_offsets;
    int failed = 0;
#pragma omp parallel num_threads(n_threads > 0 ? n_threads : 1) reduction(| : failed)
    {
        uint64_t *P = (uint64_t *)malloc(cells * sizeof(uint64_t));
        if (!P) failed = 1;
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < n_rois; ++r) {
            if (!P) continue;
            oracle_glcm_roi(intensity, labels, nz, ny, nx, roi_label[r], roi_min[r], roi_max[r],
                            roi_bbox + 6 * r, n_bins, offsets, n_offsets, symmetric, P);
            oracle_features_roi(P, n_bins, n_offsets, table + (size_t)r * (size_t)(n_offsets + 1) * NFEAT);
            if (shade_mag)
                for (int32_t k = 0; k < n_offsets; ++k)
                    shade_mag[(size_t)r * (size_t)n_offsets + (size_t)k] =
                        oracle_shade_magnitude(P + (size_t)k * (size_t)n_bins * (size_t)n_bins, n_bins);
        }
        free(P);
    }
    return failed ? -1 : 0;
}

/* Default offsets at distance d [A4]: 2D = 0, 45, 90, 135 degrees with y
 * increasing downward; 3D = one representative of each +/- pair of the 26
 * neighbours.  Writes (dz, dy, dx) triples; returns the count (4 or 13). */
int32_t oracle_default_offsets(int32_t dims, int32_t d, int32_t *out) {
    static const int32_t two[4][3] = {{0, 0, 1}, {0, -1, 1}, {0, -1, 0}, {0, -1, -1}};
    static const int32_t three[13][3] = {
        {0, 0, 1}, {0, 1, 0}, {1, 0, 0}, {0, 1, 1}, {0, 1, -1}, {1, 0, 1}, {1, 0, -1},
        {1, 1, 0}, {1, -1, 0}, {1, 1, 1}, {1, 1, -1}, {1, -1, 1}, {1, -1, -1}};
    if (dims == 2) {
        for (int k = 0; k < 4; ++k) for (int a = 0; a < 3; ++a) out[3 * k + a] = two[k][a] * d;
        return 4;
    }
    if (dims == 3) {
        for (int k = 0; k < 13; ++k) for (int a = 0; a < 3; ++a) out[3 * k + a] = three[k][a] * d;
        return 13;
    }
    return -1;
}
