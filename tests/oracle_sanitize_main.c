/* oracle_sanitize_main.c -- test driver (not part of the library): runs the
 * oracle's entry points on small seeded inputs in one process built with
 * AddressSanitizer and UndefinedBehaviorSanitizer, so out-of-bounds accesses,
 * leaks and undefined arithmetic in the oracle fail the CPU test suite.
 * Exit status 0 means every call returned normally with sane results. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int64_t oracle_roi_count(const uint32_t *labels, int64_t nvox);
int64_t oracle_roi_stats(const uint16_t *, const uint32_t *, int64_t, int64_t, int64_t, int64_t, uint32_t *,
                         uint64_t *, uint16_t *, uint16_t *, int32_t *);
int oracle_bin_image(const uint16_t *, const uint32_t *, int64_t, int64_t, const uint32_t *, const uint16_t *,
                     const uint16_t *, int32_t, uint16_t *);
int oracle_glcm_roi(const uint16_t *, const uint32_t *, int64_t, int64_t, int64_t, uint32_t, uint16_t, uint16_t,
                    const int32_t *, int32_t, const int32_t *, int32_t, int32_t, uint64_t *);
void oracle_features_roi(const uint64_t *, int32_t, int32_t, double *);
double oracle_shade_magnitude(const uint64_t *, int32_t);
int oracle_extract(const uint16_t *, const uint32_t *, int64_t, int64_t, int64_t, int32_t, const int32_t *, int32_t,
                   int64_t, const uint32_t *, const uint16_t *, const uint16_t *, const int32_t *, double *,
                   double *, int32_t, int32_t);
int32_t oracle_default_offsets(int32_t dims, int32_t d, int32_t *out);

static uint64_t state = 0x9E3779B97F4A7C15ull;
static uint64_t next(void) { /* SplitMix64 */
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int run(int64_t nz, int64_t ny, int64_t nx, int32_t ng, int32_t dims, int32_t dist, uint32_t labels_max) {
    const int64_t n = nz * ny * nx;
    uint16_t *I = malloc((size_t)n * sizeof *I);
    uint32_t *L = malloc((size_t)n * sizeof *L);
    for (int64_t v = 0; v < n; ++v) {
        I[v] = (uint16_t)(next() >> 48);
        L[v] = (uint32_t)(next() % (labels_max + 1));
    }
    int32_t off[13 * 3];
    const int32_t K = oracle_default_offsets(dims, dist, off);
    const int64_t r = oracle_roi_count(L, n);
    uint32_t *lab = malloc((size_t)(r + 1) * sizeof *lab);
    uint64_t *cnt = malloc((size_t)(r + 1) * sizeof *cnt);
    uint16_t *lo = malloc((size_t)(r + 1) * sizeof *lo), *hi = malloc((size_t)(r + 1) * sizeof *hi);
    int32_t *bb = malloc((size_t)(r + 1) * 6 * sizeof *bb);
    if (oracle_roi_stats(I, L, nz, ny, nx, r, lab, cnt, lo, hi, bb) != r) return 1;
    uint16_t *bins = malloc((size_t)n * sizeof *bins);
    if (oracle_bin_image(I, L, n, r, lab, lo, hi, ng, bins) != 0) return 2;
    double *table = malloc((size_t)(r + 1) * (size_t)(K + 1) * 30 * sizeof *table);
    double *mag = malloc((size_t)(r + 1) * (size_t)K * sizeof *mag);
    for (int32_t sym = 0; sym <= 1; ++sym)
        if (oracle_extract(I, L, nz, ny, nx, ng, off, K, r, lab, lo, hi, bb, table, mag, sym, 1) != 0) return 3;
    uint64_t *P = malloc((size_t)K * (size_t)ng * (size_t)ng * sizeof *P);
    for (int64_t q = 0; q < r; ++q) {
        oracle_glcm_roi(I, L, nz, ny, nx, lab[q], lo[q], hi[q], bb + 6 * q, ng, off, K, (int32_t)(q & 1), P);
        double f[(13 + 1) * 30];
        oracle_features_roi(P, ng, K, f);
        for (int32_t k = 0; k < K; ++k) {
            const double m = oracle_shade_magnitude(P + (size_t)k * (size_t)ng * (size_t)ng, ng);
            if (!(isnan(m) || m >= fabs(f[k * 30 + 3]) * (1 - 1e-12))) return 4;
        }
    }
    free(I); free(L); free(lab); free(cnt); free(lo); free(hi); free(bb); free(bins); free(table); free(mag); free(P);
    return 0;
}

int main(void) {
    int rc;
    if ((rc = run(1, 13, 17, 8, 2, 1, 5))) return rc;
    if ((rc = run(1, 9, 31, 30, 2, 2, 3))) return rc;
    if ((rc = run(4, 6, 7, 5, 3, 1, 4))) return rc;
    if ((rc = run(1, 1, 1, 2, 2, 1, 1))) return rc;   /* one voxel: every direction empty */
    if ((rc = run(1, 5, 5, 100, 2, 1, 0))) return rc; /* background only: no ROI */
    printf("oracle sanitized run ok\n");
    return 0;
}
