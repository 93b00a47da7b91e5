/*
 * synth.c -- seeded synthetic inputs (intensity images and label masks).
 *
 * Shared by the tests and the benchmark as INPUT GENERATION ONLY: nothing
 * here bins, counts or reduces anything the texture method computes.
 * The inputs stand in for the paper's workloads (Results, "Scalability":
 * TissueNet-like 2D images with many small cell regions; Decathlon-like
 * volumes with few large regions; the synthetic ROI-size / ROI-count sweep).
 *
 * Randomness: SplitMix64 (Steele, Lea & Flood 2014), used counter-style:
 * every draw is mix(seed, stream, index), so results do not depend on the
 * number of threads or on evaluation order.  Uniform doubles take the top
 * 53 bits; normals use Box-Muller; Poisson noise uses inversion for
 * lambda < 64 and round(lambda + sqrt(lambda) z) above.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

static inline uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
/* Counter-based draw: stream separates independent uses of one seed. */
static inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t idx) {
    return mix64(mix64(seed * 0x9E3779B97F4A7C15ull + stream) ^ (idx * 0xD1B54A32D192ED03ull));
}
static inline double u01(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }
/* (0, 1]: safe for log */
static inline double u01_open(uint64_t x) { return ((double)(x >> 11) + 1.0) * 0x1.0p-53; }
static inline double normal(uint64_t seed, uint64_t stream, uint64_t idx) {
    double u1 = u01_open(draw(seed, stream, 2 * idx));
    double u2 = u01(draw(seed, stream, 2 * idx + 1));
    return sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
}

/* iid integers in [0, 4095] (x >> 52 is exactly uniform). */
void synth_uniform12(uint64_t seed, int64_t n, uint16_t *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) out[i] = (uint16_t)(draw(seed, 1, (uint64_t)i) >> 52);
}

static uint16_t poisson_clip(uint64_t seed, uint64_t idx, double lam) {
    double v;
    if (lam <= 0) v = 0;
    else if (lam < 64.0) { /* inversion */
        double u = u01(draw(seed, 7, idx));
        double p = exp(-lam), c = p;
        int k = 0;
        while (u > c && k < 1000) { ++k; p *= lam / k; c += p; }
        v = k;
    } else {
        v = floor(lam + sqrt(lam) * normal(seed, 8, idx) + 0.5);
    }
    if (v < 0) v = 0;
    if (v > 65535) v = 65535;
    return (uint16_t)v;
}

/* Background plus Gaussian blobs (sigma ~ U[s_lo, s_hi], amplitude ~
 * U[a_lo, a_hi], centres uniform, rendered out to 4 sigma), then Poisson
 * noise, clipped to [0, 65535]. */
static void blob_image(uint64_t seed, int64_t ny, int64_t nx, int64_t n_blobs,
                       double s_lo, double s_hi, double a_lo, double a_hi,
                       double background, uint16_t *out, int par) {
    double *canvas = (double *)malloc((size_t)(ny * nx) * sizeof(double));
    for (int64_t i = 0; i < ny * nx; ++i) canvas[i] = background;
    for (int64_t b = 0; b < n_blobs; ++b) {
        double cx = u01(draw(seed, 2, 4 * b + 0)) * (double)nx;
        double cy = u01(draw(seed, 2, 4 * b + 1)) * (double)ny;
        double s = s_lo + (s_hi - s_lo) * u01(draw(seed, 2, 4 * b + 2));
        double a = a_lo + (a_hi - a_lo) * u01(draw(seed, 2, 4 * b + 3));
        int64_t x0 = (int64_t)floor(cx - 4 * s), x1 = (int64_t)ceil(cx + 4 * s);
        int64_t y0 = (int64_t)floor(cy - 4 * s), y1 = (int64_t)ceil(cy + 4 * s);
        if (x0 < 0) x0 = 0;
        if (y0 < 0) y0 = 0;
        if (x1 > nx - 1) x1 = nx - 1;
        if (y1 > ny - 1) y1 = ny - 1;
        double inv = 1.0 / (2 * s * s);
        for (int64_t y = y0; y <= y1; ++y)
            for (int64_t x = x0; x <= x1; ++x) {
                double dx = (double)x - cx, dy = (double)y - cy;
                double r2 = dx * dx + dy * dy;
                if (r2 <= 16 * s * s) canvas[y * nx + x] += a * exp(-r2 * inv);
            }
    }
#pragma omp parallel for schedule(static) if (par)
    for (int64_t i = 0; i < ny * nx; ++i) out[i] = poisson_clip(seed, (uint64_t)i, canvas[i]);
    free(canvas);
}

void synth_blob_image(uint64_t seed, int64_t ny, int64_t nx, int64_t n_blobs,
                      double s_lo, double s_hi, double a_lo, double a_hi,
                      double background, uint16_t *out) {
    blob_image(seed, ny, nx, n_blobs, s_lo, s_hi, a_lo, a_hi, background, out, 1);
}

/* n_images independent blob images, image k seeded seeds[k]; images run on
 * OpenMP threads (each image's content does not depend on the thread count). */
void synth_blob_images(const uint64_t *seeds, int64_t n_images, int64_t ny, int64_t nx,
                       int64_t n_blobs, double s_lo, double s_hi, double a_lo, double a_hi,
                       double background, uint16_t *out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < n_images; ++k)
        blob_image(seeds[k], ny, nx, n_blobs, s_lo, s_hi, a_lo, a_hi, background,
                   out + (size_t)k * (size_t)(ny * nx), 0);
}

/* 3D Gaussian random field: white N(0,1) -> separable Gaussian blur (sigma,
 * mirror boundary, radius ceil(3 sigma)) -> rescaled to unit variance ->
 * round(clip(mean + sd_g g + sd_n n, 0, 65535)) with n iid N(0,1). */
void synth_grf_volume(uint64_t seed, int64_t nz, int64_t ny, int64_t nx, double sigma,
                      double mean, double sd_g, double sd_n, uint16_t *out) {
    int64_t n = nz * ny * nx;
    float *a = (float *)malloc((size_t)n * sizeof(float));
    float *b = (float *)malloc((size_t)n * sizeof(float));
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) a[i] = (float)normal(seed, 3, (uint64_t)i);
    int r = (int)ceil(3 * sigma);
    double *w = (double *)malloc((size_t)(2 * r + 1) * sizeof(double));
    double ws = 0;
    for (int t = -r; t <= r; ++t) { w[t + r] = exp(-(double)(t * t) / (2 * sigma * sigma)); ws += w[t + r]; }
    for (int t = 0; t < 2 * r + 1; ++t) w[t] /= ws;
    int64_t dims[3] = {nx, ny, nz};
    int64_t strides[3] = {1, nx, nx * ny};
    for (int ax = 0; ax < 3; ++ax) {
        int64_t len = dims[ax], st = strides[ax];
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            int64_t c = (i / st) % len;
            double acc = 0;
            for (int t = -r; t <= r; ++t) {
                int64_t q = c + t;
                while (q < 0 || q >= len) q = q < 0 ? -q - 1 : 2 * len - q - 1; /* mirror */
                acc += w[t + r] * (double)a[i + (q - c) * st];
            }
            b[i] = (float)acc;
        }
        float *t = a; a = b; b = t;
    }
    /* plane partial sums combined in a fixed order: independent of threads */
    double *ps1 = (double *)calloc((size_t)nz, sizeof(double));
    double *ps2 = (double *)calloc((size_t)nz, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t i = z * nx * ny; i < (z + 1) * nx * ny; ++i) {
            ps1[z] += a[i];
            ps2[z] += (double)a[i] * a[i];
        }
    double s1 = 0, s2 = 0;
    for (int64_t z = 0; z < nz; ++z) { s1 += ps1[z]; s2 += ps2[z]; }
    free(ps1); free(ps2);
    double m = s1 / (double)n, sd = sqrt(s2 / (double)n - m * m);
    if (sd <= 0) sd = 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double g = ((double)a[i] - m) / sd;
        double v = floor(mean + sd_g * g + sd_n * normal(seed, 4, (uint64_t)i) + 0.5);
        if (v < 0) v = 0;
        if (v > 65535) v = 65535;
        out[i] = (uint16_t)v;
    }
    free(a); free(b); free(w);
}

static int cmp_desc(const void *pa, const void *pb) {
    double a = *(const double *)pa, b = *(const double *)pb;
    return (a < b) - (a > b);
}

/* Target areas: dist 0 = log-uniform on [p0, p1]; dist 1 = log-normal with
 * median p0 and log-sd p1, redrawn until inside [lo, hi]. */
static double draw_area(uint64_t seed, int64_t i, int dist, double p0, double p1, double lo, double hi) {
    if (dist == 0) return exp(log(p0) + (log(p1) - log(p0)) * u01(draw(seed, 10, (uint64_t)i)));
    for (uint64_t t = 0;; ++t) {
        double a = p0 * exp(p1 * normal(seed, 11, (uint64_t)i * 64 + t));
        if ((a >= lo && a <= hi) || t == 63) return a < lo ? lo : (a > hi ? hi : a);
    }
}

/* Non-overlapping random ellipses painted largest first.  Each shape claims
 * only unclaimed pixels; a placement keeping fewer than max(min_keep,
 * target/2) pixels is rejected and retried (at most 50 times).  Labels run
 * first_label, first_label+1, ... in placement order; existing nonzero
 * pixels of `out` are never overwritten.  Returns the number placed. */
int64_t synth_ellipse_labels(uint64_t seed, int64_t ny, int64_t nx, int64_t n_target,
                             int dist, double p0, double p1, double lo, double hi,
                             double ratio_hi, double min_keep, uint32_t first_label,
                             int64_t row_lo, int64_t row_hi, uint32_t *out) {
    double *areas = (double *)malloc((size_t)(n_target > 0 ? n_target : 1) * sizeof(double));
    for (int64_t i = 0; i < n_target; ++i) areas[i] = draw_area(seed, i, dist, p0, p1, lo, hi);
    qsort(areas, (size_t)n_target, sizeof(double), cmp_desc);
    int64_t placed = 0;
    for (int64_t i = 0; i < n_target; ++i) {
        double A = areas[i];
        double keep = 0.5 * A > min_keep ? 0.5 * A : min_keep;
        for (int t = 0; t < 50; ++t) {
            uint64_t k = (uint64_t)i * 64 + (uint64_t)t;
            double r = 1.0 + (ratio_hi - 1.0) * u01(draw(seed, 12, 4 * k + 0));
            double th = M_PI * u01(draw(seed, 12, 4 * k + 1));
            double cx = u01(draw(seed, 12, 4 * k + 2)) * (double)nx;
            double cy = (double)row_lo + u01(draw(seed, 12, 4 * k + 3)) * (double)(row_hi - row_lo);
            double a = sqrt(A * r / M_PI), b = sqrt(A / (r * M_PI));
            double c = cos(th), s = sin(th);
            double ex = sqrt(a * a * c * c + b * b * s * s), ey = sqrt(a * a * s * s + b * b * c * c);
            int64_t x0 = (int64_t)floor(cx - ex), x1 = (int64_t)ceil(cx + ex);
            int64_t y0 = (int64_t)floor(cy - ey), y1 = (int64_t)ceil(cy + ey);
            if (x0 < 0) x0 = 0;
            if (y0 < 0) y0 = 0;
            if (x1 > nx - 1) x1 = nx - 1;
            if (y1 > ny - 1) y1 = ny - 1;
            int64_t cnt = 0;
            for (int pass = 0; pass < 2; ++pass) {
                for (int64_t y = y0; y <= y1; ++y)
                    for (int64_t x = x0; x <= x1; ++x) {
                        double dx = (double)x - cx, dy = (double)y - cy;
                        double u = (dx * c + dy * s) / a, v = (-dx * s + dy * c) / b;
                        if (u * u + v * v > 1.0 || out[y * nx + x] != 0) continue;
                        if (pass == 0) ++cnt;
                        else out[y * nx + x] = first_label + (uint32_t)placed;
                    }
                if (pass == 0 && (double)cnt < keep) break;
            }
            if ((double)cnt >= keep) { ++placed; break; }
        }
    }
    free(areas);
    return placed;
}

/* n_images independent ellipse masks (image k seeded seeds[k], labels from
 * 1), painted on OpenMP threads; placed counts go to placed_out[k]. */
void synth_ellipse_label_images(const uint64_t *seeds, int64_t n_images, int64_t ny, int64_t nx,
                                int64_t n_target, int dist, double p0, double p1, double lo,
                                double hi, double ratio_hi, double min_keep, uint32_t *out,
                                int64_t *placed_out) {
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < n_images; ++k)
        placed_out[k] = synth_ellipse_labels(seeds[k], ny, nx, n_target, dist, p0, p1, lo, hi,
                                             ratio_hi, min_keep, 1u, 0, ny,
                                             out + (size_t)k * (size_t)(ny * nx));
}

/* Non-overlapping random ellipsoids (volume log-uniform on [v_lo, v_hi],
 * semi-axis ratios U[1, r_hi], uniformly random rotation), painted largest
 * first with the same claim / reject rule as the ellipses.  Returns the
 * number placed; labels run 1, 2, ... */
int64_t synth_ellipsoid_labels(uint64_t seed, int64_t nz, int64_t ny, int64_t nx, int64_t n_target,
                               double v_lo, double v_hi, double r_hi, uint32_t *out) {
    double *vols = (double *)malloc((size_t)(n_target > 0 ? n_target : 1) * sizeof(double));
    for (int64_t i = 0; i < n_target; ++i) vols[i] = draw_area(seed, i, 0, v_lo, v_hi, v_lo, v_hi);
    qsort(vols, (size_t)n_target, sizeof(double), cmp_desc);
    int64_t placed = 0;
    for (int64_t i = 0; i < n_target; ++i) {
        double V = vols[i];
        for (int t = 0; t < 50; ++t) {
            uint64_t k = (uint64_t)i * 64 + (uint64_t)t;
            double r1 = 1.0 + (r_hi - 1.0) * u01(draw(seed, 13, 8 * k + 0));
            double r2 = 1.0 + (r_hi - 1.0) * u01(draw(seed, 13, 8 * k + 1));
            double a = cbrt(3.0 * V / (4.0 * M_PI * r1 * r2)), b = a * r1, cc = a * r2;
            /* uniform random rotation from a unit quaternion (Shoemake) */
            double q1 = u01(draw(seed, 13, 8 * k + 2)), q2 = u01(draw(seed, 13, 8 * k + 3));
            double q3 = u01(draw(seed, 13, 8 * k + 4));
            double qw = sqrt(1 - q1) * sin(2 * M_PI * q2), qx = sqrt(1 - q1) * cos(2 * M_PI * q2);
            double qy = sqrt(q1) * sin(2 * M_PI * q3), qz = sqrt(q1) * cos(2 * M_PI * q3);
            double R[3][3] = {
                {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qz * qw), 2 * (qx * qz + qy * qw)},
                {2 * (qx * qy + qz * qw), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qx * qw)},
                {2 * (qx * qz - qy * qw), 2 * (qy * qz + qx * qw), 1 - 2 * (qx * qx + qy * qy)}};
            double cx = u01(draw(seed, 13, 8 * k + 5)) * (double)nx;
            double cy = u01(draw(seed, 13, 8 * k + 6)) * (double)ny;
            double cz = u01(draw(seed, 13, 8 * k + 7)) * (double)nz;
            double ax[3] = {a, b, cc};
            double e[3];
            for (int d = 0; d < 3; ++d) {
                double acc = 0;
                for (int m = 0; m < 3; ++m) acc += R[d][m] * R[d][m] * ax[m] * ax[m];
                e[d] = sqrt(acc);
            }
            int64_t x0 = (int64_t)floor(cx - e[0]), x1 = (int64_t)ceil(cx + e[0]);
            int64_t y0 = (int64_t)floor(cy - e[1]), y1 = (int64_t)ceil(cy + e[1]);
            int64_t z0 = (int64_t)floor(cz - e[2]), z1 = (int64_t)ceil(cz + e[2]);
            if (x0 < 0) x0 = 0;
            if (y0 < 0) y0 = 0;
            if (z0 < 0) z0 = 0;
            if (x1 > nx - 1) x1 = nx - 1;
            if (y1 > ny - 1) y1 = ny - 1;
            if (z1 > nz - 1) z1 = nz - 1;
            int64_t cnt = 0;
            for (int pass = 0; pass < 2; ++pass) {
                for (int64_t z = z0; z <= z1; ++z)
                    for (int64_t y = y0; y <= y1; ++y)
                        for (int64_t x = x0; x <= x1; ++x) {
                            double d[3] = {(double)x - cx, (double)y - cy, (double)z - cz};
                            double s2 = 0;
                            for (int m = 0; m < 3; ++m) {
                                double u = (R[0][m] * d[0] + R[1][m] * d[1] + R[2][m] * d[2]) / ax[m];
                                s2 += u * u;
                            }
                            int64_t v = (z * ny + y) * nx + x;
                            if (s2 > 1.0 || out[v] != 0) continue;
                            if (pass == 0) ++cnt;
                            else out[v] = (uint32_t)(placed + 1);
                        }
                if (pass == 0 && (double)cnt < 0.5 * V) break;
            }
            if ((double)cnt >= 0.5 * V) { ++placed; break; }
        }
    }
    free(vols);
    return placed;
}

/* Large-region fill: label `lab` on every unclaimed pixel of rows [0, R),
 * with R the smallest row count whose fill reaches `frac` of the image.
 * Returns R. */
int64_t synth_fill_rows(int64_t ny, int64_t nx, double frac, uint32_t lab, uint32_t *out) {
    double need = frac * (double)(ny * nx);
    int64_t acc = 0, R = 0;
    while (R < ny && (double)acc < need) {
        for (int64_t x = 0; x < nx; ++x) if (out[R * nx + x] == 0) ++acc;
        ++R;
    }
    for (int64_t y = 0; y < R; ++y)
        for (int64_t x = 0; x < nx; ++x)
            if (out[y * nx + x] == 0) out[y * nx + x] = lab;
    return R;
}
