/*
 * Plain FP64 CPU oracle for direct inverse ray-shooting.
 *
 * Vernardos & Fluke 2014, Section 2.1: rays on a regular image-plane grid are
 * deflected by N_* point masses plus a smooth sheet kappa_s and an external
 * shear gamma (eq. 1), then counted on a pixellated source plane; a pixel's
 * magnification is its ray count over the count expected without lensing
 * (eq. 4). The smooth fraction s = kappa_s / kappa (eq. 2) defines kappa_s.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark. It is deliberately the slow, obvious
 * form: one ray at a time, lenses summed in input order, FP64 throughout,
 * compiled with -ffp-contract=off and without fast-math so that every
 * operation is a single IEEE-754 double operation.
 *
 * Readings of points the paper leaves open (all listed with their reasons in
 * the design notes of the repository):
 *   - rays sit at cell centres: x = (c - h) + (i + 1/2) * (2h / n);
 *   - the shear acts along x1 (the diagonal matrix of eq. 1);
 *   - pixels are half-open [lo, lo + W/P); rays outside the window, rays with a
 *     non-finite position and rays that hit a lens exactly (r^2 == 0, where
 *     eq. 1 is singular) are counted as escaped;
 *   - N_avg is the unlensed ray density times the pixel area.
 */
#include "oracle.h"

#include <math.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

static int grid_ok(int64_t n1, int64_t n2, double h1, double h2) {
    return n1 > 0 && n2 > 0 && isfinite(h1) && isfinite(h2) && h1 > 0.0 && h2 > 0.0;
}

static int window_ok(int32_t p1, int32_t p2, double w1, double w2, double W1, double W2) {
    return p1 > 0 && p2 > 0 && isfinite(w1) && isfinite(w2) && isfinite(W1) && isfinite(W2) &&
           W1 > 0.0 && W2 > 0.0;
}

/* One ray through eq. 1 (Section 2.1): the deflection is the sum over lenses of
 * m_k (x - x_k) / |x - x_k|^2, taken in input order; the macro part is
 * diag(1 - gamma, 1 + gamma) x - kappa_s x. */
static void shoot_one(const double* lx1, const double* lx2, const double* lm, int64_t n_lens,
                      double a1, double a2, double x1, double x2,
                      double* y1, double* y2, int* singular, double* rmin) {
    double alpha1 = 0.0;
    double alpha2 = 0.0;
    double r2min = INFINITY;
    int sing = 0;
    for (int64_t k = 0; k < n_lens; ++k) {
        const double d1 = x1 - lx1[k];
        const double d2 = x2 - lx2[k];
        const double r2 = d1 * d1 + d2 * d2;
        if (r2 == 0.0) sing = 1;
        if (r2 < r2min) r2min = r2;
        const double m = lm ? lm[k] : 1.0;
        const double q = m / r2;
        alpha1 = alpha1 + q * d1;
        alpha2 = alpha2 + q * d2;
    }
    *y1 = a1 * x1 - alpha1;
    *y2 = a2 * x2 - alpha2;
    *singular = sing;
    if (rmin) *rmin = sqrt(r2min);
}

/* Pixel of a source-plane position, or -1 when the ray escapes the window.
 * u = (y - lo) * P / W per axis; binned iff 0 <= u < P on both axes (NaN fails
 * every comparison, so non-finite positions escape). Truncation equals floor
 * because u >= 0 here. */
static int64_t pixel_of(double y1, double y2, int32_t p1, int32_t p2,
                        double lo1, double lo2, double inv1, double inv2) {
    const double u1 = (y1 - lo1) * inv1;
    const double u2 = (y2 - lo2) * inv2;
    if (!(u1 >= 0.0 && u1 < (double)p1)) return -1;
    if (!(u2 >= 0.0 && u2 < (double)p2)) return -1;
    const int64_t ix = (int64_t)u1;
    const int64_t iy = (int64_t)u2;
    return iy * (int64_t)p1 + ix;
}

int oracle_max_threads(void) { return omp_get_max_threads(); }

int oracle_ray_positions(const double* lx1, const double* lx2, const double* lm, int64_t n_lens,
                         double kappa, double gamma, double s,
                         int64_t n1, int64_t n2, double c1, double c2, double h1, double h2,
                         int64_t row_begin, int64_t row_end,
                         double* y1, double* y2, uint8_t* singular, double* rmin) {
    if (!grid_ok(n1, n2, h1, h2) || n_lens < 0) return -1;
    if (!isfinite(kappa) || !isfinite(gamma) || !isfinite(s) || !isfinite(c1) || !isfinite(c2)) return -1;
    if (row_begin < 0 || row_end < row_begin || row_end > n2) return -1;
    if (n_lens > 0 && (!lx1 || !lx2)) return -1;
    if (!y1 || !y2 || !singular) return -1;

    const double kappa_s = s * kappa;                /* eq. 2 */
    const double a1 = (1.0 - gamma) - kappa_s;       /* eq. 1, x1 diagonal */
    const double a2 = (1.0 + gamma) - kappa_s;       /* eq. 1, x2 diagonal */
    const double d1 = (2.0 * h1) / (double)n1;
    const double d2 = (2.0 * h2) / (double)n2;
    const double base1 = c1 - h1;
    const double base2 = c2 - h2;

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t j = row_begin; j < row_end; ++j) {
        const double x2 = base2 + ((double)j + 0.5) * d2;
        for (int64_t i = 0; i < n1; ++i) {
            const double x1 = base1 + ((double)i + 0.5) * d1;
            const int64_t o = (j - row_begin) * n1 + i;
            int sing = 0;
            shoot_one(lx1, lx2, lm, n_lens, a1, a2, x1, x2, &y1[o], &y2[o], &sing,
                      rmin ? &rmin[o] : NULL);
            singular[o] = (uint8_t)sing;
        }
    }
    return 0;
}

int oracle_bin(const double* y1, const double* y2, const uint8_t* singular, int64_t n,
               int32_t p1, int32_t p2, double w1, double w2, double W1, double W2,
               int32_t* counts, int64_t* escaped) {
    if (n < 0 || !window_ok(p1, p2, w1, w2, W1, W2)) return -1;
    if (n > 0 && (!y1 || !y2)) return -1;
    if (!counts || !escaped) return -1;
    const double lo1 = w1 - 0.5 * W1;
    const double lo2 = w2 - 0.5 * W2;
    const double inv1 = (double)p1 / W1;
    const double inv2 = (double)p2 / W2;
    int64_t esc = 0;
    for (int64_t k = 0; k < n; ++k) {
        const int64_t pix = (singular && singular[k]) ? -1
                          : pixel_of(y1[k], y2[k], p1, p2, lo1, lo2, inv1, inv2);
        if (pix < 0) esc += 1;
        else counts[pix] += 1;
    }
    *escaped += esc;
    return 0;
}

int oracle_shoot(const double* lx1, const double* lx2, const double* lm, int64_t n_lens,
                 double kappa, double gamma, double s,
                 int64_t n1, int64_t n2, double c1, double c2, double h1, double h2,
                 int32_t p1, int32_t p2, double w1, double w2, double W1, double W2,
                 int64_t row_begin, int64_t row_end,
                 int32_t* counts, int64_t* escaped, int nthreads) {
    if (!grid_ok(n1, n2, h1, h2) || n_lens < 0) return -1;
    if (!window_ok(p1, p2, w1, w2, W1, W2)) return -1;
    if (!isfinite(kappa) || !isfinite(gamma) || !isfinite(s) || !isfinite(c1) || !isfinite(c2)) return -1;
    if (row_begin < 0 || row_end < row_begin || row_end > n2) return -1;
    if (n_lens > 0 && (!lx1 || !lx2)) return -1;
    if (!counts || !escaped) return -1;

    const double kappa_s = s * kappa;
    const double a1 = (1.0 - gamma) - kappa_s;
    const double a2 = (1.0 + gamma) - kappa_s;
    const double d1 = (2.0 * h1) / (double)n1;
    const double d2 = (2.0 * h2) / (double)n2;
    const double base1 = c1 - h1;
    const double base2 = c2 - h2;
    const double lo1 = w1 - 0.5 * W1;
    const double lo2 = w2 - 0.5 * W2;
    const double inv1 = (double)p1 / W1;
    const double inv2 = (double)p2 / W2;
    if (nthreads <= 0) nthreads = omp_get_max_threads();

    int64_t esc = 0;
    /* Integer counts are order-free, so the rows can be split across threads
     * and each increment made atomically without changing the result. */
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(+ : esc)
    for (int64_t j = row_begin; j < row_end; ++j) {
        const double x2 = base2 + ((double)j + 0.5) * d2;
        for (int64_t i = 0; i < n1; ++i) {
            const double x1 = base1 + ((double)i + 0.5) * d1;
            double y1, y2;
            int sing = 0;
            shoot_one(lx1, lx2, lm, n_lens, a1, a2, x1, x2, &y1, &y2, &sing, NULL);
            const int64_t pix = sing ? -1 : pixel_of(y1, y2, p1, p2, lo1, lo2, inv1, inv2);
            if (pix < 0) {
                esc += 1;
            } else {
#pragma omp atomic
                counts[pix] += 1;
            }
        }
    }
    *escaped += esc;
    return 0;
}

/* Eq. 4's N_avg: rays per unit image-plane area times the pixel area, i.e. the
 * count a pixel receives when nothing deflects the rays. */
double oracle_n_avg(int64_t n1, int64_t n2, double h1, double h2,
                    int32_t p1, int32_t p2, double W1, double W2) {
    const double ray_density = ((double)n1 * (double)n2) / (4.0 * h1 * h2);
    const double pixel_area = (W1 / (double)p1) * (W2 / (double)p2);
    return ray_density * pixel_area;
}

/* Eq. 4: mu_ij = N_ij / N_avg. */
int oracle_normalise(const int32_t* counts, int64_t n_pix, double n_avg, float* mu) {
    if (n_pix < 0 || !(n_avg > 0.0) || !isfinite(n_avg)) return -1;
    if (n_pix > 0 && (!counts || !mu)) return -1;
    for (int64_t k = 0; k < n_pix; ++k) mu[k] = (float)((double)counts[k] / n_avg);
    return 0;
}

int oracle_stats(const int32_t* counts, int64_t n_pix, double n_avg, double kappa, double gamma,
                 double* out) {
    if (n_pix <= 0 || !counts || !out || !(n_avg > 0.0)) return -1;
    int64_t total = 0;
    for (int64_t k = 0; k < n_pix; ++k) total += counts[k];
    const double mean_count = (double)total / (double)n_pix;
    out[0] = (double)total;
    out[1] = mean_count;
    out[2] = mean_count / n_avg;
    /* macro-magnification of the smooth model (Section 4.4, used to place the
     * probability thresholds): 1 / ((1 - kappa)^2 - gamma^2). */
    out[3] = 1.0 / ((1.0 - kappa) * (1.0 - kappa) - gamma * gamma);
    return 0;
}

/* ------------------------------------------------------------------------
 * Magnification probability distributions (Section 3.2.1 and Section 4)
 * ------------------------------------------------------------------------ */

int oracle_count_histogram(const int32_t* counts, int64_t n_pix, int64_t n_values, int64_t* hist) {
    if (n_pix < 0 || n_values < 1 || !hist || (n_pix > 0 && !counts)) return -1;
    for (int64_t v = 0; v < n_values; ++v) hist[v] = 0;
    for (int64_t k = 0; k < n_pix; ++k) {
        const int64_t c = counts[k];
        if (c < 0) return -1;
        hist[c < n_values - 1 ? c : n_values - 1] += 1;
    }
    return 0;
}

int oracle_mpd_thresholds(double n_avg, double mu_ref, double log_lo, double log_hi, int32_t nbins,
                          double* thr) {
    if (!(n_avg > 0.0) || !(mu_ref > 0.0) || !isfinite(n_avg) || !isfinite(mu_ref)) return -1;
    if (!isfinite(log_lo) || !isfinite(log_hi) || !(log_hi > log_lo) || nbins < 1 || !thr) return -1;
    const double step = (log_hi - log_lo) / (double)nbins;
    const double scale = n_avg * mu_ref;
    for (int32_t k = 0; k <= nbins; ++k) thr[k] = scale * pow(10.0, log_lo + (double)k * step);
    return 0;
}

int oracle_mpd(const int32_t* counts, int64_t n_pix, const double* thr, int32_t nbins, int64_t* bins) {
    if (n_pix < 0 || nbins < 1 || !thr || !bins || (n_pix > 0 && !counts)) return -1;
    for (int32_t b = 0; b < nbins + 2; ++b) bins[b] = 0;
    for (int64_t k = 0; k < n_pix; ++k) {
        const double c = (double)counts[k];
        /* the number of thresholds at or below c picks the bin */
        int32_t b = 0;
        while (b <= nbins && thr[b] <= c) ++b;
        bins[b] += 1;
    }
    return 0;
}

/* The binned MPD of a magnification map of real values (a finite-source map,
 * Section 2.4, whose MPD is stored for every convolution as for every map,
 * Section 3): the same rule as oracle_mpd, a value goes to the bin numbered
 * by how many thresholds lie at or below it (NaN and -inf: none, bin 0). */
int oracle_mpd_values(const double* mu, int64_t n_pix, const double* thr, int32_t nbins, int64_t* bins) {
    if (n_pix < 0 || nbins < 1 || !thr || !bins || (n_pix > 0 && !mu)) return -1;
    for (int32_t b = 0; b < nbins + 2; ++b) bins[b] = 0;
    for (int64_t k = 0; k < n_pix; ++k) {
        int32_t b = 0;
        while (b <= nbins && thr[b] <= mu[k]) ++b;
        bins[b] += 1;
    }
    return 0;
}

int oracle_probability_sums(const int32_t* counts, int64_t n_pix, double n_avg, double mu_lim,
                            int64_t* below, int64_t* above) {
    if (n_pix < 0 || !(n_avg > 0.0) || !isfinite(n_avg) || isnan(mu_lim) || !below || !above) return -1;
    if (n_pix > 0 && !counts) return -1;
    int64_t lo = 0;
    for (int64_t k = 0; k < n_pix; ++k)
        if ((double)counts[k] / n_avg < mu_lim) lo += 1;
    *below = lo;
    *above = n_pix - lo;
    return 0;
}

/* ------------------------------------------------------------------------
 * Indexed-map codec (Appendix B)
 * ------------------------------------------------------------------------ */

static int cmp_i32(const void* a, const void* b) {
    const int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* position of v in the ascending table values[0..n) (v is present) */
static int64_t index_of(const int32_t* values, int64_t n, int32_t v) {
    int64_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi) / 2;
        if (values[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

int oracle_codec_encode(const int32_t* counts, int64_t n_pix, int32_t* values, int64_t* n_distinct,
                        int32_t* bits, uint32_t* packed) {
    if (n_pix < 1 || !counts || !values || !n_distinct || !bits || !packed) return -1;
    for (int64_t k = 0; k < n_pix; ++k) if (counts[k] < 0) return -1;
    /* distinct values: sort a copy, keep the first of each run */
    memcpy(values, counts, (size_t)n_pix * sizeof(int32_t));
    qsort(values, (size_t)n_pix, sizeof(int32_t), cmp_i32);
    int64_t nd = 0;
    for (int64_t k = 0; k < n_pix; ++k)
        if (k == 0 || values[k] != values[nd - 1]) values[nd++] = values[k];
    /* fewest bits b >= 1 with 2^b >= nd */
    int32_t b = 1;
    while (b < 32 && ((int64_t)1 << b) < nd) ++b;
    for (int64_t w = 0; w < n_pix; ++w) packed[w] = 0;
    for (int64_t p = 0; p < n_pix; ++p) {
        const int64_t idx = index_of(values, nd, counts[p]);
        for (int32_t t = 0; t < b; ++t) {
            if ((idx >> t) & 1) {
                const int64_t bit = p * (int64_t)b + t;
                packed[bit / 32] |= (uint32_t)1u << (bit % 32);
            }
        }
    }
    *n_distinct = nd;
    *bits = b;
    return 0;
}

int oracle_codec_decode(const uint32_t* packed, int64_t n_pix, int32_t bits, const int32_t* values,
                        int64_t n_distinct, int32_t* counts) {
    if (n_pix < 1 || bits < 1 || bits > 32 || !packed || !values || n_distinct < 1 || !counts) return -1;
    for (int64_t p = 0; p < n_pix; ++p) {
        int64_t idx = 0;
        for (int32_t t = 0; t < bits; ++t) {
            const int64_t bit = p * (int64_t)bits + t;
            if ((packed[bit / 32] >> (bit % 32)) & 1u) idx |= (int64_t)1 << t;
        }
        if (idx >= n_distinct) return -1;
        counts[p] = values[idx];
    }
    return 0;
}
