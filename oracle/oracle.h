/*
 * Plain FP64 CPU oracle for direct inverse ray-shooting (Vernardos & Fluke 2014,
 * "Adventures in the microlensing cloud", Section 2.1).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may include, link or
 * call this code: only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark use it. It shares no code, header, table or helper with the
 * HIP library; both sides implement the paper's equations independently.
 *
 * Every routine returns 0 on success and a negative value on invalid arguments.
 * All pointers are host pointers; the caller owns every buffer.
 */
#ifndef RAYSHOOT_ORACLE_H
#define RAYSHOOT_ORACLE_H
#include <stdint.h>
#ifdef __cplusplus
extern "C" {
#endif

/* Per-ray source-plane positions (eq. 1), for ray rows [row_begin, row_end).
 * Lens positions lx1/lx2 and masses lm (lm == NULL means unit masses) in units
 * of the Einstein radius of the mean mass. Rays sit at cell centres of an
 * n1 x n2 grid covering [c1-h1, c1+h1) x [c2-h2, c2+h2). Outputs are row-major,
 * x1 fastest, (row_end-row_begin)*n1 entries each. singular[k] is set to 1 when
 * the ray coincides exactly with a lens (r^2 == 0). rmin (nullable) receives the
 * distance to the nearest lens. */
int oracle_ray_positions(const double* lx1, const double* lx2, const double* lm, int64_t n_lens,
                         double kappa, double gamma, double s,
                         int64_t n1, int64_t n2, double c1, double c2, double h1, double h2,
                         int64_t row_begin, int64_t row_end,
                         double* y1, double* y2, uint8_t* singular, double* rmin);

/* Bins given source-plane positions into a p1 x p2 pixel window of widths
 * W1 x W2 centred at (w1, w2). Pixels are half-open; counts is row-major
 * (x1 fastest) and is ACCUMULATED into; *escaped is accumulated too.
 * singular may be NULL. */
int oracle_bin(const double* y1, const double* y2, const uint8_t* singular, int64_t n,
               int32_t p1, int32_t p2, double w1, double w2, double W1, double W2,
               int32_t* counts, int64_t* escaped);

/* Full shoot of rows [row_begin,row_end): eq. 1 per ray followed by binning.
 * Accumulates into counts / *escaped. nthreads <= 0 uses the OpenMP default. */
int oracle_shoot(const double* lx1, const double* lx2, const double* lm, int64_t n_lens,
                 double kappa, double gamma, double s,
                 int64_t n1, int64_t n2, double c1, double c2, double h1, double h2,
                 int32_t p1, int32_t p2, double w1, double w2, double W1, double W2,
                 int64_t row_begin, int64_t row_end,
                 int32_t* counts, int64_t* escaped, int nthreads);

/* Rays per pixel in the absence of lensing (eq. 4's N_avg). */
double oracle_n_avg(int64_t n1, int64_t n2, double h1, double h2,
                    int32_t p1, int32_t p2, double W1, double W2);

/* mu_ij = N_ij / N_avg (eq. 4), one FP64 division per pixel rounded once to float. */
int oracle_normalise(const int32_t* counts, int64_t n_pix, double n_avg, float* mu);

/* Map statistics: out[0]=binned (sum of counts), out[1]=mean count, out[2]=mean mu,
 * out[3]=theoretical macro-magnification 1/((1-kappa)^2-gamma^2). */
int oracle_stats(const int32_t* counts, int64_t n_pix, double n_avg, double kappa, double gamma,
                 double* out);

/* Magnification probability distribution (Section 3.2.1, mpd.dat: the
 * frequency of each value in the map divided by the number of pixels).
 * hist[v] counts the pixels holding v for v < n_values - 1; pixels holding
 * n_values - 1 or more are counted in hist[n_values - 1]. hist is overwritten. */
int oracle_count_histogram(const int32_t* counts, int64_t n_pix, int64_t n_values, int64_t* hist);

/* Bin edges of a histogram in log10(mu / mu_ref) over [log_lo, log_hi) with
 * nbins equal bins (Section 4: MPDs binned into 100-400 bins, magnification
 * measured against mu_th), expressed as count thresholds:
 * thr[k] = (n_avg * mu_ref) * 10^(log_lo + k (log_hi - log_lo) / nbins), k = 0..nbins. */
int oracle_mpd_thresholds(double n_avg, double mu_ref, double log_lo, double log_hi, int32_t nbins,
                          double* thr);

/* Binned MPD: bins[0] counts pixels below thr[0] (zero counts included),
 * bins[1 + k] those with thr[k] <= N < thr[k + 1], bins[nbins + 1] those at
 * or above thr[nbins]. bins (nbins + 2 entries) is overwritten. */
int oracle_mpd(const int32_t* counts, int64_t n_pix, const double* thr, int32_t nbins, int64_t* bins);
/* The same binning of real magnification values (thresholds from
 * oracle_mpd_thresholds with n_avg = 1). */
int oracle_mpd_values(const double* mu, int64_t n_pix, const double* thr, int32_t nbins, int64_t* bins);

/* Probability sums (Section 4: P(mu < mu_lim) and P(mu > mu_lim), which add
 * to one): *below counts pixels with N / N_avg < mu_lim, *above the rest. */
int oracle_probability_sums(const int32_t* counts, int64_t n_pix, double n_avg, double mu_lim,
                            int64_t* below, int64_t* above);

/* Indexed maps (Appendix B): the distinct count values of a map, ascending,
 * form the index file values[0 .. n_distinct); each pixel is replaced by the
 * position of its value, written with the fewest bits that hold every index
 * (bits = smallest b >= 1 with 2^b >= n_distinct). Pixel p's index occupies
 * bits [p*bits, (p+1)*bits) of a stream of 32-bit words, least significant
 * bit first. values must hold n_pix entries and packed n_pix words (always
 * enough: bits <= 32); the words past ceil(n_pix * bits / 32) are left zero.
 * Counts must be >= 0. */
int oracle_codec_encode(const int32_t* counts, int64_t n_pix, int32_t* values, int64_t* n_distinct,
                        int32_t* bits, uint32_t* packed);

/* Inverse of oracle_codec_encode. */
int oracle_codec_decode(const uint32_t* packed, int64_t n_pix, int32_t bits, const int32_t* values,
                        int64_t n_distinct, int32_t* counts);

int oracle_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
