/*
 * raylens — direct inverse ray-shooting on MI355X (gfx950).
 *
 * The method is the brute-force ray-shooting of Vernardos & Fluke 2014
 * (Section 2.1): every ray of a regular image-plane grid is taken through the
 * lens equation (eq. 1) with a smooth sheet kappa_s, an external shear gamma
 * and N_* point masses,
 *
 *     y = diag(1 - gamma, 1 + gamma) x - kappa_s x - sum_k m_k (x - x_k) / |x - x_k|^2,
 *
 * with kappa_s = s * kappa (eq. 2), and counted on a pixellated source plane;
 * a pixel's magnification is its count over the count N_avg it would receive
 * without lensing (eq. 4). A map is defined by (kappa, gamma, s) plus the
 * lens positions, width and resolution (Section 3.2.1's map-table fields); its
 * outputs are the int32 ray counts per pixel and the mean count and mean
 * magnification (the map.bin / mapmeta.dat contents of Section 3.2.1).
 *
 * Conventions for every entry point
 *   - Every call returns rl_status; RL_OK is 0. No C++ exception crosses the
 *     ABI. On failure rl_last_error() gives a message (thread-local, valid
 *     until the next rl_* call on the same thread).
 *   - Every argument is validated on the host before any HIP call is made, so
 *     an invalid call fails with RL_E_INVALID even on a machine without a GPU.
 *   - "d_" pointers are device pointers (HIP device memory of the context's
 *     device); "h_" pointers are host pointers. The caller owns every buffer;
 *     the library never frees caller memory. Only the context owns memory of
 *     its own (prepared lens copies, work lists, FFT planes, and a pinned,
 *     device-mapped host buffer into which the reductions behind the calls
 *     that return host values store their partial results).
 *   - Work is enqueued on the given stream (NULL = the default stream) and is
 *     asynchronous unless stated otherwise. Buffers passed in must stay alive
 *     until the stream reaches that work.
 *   - Lengths are in Einstein radii of the mean microlens mass <M> (eq. 5);
 *     masses are in units of <M>.
 *   - Layouts: count and magnification maps are row-major p2 x p1 (x1
 *     fastest, row index = x2 pixel); per-ray outputs are row-major
 *     (row_end - row_begin) x n1 (x1 fastest).
 *   - A context is used by one host thread at a time.
 */
#ifndef RAYLENS_H
#define RAYLENS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RL_OK = 0,
    RL_E_INVALID = 1,   /* an argument failed validation */
    RL_E_NOMEM = 2,     /* a device or host allocation failed */
    RL_E_DEVICE = 3,    /* a HIP call failed (no device, launch error, ...) */
    RL_E_BUSY = 4,      /* reserved */
    RL_E_CANCELLED = 5, /* reserved */
    RL_E_OVERFLOW = 6   /* a pixel count reached INT32_MAX */
} rl_status;

/* Macro model of eq. 1-2: total convergence kappa, shear gamma (acting along
 * x1) and smooth-matter fraction s = kappa_s / kappa. kappa_* = (1 - s) kappa
 * only sets how many point lenses the caller places (eq. 3). All finite. */
typedef struct {
    double kappa;
    double gamma;
    double s;
} rl_macro;

/* Regular ray grid (Fig. 1): n1 x n2 rays at the centres of the cells of
 * [c1 - half1, c1 + half1) x [c2 - half2, c2 + half2), i.e. ray (i, j) sits at
 * x1 = (c1 - half1) + (i + 1/2) * 2 half1 / n1 and likewise for x2.
 * 0 < n1 <= 2^26, 0 < n2 <= 2^40 and n1 n2 <= 2^50; half-widths finite and
 * > 0. */
typedef struct {
    int64_t n1;
    int64_t n2;
    double c1;
    double c2;
    double half1;
    double half2;
} rl_raygrid;

/* Source-plane map window: p1 x p2 half-open pixels covering
 * [c1 - width1/2, c1 + width1/2) x [c2 - width2/2, c2 + width2/2).
 * p1, p2 > 0; widths finite and > 0. */
typedef struct {
    int32_t p1;
    int32_t p2;
    double c1;
    double c2;
    double width1;
    double width2;
} rl_window;

/* Point lenses as a device structure of arrays (the lenspos.dat content of
 * Section 3.2.1): positions x1[n], x2[n] and masses m[n] in FP64.
 * m == NULL means unit masses. n >= 0 (n == 0 is a pure sheet); with n > 0
 * x1 and x2 must be non-NULL. Masses may be zero or negative; RL_FP32_COMP
 * takes a lens with |m| < 2^-40 as massless (its terms are exactly zero).
 * The arrays are read on the device and not checked for finiteness. */
typedef struct {
    const double* x1;
    const double* x2;
    const double* m;
    int64_t n;
} rl_lenses;

typedef enum {
    /* Deflection sum in FP32 with lens coordinates rebased to per-cell
     * origins and blocked TwoSum compensation; FP64 only for the final
     * y = a x - alpha and the binning. */
    RL_FP32_COMP = 0,
    /* Everything in FP64 in the oracle's operation order (bit-identical to a
     * plain sequential FP64 evaluation of eq. 1 with no contraction). */
    RL_FP64_PLAIN = 1
} rl_precision;
/* Entry points take the precision as an int32_t holding one of these values
 * (any other value is refused with RL_E_INVALID). */

/* Map statistics (mapmeta.dat of Section 3.2.1, eq. 4). */
typedef struct {
    int64_t shot;        /* rays shot (rows x n1 over the rows given) */
    int64_t binned;      /* sum of all pixel counts */
    int64_t escaped;     /* rays outside the window or singular */
    double n_avg;        /* unlensed rays per pixel, eq. 4 */
    double mean_count;   /* <N> = binned / (p1 p2) */
    double mean_mu;      /* <mu> = <N> / N_avg */
    double mu_th;        /* 1 / ((1 - kappa)^2 - gamma^2), signed */
    int32_t max_count;   /* largest pixel count */
} rl_stats;

typedef struct rl_context rl_context;

/* Creates a context bound to HIP device `hip_device` (the "initialise the GPU
 * device" step of the driver flow in Appendix A, Fig. "gpud_flow"). No HIP
 * call is made here; the device is touched on the first call that uses it,
 * so creation never fails for want of a GPU. *out receives the context, which
 * the caller owns and releases with rl_destroy. RL_E_INVALID if out is NULL or
 * hip_device < 0; RL_E_NOMEM if the host allocation fails. */
rl_status rl_create(int32_t hip_device, rl_context** out);

/* Releases the context and the device and pinned host memory it owns (the
 * memory the driver flow of Appendix A, Fig. "gpud_flow", allocates before
 * running the kernel). Waits for the device first. NULL is accepted. */
rl_status rl_destroy(rl_context* ctx);

/* Message for the last failing call on this thread ("" if none); the
 * returned string is owned by the library and valid until the next rl_* call
 * on the same thread. (Error reporting of this interface; the paper defines
 * no error behaviour.) */
const char* rl_last_error(void);

/* Library version string. */
const char* rl_version(void);

/* N_avg of eq. 4 (rays per pixel without lensing) for a grid and window:
 * (n1 n2 / (4 half1 half2)) * (width1 / p1) * (width2 / p2). Host only. */
rl_status rl_n_avg(const rl_raygrid* grid, const rl_window* win, double* h_out);

/* Shoots ray rows [row_begin, row_end) (0 <= row_begin <= row_end <= n2)
 * through eq. 1 and ACCUMULATES them into the caller-zeroed count map
 * d_counts (int32, p2 x p1) and the escaped counter *d_escaped (int64).
 * Calling it with [0, n2) shoots one whole map; disjoint row ranges add up
 * exactly to the whole map. A ray is binned iff 0 <= (y - lo) P / W < P on
 * both axes (lo = window centre - width/2); rays outside, with a non-finite
 * position, or exactly on a lens are escaped. Asynchronous on `stream`. */
rl_status rl_shoot(rl_context* ctx, const rl_lenses* lenses, const rl_macro* macro,
                   const rl_raygrid* grid, const rl_window* win, int32_t precision,
                   int64_t row_begin, int64_t row_end,
                   int32_t* d_counts, int64_t* d_escaped, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): rl_shoot
 * with the same arguments, validation and results (bit for bit the counts
 * and escaped count rl_shoot gives with the same context), but it allocates
 * nothing, neither device, host nor pinned memory, and creates no HIP object.
 * The FP32 lens copies it stages go to one fixed array of the library per
 * GPU, RL_NOALLOC_MAX_LENSES entries of 20 bytes (2.5 MiB), which each GPU
 * the library runs on holds until the process ends; its device address is
 * looked up on the first call on that device. RL_E_INVALID if lenses->n >
 * RL_NOALLOC_MAX_LENSES. Every call on one GPU shares that array and it keeps
 * the last call's contents (each call overwrites the entries it reads before
 * reading them): calls that overlap on one GPU (other streams, threads or
 * contexts) race and must be ordered by the caller. RL_FP64_PLAIN uses no
 * staging. Asynchronous on `stream`. */
#define RL_NOALLOC_MAX_LENSES 131072
rl_status rl_shoot_noalloc(rl_context* ctx, const rl_lenses* lenses, const rl_macro* macro,
                           const rl_raygrid* grid, const rl_window* win, int32_t precision,
                           int64_t row_begin, int64_t row_end,
                           int32_t* d_counts, int64_t* d_escaped, hipStream_t stream);

/* Eq. 4: d_mu[k] = (float)((double)d_counts[k] / n_avg) for the p1 x p2
 * pixels of `win`. n_avg finite and > 0. Asynchronous. */
rl_status rl_normalise(rl_context* ctx, const int32_t* d_counts, const rl_window* win,
                       double n_avg, float* d_mu, hipStream_t stream);

/* Statistics of a finished map (rows [0, n2) shot once). Synchronises the
 * stream. Returns RL_E_OVERFLOW (with *h_out filled) if a pixel count reached
 * INT32_MAX. */
rl_status rl_stats_get(rl_context* ctx, const int32_t* d_counts, const int64_t* d_escaped,
                       const rl_macro* macro, const rl_raygrid* grid, const rl_window* win,
                       rl_stats* h_out, hipStream_t stream);

/* Parity hook for the binning step alone (the pixellated source plane of
 * Section 2.1 and Fig. 1, whose pixel counts eq. 4 turns into
 * magnifications): bins n given FP64 source-plane positions d_y1[n], d_y2[n]
 * (device, caller-owned) with the rule of rl_shoot, accumulating into the
 * caller-zeroed d_counts (int32, p2 x p1) and *d_escaped (int64). n >= 0;
 * RL_E_INVALID for n < 0 or NULL pointers (positions may be NULL when n == 0).
 * Asynchronous. */
rl_status rl_bin_positions(rl_context* ctx, const double* d_y1, const double* d_y2, int64_t n,
                           const rl_window* win, int32_t* d_counts, int64_t* d_escaped,
                           hipStream_t stream);

/* Parity hook for eq. 1 alone: writes the FP64 source-plane position of every
 * ray of rows [row_begin, row_end) to d_y1, d_y2 (row-major, (row_end -
 * row_begin) x n1 each), computed exactly as rl_shoot computes it for the
 * given precision. Asynchronous. */
rl_status rl_ray_positions(rl_context* ctx, const rl_lenses* lenses, const rl_macro* macro,
                           const rl_raygrid* grid, int32_t precision,
                           int64_t row_begin, int64_t row_end,
                           double* d_y1, double* d_y2, hipStream_t stream);

/* One map of a batch: its own lenses, macro model, grid, window, row range and
 * (caller-zeroed) outputs. Pointers inside are device pointers. */
typedef struct {
    rl_lenses lenses;
    rl_macro macro;
    rl_raygrid grid;
    rl_window win;
    int64_t row_begin;
    int64_t row_end;
    int32_t* d_counts;
    int64_t* d_escaped;
} rl_map_desc;

/* Shoots every map of h_maps[0 .. n_maps-1] (host array of descriptors) in
 * one launch per tuning class present (see rl_get_tuning; more if a class
 * needs over 2^23 workgroups), the single-GPU form of the batches of map jobs
 * that GERLUMPH submits to its job queue (Section 3.2.5, the `job' table):
 * the launch's grid is the concatenation of the maps' workgroups, heaviest
 * lens fields first, so maps of uneven lens counts and sizes share the GPU,
 * each with its class's shape, and the end of the launch is made of its
 * cheapest workgroups. Results equal per-map rl_shoot calls bit for bit. n_maps >= 0; each
 * descriptor is validated as rl_shoot validates its arguments (the message
 * names the map). Asynchronous; the descriptors are copied before return. */
rl_status rl_shoot_batch(rl_context* ctx, const rl_map_desc* h_maps, int32_t n_maps,
                         int32_t precision, hipStream_t stream);

/* Kernel shape. None of these knobs changes any result bit: they only decide
 * how rays are spread over lanes and waves and how lenses are staged.
 *   rays_x, rays_y : rays per lane along x1 and x2 (product 16: 4x4, 2x8, 8x2; or
 *                    32: 4x8, 8x4, two ray cells per wave)
 *   lens_tile      : lenses staged in LDS per pass (multiple of 256, <= 2048)
 *   waves          : waves per workgroup (1, 2 or 4)
 *   submap         : binning mode. 0 = one global atomic per binned ray; 1 = an
 *                    LDS-privatised sub-map over the bounding box of the
 *                    workgroup's binned rays; 2 = an LDS-privatised 64 x 64 sub-map
 *                    around their mean pixel. In modes 1 and 2 each touched pixel
 *                    gets one global atomic; rays outside the sub-map go global. */
typedef struct {
    int32_t rays_x;
    int32_t rays_y;
    int32_t lens_tile;
    int32_t waves;
    int32_t submap;
} rl_tuning;

/* Reads / sets the kernel shape used for `precision` and tuning class
 * `n_class`: 0 (n < 1000 lenses), 1 (n < 10000), 2 (n >= 10000) for unit
 * masses, 3, 4, 5 for the same lens counts with masses (rl_lenses.m != NULL;
 * every map of a batch uses its own class). Host only. */
rl_status rl_get_tuning(rl_context* ctx, int32_t precision, int32_t n_class,
                        rl_tuning* h_out);
rl_status rl_set_tuning(rl_context* ctx, int32_t precision, int32_t n_class,
                        const rl_tuning* h_tuning);

/* Autotuner (the "timed probes" tuning of the kernel shape; the method itself,
 * Section 2.1, fixes no shape): if cache_path names a JSON table written by
 * this library build (rl_version) for this device architecture, its shapes
 * are applied and nothing is timed. Otherwise, for each precision and tuning
 * class, probe maps are shot under the candidate shapes (rays per lane, lens
 * tile, waves, binning mode; then the batch work-item size), every shape must
 * reproduce the first one's counts exactly (else RL_E_DEVICE), and the
 * fastest is applied; the table is written to cache_path (if not NULL,
 * through a temporary file and a rename). budget_ms bounds the wall time of
 * the probing: classes not reached keep their current shapes and the table
 * records "complete": false. budget_ms == 0 only applies a cache and returns
 * RL_E_INVALID if there is none. Synchronous; uses the null stream and about
 * 50 MB of device memory, freed before return. With the environment variable
 * RL_AUTOTUNE_LOG=1 it prints one line per tuned class to stderr. */
rl_status rl_autotune(rl_context* ctx, const char* cache_path, int32_t budget_ms);

/* ------------------------------------------------------------------------
 * Magnification probability distributions (MPDs)
 * ------------------------------------------------------------------------ */

/* The full MPD of a count map before division by the pixel count (Section
 * 3.2.1, mpd.dat: the frequency of each magnification value, i.e. of each
 * count N = mu N_avg): d_hist[v] += number of pixels holding v, for
 * v < n_values - 1; pixels holding n_values - 1 or more are added to
 * d_hist[n_values - 1]. Counts must be >= 0 (as rl_shoot produces them).
 * d_hist is int64[n_values], caller-zeroed, accumulated. 1 <= n_values <= 2^31.
 * Asynchronous. */
rl_status rl_count_histogram(rl_context* ctx, const int32_t* d_counts, const rl_window* win,
                             int64_t n_values, int64_t* d_hist, hipStream_t stream);

/* Binned MPD in log10(mu / mu_ref) (Section 4: the MPD tools bin the
 * distribution into 100 to 400 bins and measure magnification against the
 * macro-magnification mu_th = 1 / ((1 - kappa)^2 - gamma^2)). The nbins equal
 * bins of [log_lo, log_hi) are turned into count thresholds in FP64,
 * T_k = (n_avg mu_ref) 10^(log_lo + k (log_hi - log_lo) / nbins), k = 0..nbins,
 * and a pixel with count N goes to bin b = #{k : T_k <= N}: d_bins[0] is the
 * underflow (zero counts included), d_bins[1 + k] holds T_k <= N < T_(k+1),
 * d_bins[nbins + 1] the overflow. d_bins is int64[nbins + 2], caller-zeroed,
 * accumulated; probabilities are d_bins / (p1 p2). n_avg, mu_ref finite > 0;
 * log_lo < log_hi finite; 1 <= nbins <= 4096. Asynchronous. */
rl_status rl_mpd(rl_context* ctx, const int32_t* d_counts, const rl_window* win, double n_avg,
                 double mu_ref, double log_lo, double log_hi, int32_t nbins, int64_t* d_bins,
                 hipStream_t stream);

/* Binned MPD of a map of real magnifications, such as a finite-source map
 * from rl_convolve (Section 3: an MPD is stored for every convolution as for
 * every map): the bins of rl_mpd with thresholds T_k = mu_ref 10^(log_lo +
 * k (log_hi - log_lo) / nbins) in FP64, and a pixel with magnification mu goes
 * to bin b = #{k : T_k <= mu} (NaN, -inf, zero and negative values to the
 * underflow d_bins[0], +inf to the overflow d_bins[nbins + 1]). d_mu is
 * double[p2 x p1]; d_bins int64[nbins + 2], caller-zeroed, accumulated.
 * mu_ref finite > 0; log_lo < log_hi finite; 1 <= nbins <= 4096. Asynchronous. */
rl_status rl_mpd_values(rl_context* ctx, const double* d_mu, const rl_window* win, double mu_ref,
                        double log_lo, double log_hi, int32_t nbins, int64_t* d_bins, hipStream_t stream);

/* Probability sums for mu < mu_lim and mu > mu_lim (Section 4, MPDs tool;
 * the two add up to one): *h_below = number of pixels with N / N_avg < mu_lim
 * (the FP64 quotient, compared in FP64; the quotient is monotone in N, so the
 * decision is taken once on the host as a count threshold), *h_above =
 * p1 p2 - *h_below. mu_lim not NaN.
 * Synchronises the stream. */
rl_status rl_probability_sums(rl_context* ctx, const int32_t* d_counts, const rl_window* win,
                              double n_avg, double mu_lim, int64_t* h_below, int64_t* h_above,
                              hipStream_t stream);

/* Mean MPD and its spread over realisations (Section 4, meanMPD tool: the MPDs
 * of maps with the same kappa, gamma, s but different lens positions): for
 * each of n_bins bins, d_mean[b] = mean over the n_maps rows of d_bins (int64,
 * row-major n_maps x n_bins) of d_bins[r][b] / n_pix, and d_std[b] the sample
 * standard deviation (0 for one map). Asynchronous. */
rl_status rl_mpd_moments(rl_context* ctx, const int64_t* d_bins, int32_t n_maps, int32_t n_bins,
                         int64_t n_pix, double* d_mean, double* d_std, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Indexed maps (Appendix B)
 * ------------------------------------------------------------------------ */

/* Converts a count map into an index file and an indexed map (Appendix B):
 * d_values[0 .. n_distinct) receives the distinct counts in ascending order,
 * and pixel p's position in that table is written with the fewest bits that
 * hold every position (bits = smallest b >= 1 with 2^b >= n_distinct) into
 * d_packed, at bits [p*bits, (p+1)*bits) of a stream of 32-bit words, least
 * significant bit first (pixels in map order, x1 fastest). Needs
 * values_capacity >= n_distinct and packed_capacity >= ceil(p1 p2 bits / 32)
 * words; with d_values or d_packed NULL only *h_n_distinct and *h_bits are
 * computed (a size query). Counts must be >= 0. Synchronises the stream. */
rl_status rl_codec_encode(rl_context* ctx, const int32_t* d_counts, const rl_window* win,
                          int32_t* d_values, int64_t values_capacity, uint32_t* d_packed,
                          int64_t packed_capacity, int64_t* h_n_distinct, int32_t* h_bits,
                          hipStream_t stream);

/* Inverse of rl_codec_encode: d_counts[p] = d_values[index of p]. A position
 * past the table (a stream the encoder did not write) decodes to -1.
 * 1 <= bits <= 32, n_distinct >= 1. Asynchronous. */
rl_status rl_codec_decode(rl_context* ctx, const uint32_t* d_packed, int32_t bits,
                          const int32_t* d_values, int64_t n_distinct, const rl_window* win,
                          int32_t* d_counts, hipStream_t stream);

/* ------------------------------------------------------------------------
 * Finite sources (Section 2.4)
 * ------------------------------------------------------------------------ */

/* Source profile shapes (Section 3.1: uniform disc, Gaussian, thin-disc power
 * law, optionally with a central hole). */
typedef enum {
    RL_PROFILE_UNIFORM = 0,    /* I = 1 for r < radius */
    RL_PROFILE_GAUSSIAN = 1,   /* I = exp(-r^2 / (2 sigma^2)), sigma = radius / 3, cut at radius */
    RL_PROFILE_POWER = 2       /* I = (max(r, radius / 100) / radius)^(-3/4) for r < radius */
} rl_profile_shape;

/* A circular source: shape, radius (where the brightness drops to zero, the
 * size of Table "components") and an optional central hole (I = 0 for
 * r < hole), both in Einstein radii like the map window. */
typedef struct {
    int32_t shape;
    double radius;
    double hole;
} rl_profile;

/* Convolution kernel of a source on the map's pixel grid (Section 2.4: the
 * profile binned in pixels of the map's pixel size, padded with zeros to the
 * map's size): pixel (i, j) around the source centre gets the mean brightness
 * over an 8 x 8 grid of sub-samples, the kernel is centred on pixel (0, 0)
 * with wrap-around (so convolution does not shift the map) and normalised to
 * unit sum (so it conserves rays). d_kernel is double[p2 x p1], overwritten.
 * The source must fit: 2 ceil(radius / pixel) + 1 <= p on both axes.
 * Asynchronous. */
rl_status rl_source_kernel(rl_context* ctx, const rl_profile* profile, const rl_window* win,
                           double* d_kernel, hipStream_t stream);

/* Largest axis of a tabulated profile accepted by rl_source_kernel_table. */
#define RL_MAX_TABLE_AXIS 16384

/* Convolution kernel of a tabulated source profile (Section 3.2, the disc
 * table: profiles are stored on a regular grid of 1000 to 3000 points per axis
 * as the x positions, the y positions, then the brightness values; read with
 * x fastest). h_x[nx], h_y[ny] and h_b[ny x nx] are HOST arrays of FP32,
 * positions in Einstein radii relative to the source centre, in any order;
 * the library copies them before it returns. Sample (x, y) lies in pixel
 * (floor(x / pix1 + 1/2), floor(y / pix2 + 1/2)), pix = width / p, taken in
 * FP64; each pixel sums its samples in a fixed order (reproducible, equal to
 * the table-order sum up to rounding), and the kernel is centred on pixel
 * (0, 0) with wrap-around and normalised to unit sum like rl_source_kernel.
 * d_kernel is double[p2 x p1], overwritten. Errors (RL_E_INVALID, nothing
 * launched): 1 <= nx, ny <= RL_MAX_TABLE_AXIS violated, a position not
 * finite, a pixel box 2 h + 1 wider than p on either axis, a brightness not
 * finite or negative, or every brightness 0. Asynchronous. */
rl_status rl_source_kernel_table(rl_context* ctx, const float* h_x, int32_t nx, const float* h_y, int32_t ny,
                                 const float* h_b, const rl_window* win, double* d_kernel,
                                 hipStream_t stream);

/* Finite-source map (Section 2.4, eq. 6): d_out = F^-1[F(M) F(K)] / n_avg, the
 * circular convolution of the count map M (int32, p2 x p1) with the kernel K
 * (double, p2 x p1, e.g. from rl_source_kernel) divided by n_avg (pass N_avg
 * for a magnification map, 1 for convolved counts), in FP64. p1 and p2 must
 * be products of 2, 3 and 5 in [2, 10240] (4096 and 10000 are). d_out is
 * double[p2 x p1]; the library holds 32 p1 p2 bytes of scratch per context
 * while it runs. Asynchronous. */
rl_status rl_convolve(rl_context* ctx, const int32_t* d_counts, const double* d_kernel,
                      const rl_window* win, double n_avg, double* d_out, hipStream_t stream);

/* One map against several kernels (Section 2.4 with the data production of
 * Section 3: each map is convolved with many disc profiles and Einstein-radius
 * scalings, and each convolved map is reduced and discarded). Computes
 * h_outs[q] = rl_convolve(d_counts, h_kernels[q]) for q < n_kernels, bit for
 * bit, with the map's own transforms done once for the batch on the
 * power-of-two path (sides 256 ... 8192 and 10000). h_kernels and h_outs are
 * host arrays of n_kernels device pointers (double[p2 x p1] each); the
 * outputs must not overlap each other, the kernels or the map (an output is
 * written before the next kernel is read; equal pointers are refused with
 * RL_E_INVALID). 1 <= n_kernels <= RL_MAX_CONVOLVE_BATCH. Scratch
 * as for rl_convolve. Asynchronous; the pointer arrays are read before
 * return. */
#define RL_MAX_CONVOLVE_BATCH 4096
rl_status rl_convolve_batch(rl_context* ctx, const int32_t* d_counts, const double* const* h_kernels,
                            int32_t n_kernels, const rl_window* win, double n_avg, double* const* h_outs,
                            hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* RAYLENS_H */
