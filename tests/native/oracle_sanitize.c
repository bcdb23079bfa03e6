/* Drives every oracle function on small, edge-case inputs. Built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py:
 * any out-of-bounds access, overflow or invalid conversion aborts the run.
 * Results are also checked against facts that hold for these inputs. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                                   \
        }                                                               \
    } while (0)

static int positions_and_shoot(void) {
    /* 3 lenses, one exactly on a ray: ray (1, 2) of a 4 x 4 grid over [-2, 2)^2 */
    const double lx1[3] = {-0.5, 1.25, -1.75}, lx2[3] = {0.5, -0.3, 1.1}, lm[3] = {1.0, 0.5, 2.0};
    double y1[16], y2[16], rmin[16];
    uint8_t sing[16];
    CHECK(oracle_ray_positions(lx1, lx2, lm, 3, 0.3, 0.2, 0.5, 4, 4, 0.0, 0.0, 2.0, 2.0, 0, 4, y1, y2,
                               sing, rmin) == 0);
    int ns = 0;
    for (int i = 0; i < 16; ++i) ns += sing[i];
    CHECK(ns == 1 && sing[2 * 4 + 1] == 1);
    int32_t counts[5 * 7];
    memset(counts, 0, sizeof counts);
    int64_t esc = 0;
    CHECK(oracle_shoot(lx1, lx2, lm, 3, 0.3, 0.2, 0.5, 4, 4, 0.0, 0.0, 2.0, 2.0, 7, 5, 0.1, -0.2, 3.0,
                       2.5, 0, 4, counts, &esc, 2) == 0);
    int64_t tot = esc;
    for (int i = 0; i < 35; ++i) tot += counts[i];
    CHECK(tot == 16 && esc >= 1);
    /* empty row range, no lenses, one ray */
    CHECK(oracle_shoot(lx1, lx2, NULL, 0, 0.0, 0.0, 0.0, 1, 1, 0.0, 0.0, 1.0, 1.0, 7, 5, 0.0, 0.0, 3.0,
                       2.5, 0, 0, counts, &esc, 1) == 0);
    CHECK(oracle_shoot(lx1, lx2, NULL, 0, 0.0, 0.0, 0.0, 1, 1, 0.0, 0.0, 1.0, 1.0, 7, 5, 0.0, 0.0, 3.0,
                       2.5, 0, 1, counts, &esc, 1) == 0);
    /* invalid arguments are refused */
    CHECK(oracle_shoot(lx1, lx2, NULL, 3, 0.0, 0.0, 0.0, 4, 4, 0.0, 0.0, 2.0, 2.0, 7, 5, 0.0, 0.0, 3.0,
                       2.5, 3, 2, counts, &esc, 1) != 0);
    CHECK(oracle_shoot(lx1, lx2, NULL, 3, 0.0, 0.0, 0.0, 4, 4, 0.0, 0.0, 2.0, 2.0, 0, 5, 0.0, 0.0, 3.0,
                       2.5, 0, 4, counts, &esc, 1) != 0);
    return 0;
}

static int binning(void) {
    const double y1[8] = {NAN, INFINITY, -INFINITY, -0.0, 1e300, -1.5, 1.4999999, 0.3};
    const double y2[8] = {0.0, 0.0, 0.0, -0.0, 0.0, 0.0, 0.9999, -1.0};
    const uint8_t sing[8] = {0, 0, 0, 0, 0, 0, 0, 1};
    int32_t counts[6 * 4];
    memset(counts, 0, sizeof counts);
    int64_t esc = 0;
    CHECK(oracle_bin(y1, y2, sing, 8, 6, 4, 0.0, 0.0, 3.0, 2.0, counts, &esc) == 0);
    int64_t tot = esc;
    for (int i = 0; i < 24; ++i) tot += counts[i];
    CHECK(tot == 8 && esc == 5);
    return 0;
}

static int statistics(void) {
    int32_t c[10] = {0, 1, 2, 3, 100, 2147483647, 7, 7, 7, 0};
    float mu[10];
    CHECK(oracle_normalise(c, 10, 3.0, mu) == 0 && mu[1] == (float)(1.0 / 3.0));
    double st[4];
    CHECK(oracle_stats(c, 10, 3.0, 0.4, 0.3, st) == 0);
    CHECK(oracle_n_avg(4, 4, 2.0, 2.0, 2, 2, 4.0, 4.0) == 4.0);
    int64_t h[4];
    CHECK(oracle_count_histogram(c, 10, 4, h) == 0 && h[0] == 2 && h[3] == 6);
    int64_t h1[1];
    CHECK(oracle_count_histogram(c, 10, 1, h1) == 0 && h1[0] == 10);
    double thr[5];
    CHECK(oracle_mpd_thresholds(3.0, 1.0, -1.0, 1.0, 4, thr) == 0 && thr[0] > 0.0);
    int64_t bins[6];
    CHECK(oracle_mpd(c, 10, thr, 4, bins) == 0);
    int64_t sum = 0;
    for (int i = 0; i < 6; ++i) sum += bins[i];
    CHECK(sum == 10);
    int64_t lo = 0, hi = 0;
    CHECK(oracle_probability_sums(c, 10, 3.0, 1.0, &lo, &hi) == 0 && lo + hi == 10);
    int32_t neg[2] = {-1, 3};
    CHECK(oracle_count_histogram(neg, 2, 4, h) != 0);
    return 0;
}

static int codec(void) {
    /* sizes that are not multiples of the word, one distinct value, the
     * largest int32, and bit widths 1 .. 32 */
    const int64_t sizes[4] = {1, 31, 33, 1000};
    for (int si = 0; si < 4; ++si) {
        const int64_t n = sizes[si];
        for (int distinct = 1; distinct <= 70000; distinct = distinct < 3 ? distinct + 1 : distinct * 37) {
            int32_t* c = malloc((size_t)n * sizeof(int32_t));
            int32_t* back = malloc((size_t)n * sizeof(int32_t));
            int32_t* values = malloc((size_t)n * sizeof(int32_t));
            uint32_t* packed = calloc((size_t)n, sizeof(uint32_t));
            if (!c || !back || !values || !packed) return 1;
            for (int64_t i = 0; i < n; ++i)
                c[i] = (int32_t)((i * 7919 + 13) % distinct) * (distinct > 60000 ? 30000 : 1);
            c[n - 1] = 2147483647;
            int64_t nd = 0;
            int32_t bits = 0;
            CHECK(oracle_codec_encode(c, n, values, &nd, &bits, packed) == 0);
            CHECK(bits >= 1 && bits <= 32 && nd >= 1 && nd <= n);
            CHECK(oracle_codec_decode(packed, n, bits, values, nd, back) == 0);
            CHECK(memcmp(c, back, (size_t)n * sizeof(int32_t)) == 0);
            free(c);
            free(back);
            free(values);
            free(packed);
        }
    }
    return 0;
}

int main(void) {
    if (positions_and_shoot() || binning() || statistics() || codec()) return 1;
    printf("oracle sanitizer run ok (%d threads)\n", oracle_max_threads());
    return 0;
}
