/* Drives the host-side validation of every C-ABI entry point, with the
 * library's host code built under AddressSanitizer and
 * UndefinedBehaviorSanitizer (tests/test_abi_sanitize.py). No GPU is needed:
 * every call below is refused on the host before any HIP call, or touches no
 * device (context creation, N_avg, tuning table, version). */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "raylens.h"

#define EXPECT(call, st)                                                                  \
    do {                                                                                  \
        rl_status got_ = (call);                                                          \
        if (got_ != (st)) {                                                               \
            fprintf(stderr, "line %d: %s returned %d, expected %d (%s)\n", __LINE__, #call, \
                    (int)got_, (int)(st), rl_last_error());                               \
            return 1;                                                                     \
        }                                                                                 \
    } while (0)

int main(void) {
    rl_context* ctx = NULL;
    EXPECT(rl_create(-1, &ctx), RL_E_INVALID);
    EXPECT(rl_create(0, NULL), RL_E_INVALID);
    EXPECT(rl_create(0, &ctx), RL_OK);
    if (!ctx || strstr(rl_version(), "raylens") == NULL) return 1;

    double fake_d[4];
    int32_t fake_i[4];
    int64_t fake_l[4];
    uint32_t fake_u[4];
    float fake_f[4];
    const rl_lenses L = {fake_d, fake_d, NULL, 3};
    const rl_lenses Lbad = {fake_d, NULL, NULL, 3};
    const rl_macro M = {0.4, 0.3, 0.0};
    const rl_macro Mnan = {NAN, 0.3, 0.0};
    const rl_raygrid G = {16, 16, 0.0, 0.0, 1.0, 1.0};
    const rl_raygrid Gbad = {0, 16, 0.0, 0.0, 1.0, 1.0};
    const rl_window W = {8, 8, 0.0, 0.0, 2.0, 2.0};
    const rl_window Wbad = {8, 8, 0.0, 0.0, -2.0, 2.0};
    const rl_window W7 = {7, 8, 0.0, 0.0, 2.0, 2.0};

    double navg = 0.0;
    EXPECT(rl_n_avg(&G, &W, &navg), RL_OK);
    if (!(fabs(navg - 4.0) < 1e-12)) return 1;
    EXPECT(rl_n_avg(&Gbad, &W, &navg), RL_E_INVALID);
    EXPECT(rl_n_avg(&G, NULL, &navg), RL_E_INVALID);

    EXPECT(rl_shoot(NULL, &L, &M, &G, &W, RL_FP32_COMP, 0, 16, fake_i, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_shoot(ctx, &Lbad, &M, &G, &W, RL_FP32_COMP, 0, 16, fake_i, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_shoot(ctx, &L, &Mnan, &G, &W, RL_FP32_COMP, 0, 16, fake_i, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_shoot(ctx, &L, &M, &Gbad, &W, RL_FP32_COMP, 0, 16, fake_i, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_shoot(ctx, &L, &M, &G, &Wbad, RL_FP32_COMP, 0, 16, fake_i, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_shoot(ctx, &L, &M, &G, &W, (rl_precision)7, 0, 16, fake_i, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_shoot(ctx, &L, &M, &G, &W, RL_FP32_COMP, 5, 3, fake_i, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_shoot(ctx, &L, &M, &G, &W, RL_FP32_COMP, 0, 17, fake_i, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_shoot(ctx, &L, &M, &G, &W, RL_FP32_COMP, 0, 16, NULL, fake_l, NULL), RL_E_INVALID);
    {
        const rl_lenses Lbig = {fake_d, fake_d, NULL, (int64_t)RL_NOALLOC_MAX_LENSES + 1};
        EXPECT(rl_shoot_noalloc(NULL, &L, &M, &G, &W, RL_FP32_COMP, 0, 16, fake_i, fake_l, NULL), RL_E_INVALID);
        EXPECT(rl_shoot_noalloc(ctx, &Lbad, &M, &G, &W, RL_FP32_COMP, 0, 16, fake_i, fake_l, NULL), RL_E_INVALID);
        EXPECT(rl_shoot_noalloc(ctx, &L, &Mnan, &G, &W, RL_FP32_COMP, 0, 16, fake_i, fake_l, NULL), RL_E_INVALID);
        EXPECT(rl_shoot_noalloc(ctx, &L, &M, &Gbad, &W, RL_FP32_COMP, 0, 16, fake_i, fake_l, NULL), RL_E_INVALID);
        EXPECT(rl_shoot_noalloc(ctx, &L, &M, &G, &Wbad, RL_FP32_COMP, 0, 16, fake_i, fake_l, NULL), RL_E_INVALID);
        EXPECT(rl_shoot_noalloc(ctx, &L, &M, &G, &W, 7, 0, 16, fake_i, fake_l, NULL), RL_E_INVALID);
        EXPECT(rl_shoot_noalloc(ctx, &L, &M, &G, &W, RL_FP32_COMP, 5, 3, fake_i, fake_l, NULL), RL_E_INVALID);
        EXPECT(rl_shoot_noalloc(ctx, &L, &M, &G, &W, RL_FP32_COMP, 0, 16, fake_i, NULL, NULL), RL_E_INVALID);
        EXPECT(rl_shoot_noalloc(ctx, &Lbig, &M, &G, &W, RL_FP32_COMP, 0, 16, fake_i, fake_l, NULL), RL_E_INVALID);
    }
    EXPECT(rl_ray_positions(ctx, &L, &M, &G, RL_FP64_PLAIN, 0, 17, fake_d, fake_d, NULL), RL_E_INVALID);
    EXPECT(rl_ray_positions(ctx, &L, &M, &G, RL_FP64_PLAIN, 0, 1, NULL, fake_d, NULL), RL_E_INVALID);
    EXPECT(rl_normalise(ctx, fake_i, &W, 0.0, fake_f, NULL), RL_E_INVALID);
    EXPECT(rl_normalise(ctx, fake_i, &W, INFINITY, fake_f, NULL), RL_E_INVALID);
    EXPECT(rl_normalise(ctx, NULL, &W, 1.0, fake_f, NULL), RL_E_INVALID);
    rl_stats st;
    EXPECT(rl_stats_get(ctx, fake_i, fake_l, &M, &G, &W, NULL, NULL), RL_E_INVALID);
    EXPECT(rl_stats_get(ctx, NULL, fake_l, &M, &G, &W, &st, NULL), RL_E_INVALID);
    EXPECT(rl_bin_positions(ctx, fake_d, fake_d, -1, &W, fake_i, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_bin_positions(ctx, fake_d, NULL, 4, &W, fake_i, fake_l, NULL), RL_E_INVALID);

    rl_map_desc maps[2];
    memset(maps, 0, sizeof maps);
    maps[0] = (rl_map_desc){L, M, G, W, 0, 16, fake_i, fake_l};
    maps[1] = (rl_map_desc){L, M, Gbad, W, 0, 16, fake_i, fake_l};
    EXPECT(rl_shoot_batch(ctx, maps, 2, RL_FP32_COMP, NULL), RL_E_INVALID);
    EXPECT(rl_shoot_batch(ctx, NULL, 2, RL_FP32_COMP, NULL), RL_E_INVALID);
    EXPECT(rl_shoot_batch(ctx, maps, -1, RL_FP32_COMP, NULL), RL_E_INVALID);
    EXPECT(rl_shoot_batch(ctx, maps, 0, RL_FP32_COMP, NULL), RL_OK);

    rl_tuning t;
    EXPECT(rl_get_tuning(ctx, RL_FP32_COMP, 1, &t), RL_OK);
    EXPECT(rl_get_tuning(ctx, RL_FP32_COMP, 6, &t), RL_E_INVALID);
    t.lens_tile = 100;
    EXPECT(rl_set_tuning(ctx, RL_FP32_COMP, 1, &t), RL_E_INVALID);
    t = (rl_tuning){4, 8, 512, 2, 2, 8};
    EXPECT(rl_set_tuning(ctx, RL_FP32_COMP, 4, &t), RL_OK);
    EXPECT(rl_set_tuning(ctx, RL_FP64_PLAIN, 4, &t), RL_E_INVALID);
    EXPECT(rl_autotune(NULL, NULL, 0), RL_E_INVALID);
    EXPECT(rl_autotune(ctx, NULL, -5), RL_E_INVALID);

    EXPECT(rl_count_histogram(ctx, fake_i, &W, 0, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_count_histogram(ctx, fake_i, &W, 4, NULL, NULL), RL_E_INVALID);
    EXPECT(rl_mpd(ctx, fake_i, &W, 1.0, 1.0, 1.0, -1.0, 10, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_mpd(ctx, fake_i, &W, 1.0, 1.0, -1.0, 1.0, 0, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_mpd(ctx, fake_i, &W, 1.0, 1.0, -1.0, 1.0, 5000, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_mpd_values(ctx, fake_d, &W, 1.0, 1.0, -1.0, 10, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_mpd_values(ctx, fake_d, &W, NAN, -1.0, 1.0, 10, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_mpd_values(ctx, fake_d, &W, 1.0, -1.0, 1.0, 0, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_mpd_values(ctx, NULL, &W, 1.0, -1.0, 1.0, 10, fake_l, NULL), RL_E_INVALID);
    EXPECT(rl_mpd(ctx, fake_i, &W, -1.0, 1.0, -1.0, 1.0, 10, fake_l, NULL), RL_E_INVALID);
    int64_t lo = 0, hi = 0;
    EXPECT(rl_probability_sums(ctx, fake_i, &W, 1.0, 1.0, NULL, &hi, NULL), RL_E_INVALID);
    EXPECT(rl_probability_sums(ctx, fake_i, &W, NAN, 1.0, &lo, &hi, NULL), RL_E_INVALID);
    EXPECT(rl_mpd_moments(ctx, fake_l, 0, 4, 10, fake_d, fake_d, NULL), RL_E_INVALID);
    EXPECT(rl_mpd_moments(ctx, NULL, 2, 4, 10, fake_d, fake_d, NULL), RL_E_INVALID);
    int64_t nd = 0;
    int32_t bits = 0;
    EXPECT(rl_codec_encode(ctx, NULL, &W, fake_i, 4, fake_u, 4, &nd, &bits, NULL), RL_E_INVALID);
    EXPECT(rl_codec_encode(ctx, fake_i, &W, fake_i, 4, fake_u, 4, NULL, &bits, NULL), RL_E_INVALID);
    EXPECT(rl_codec_decode(ctx, fake_u, 0, fake_i, 4, &W, fake_i, NULL), RL_E_INVALID);
    EXPECT(rl_codec_decode(ctx, fake_u, 33, fake_i, 4, &W, fake_i, NULL), RL_E_INVALID);
    EXPECT(rl_codec_decode(ctx, fake_u, 4, fake_i, 0, &W, fake_i, NULL), RL_E_INVALID);

    const rl_profile P = {RL_PROFILE_GAUSSIAN, 0.3, 0.0};
    const rl_profile Pbad = {9, 0.3, 0.0};
    const rl_profile Pbig = {RL_PROFILE_UNIFORM, 5.0, 0.0};
    EXPECT(rl_source_kernel(ctx, &Pbad, &W, fake_d, NULL), RL_E_INVALID);
    EXPECT(rl_source_kernel(ctx, &Pbig, &W, fake_d, NULL), RL_E_INVALID);
    EXPECT(rl_source_kernel(ctx, &P, &W, NULL, NULL), RL_E_INVALID);
    EXPECT(rl_convolve(ctx, fake_i, fake_d, &W7, 1.0, fake_d, NULL), RL_E_INVALID);
    EXPECT(rl_convolve(ctx, fake_i, fake_d, &W, 0.0, fake_d, NULL), RL_E_INVALID);
    EXPECT(rl_convolve(ctx, fake_i, NULL, &W, 1.0, fake_d, NULL), RL_E_INVALID);
    const double* ks[3] = {fake_d, fake_d + 1, fake_d + 2};
    double* outs[3] = {fake_d + 3, fake_d + 1, fake_d + 3};
    EXPECT(rl_convolve_batch(ctx, fake_i, ks, 0, &W, 1.0, outs, NULL), RL_E_INVALID);
    EXPECT(rl_convolve_batch(ctx, fake_i, ks, RL_MAX_CONVOLVE_BATCH + 1, &W, 1.0, outs, NULL), RL_E_INVALID);
    EXPECT(rl_convolve_batch(ctx, fake_i, ks, 3, &W, 1.0, outs, NULL), RL_E_INVALID); /* outputs alias */

    /* tabulated profiles: the host loops over the tables (positions far out of
     * int range, NaN, negative or all-zero brightness) */
    const float tx[3] = {-0.1f, 0.0f, 0.1f};
    const float tfar[3] = {-0.1f, 3.0e38f, 0.1f};
    const float tnan[3] = {-0.1f, NAN, 0.1f};
    const float tb[9] = {1, 1, 1, 1, 1, 1, 1, 1, 1};
    const float tneg[9] = {1, 1, 1, 1, -1, 1, 1, 1, 1};
    const float tzero[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    EXPECT(rl_source_kernel_table(ctx, tx, 0, tx, 3, tb, &W, fake_d, NULL), RL_E_INVALID);
    EXPECT(rl_source_kernel_table(ctx, tx, 3, tx, RL_MAX_TABLE_AXIS + 1, tb, &W, fake_d, NULL), RL_E_INVALID);
    EXPECT(rl_source_kernel_table(ctx, tfar, 3, tx, 3, tb, &W, fake_d, NULL), RL_E_INVALID);
    EXPECT(rl_source_kernel_table(ctx, tx, 3, tnan, 3, tb, &W, fake_d, NULL), RL_E_INVALID);
    EXPECT(rl_source_kernel_table(ctx, tx, 3, tx, 3, tneg, &W, fake_d, NULL), RL_E_INVALID);
    EXPECT(rl_source_kernel_table(ctx, tx, 3, tx, 3, tzero, &W, fake_d, NULL), RL_E_INVALID);
    EXPECT(rl_source_kernel_table(ctx, tx, 3, tx, 3, tb, &W, NULL, NULL), RL_E_INVALID);

    if (rl_last_error()[0] == '\0') return 1;
    EXPECT(rl_destroy(ctx), RL_OK);
    EXPECT(rl_destroy(NULL), RL_OK);
    printf("abi sanitizer run ok\n");
    return 0;
}
