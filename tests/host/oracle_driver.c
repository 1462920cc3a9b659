/*
 * Runs the CPU oracle under AddressSanitizer and UBSan: a small random scene
 * through both modes (preprocess, pairs, tiled and brute-force blending) and
 * the binary64 adjoint, with the ragged image edges, empty tiles and the
 * three binning modes.  Also checks that the binary64 tiled image equals the
 * brute-force one bit for bit.  Prints "oracle sanitize ok" on success.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define REAL double
#define TYPE(name) name##_f64
#include "orc_types.h"
#undef REAL
#undef TYPE
#define REAL float
#define TYPE(name) name##_f32
#include "orc_types.h"
#undef REAL
#undef TYPE

int64_t orc_preprocess_f64(const orc_scene_f64 *, const orc_camera_f64 *, int, int, const orc_options_f64 *,
                           double *, int32_t *);
void orc_pairs_f64(const orc_scene_f64 *, int, int, const orc_options_f64 *, const double *, const int32_t *,
                   int64_t, uint32_t *, uint32_t *, int64_t *);
void orc_blend_tiled_f64(const double *, int, int, const orc_options_f64 *, const uint32_t *, const int64_t *,
                         double *, double *, uint32_t *);
void orc_blend_brute_f64(const double *, const int32_t *, int64_t, int, int, const orc_options_f64 *, double *,
                         double *, uint32_t *);
int64_t orc_preprocess_f32(const orc_scene_f32 *, const orc_camera_f32 *, int, int, const orc_options_f32 *,
                           float *, int32_t *);
void orc_pairs_f32(const orc_scene_f32 *, int, int, const orc_options_f32 *, const float *, const int32_t *,
                   int64_t, uint32_t *, uint32_t *, int64_t *);
void orc_blend_tiled_f32(const float *, int, int, const orc_options_f32 *, const uint32_t *, const int64_t *,
                         float *, float *, uint32_t *);
void orc_backward_f64(const orc_scene_f64 *, const orc_camera_f64 *, int, int, const orc_options_f64 *,
                      const double *, const int32_t *, const uint32_t *, const int64_t *, const double *, double *,
                      double *, double *, double *, double *, double *);

static uint64_t rng_state = 88172645463325252ull;
static double urand(void) /* xorshift64, uniform in [0, 1) */
{
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

static int failures = 0;
static void check(int ok, const char *what)
{
    if (!ok) {
        fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

enum { P = 400, D = 2, NK = 9, W = 45, H = 37 };

int main(void)
{
    /* planes of the scene, binary64 and binary32 copies */
    const int nplanes = 3 + 3 + 4 + 1 + 3 * NK;
    double *p64 = calloc((size_t)nplanes * P, sizeof(double));
    float *p32 = calloc((size_t)nplanes * P, sizeof(float));
    for (int g = 0; g < P; ++g) {
        double *m = p64, *ls = p64 + 3 * P, *q = p64 + 6 * P, *lg = p64 + 10 * P, *sh = p64 + 11 * P;
        m[g] = 2.0 * urand() - 1.0;
        m[P + g] = 2.0 * urand() - 1.0;
        m[2 * P + g] = 4.0 + 2.0 * urand() - 1.0;
        for (int c = 0; c < 3; ++c) ls[c * P + g] = -3.0 + 1.5 * (urand() - 0.5);
        for (int c = 0; c < 4; ++c) q[c * P + g] = urand() - 0.5;
        lg[g] = 4.0 * (urand() - 0.5);
        for (int c = 0; c < 3 * NK; ++c) sh[c * P + g] = 0.4 * (urand() - 0.5);
    }
    /* a few degenerate Gaussians: zero quaternion, NaN mean, behind the camera */
    for (int c = 0; c < 4; ++c) p64[(6 + c) * P + 5] = 0.0;
    p64[7] = NAN;
    p64[2 * P + 9] = -1.0;
    for (size_t i = 0; i < (size_t)nplanes * P; ++i) p32[i] = (float)p64[i];

    orc_scene_f64 s64 = {P, P, D, 0, p64, p64 + 3 * P, p64 + 6 * P, p64 + 10 * P, p64 + 11 * P};
    orc_scene_f32 s32 = {P, P, D, 0, p32, p32 + 3 * P, p32 + 6 * P, p32 + 10 * P, p32 + 11 * P};
    orc_camera_f64 c64;
    orc_camera_f32 c32;
    memset(&c64, 0, sizeof c64);
    memset(&c32, 0, sizeof c32);
    c64.R[0] = c64.R[4] = c64.R[8] = 1.0;
    c64.fx = c64.fy = 40.0;
    c64.cx = W / 2.0;
    c64.cy = H / 2.0;
    c64.near_z = (double)0.2f;
    c32.R[0] = c32.R[4] = c32.R[8] = 1.0f;
    c32.fx = c32.fy = 40.0f;
    c32.cx = W / 2.0f;
    c32.cy = H / 2.0f;
    c32.near_z = 0.2f;

    const int ntiles = ((W + 15) / 16) * ((H + 15) / 16);
    for (int binning = 0; binning <= 2; ++binning) {
        orc_options_f64 o64 = {1.0 / 255.0, 1e-4, 0.99, 0.3, 1.3, {0.1, 0.2, 0.3}, 1, binning};
        orc_options_f32 o32 = {1.0f / 255.0f, 1e-4f, 0.99f, 0.3f, 1.3f, {0.1f, 0.2f, 0.3f}, 1, binning};
        double *st64 = calloc((size_t)P * S_N, sizeof(double));
        float *st32 = calloc((size_t)P * S_N, sizeof(float));
        int32_t *iv64 = calloc((size_t)P * I_N, sizeof(int32_t));
        int32_t *iv32 = calloc((size_t)P * I_N, sizeof(int32_t));
        const int64_t n64 = orc_preprocess_f64(&s64, &c64, W, H, &o64, st64, iv64);
        const int64_t n32 = orc_preprocess_f32(&s32, &c32, W, H, &o32, st32, iv32);
        check(n64 > 0 && n32 > 0, "pairs emitted");
        check(!iv64[5 * I_N + I_VALID] && !iv64[7 * I_N + I_VALID] && !iv64[9 * I_N + I_VALID],
              "degenerate Gaussians culled");
        uint32_t *t64 = calloc((size_t)n64 + 1, 4), *v64 = calloc((size_t)n64 + 1, 4);
        uint32_t *t32 = calloc((size_t)n32 + 1, 4), *v32 = calloc((size_t)n32 + 1, 4);
        int64_t *r64 = calloc(2 * (size_t)ntiles, sizeof(int64_t)), *r32 = calloc(2 * (size_t)ntiles, sizeof(int64_t));
        orc_pairs_f64(&s64, W, H, &o64, st64, iv64, n64, t64, v64, r64);
        orc_pairs_f32(&s32, W, H, &o32, st32, iv32, n32, t32, v32, r32);
        double *rgb = calloc(3 * (size_t)W * H, sizeof(double)), *T = calloc((size_t)W * H, sizeof(double));
        double *rgbb = calloc(3 * (size_t)W * H, sizeof(double)), *Tb = calloc((size_t)W * H, sizeof(double));
        float *rgb32 = calloc(3 * (size_t)W * H, sizeof(float)), *T32 = calloc((size_t)W * H, sizeof(float));
        uint32_t *last = calloc((size_t)W * H, 4), *lastb = calloc((size_t)W * H, 4), *last32 = calloc((size_t)W * H, 4);
        orc_blend_tiled_f64(st64, W, H, &o64, v64, r64, rgb, T, last);
        orc_blend_brute_f64(st64, iv64, P, W, H, &o64, rgbb, Tb, lastb);
        orc_blend_tiled_f32(st32, W, H, &o32, v32, r32, rgb32, T32, last32);
        check(memcmp(rgb, rgbb, 3 * (size_t)W * H * sizeof(double)) == 0, "tiled image equals brute force");
        check(memcmp(T, Tb, (size_t)W * H * sizeof(double)) == 0, "tiled T equals brute force");
        double worst = 0.0;
        for (int i = 0; i < 3 * W * H; ++i) worst = fmax(worst, fabs(rgb[i] - (double)rgb32[i]));
        check(worst < 1e-2, "binary32 mode close to binary64");
        if (binning == 0) {
            double *dL = calloc(3 * (size_t)W * H, sizeof(double));
            for (int i = 0; i < 3 * W * H; ++i) dL[i] = urand() - 0.5;
            double *gm = calloc(3 * (size_t)P, 8), *gls = calloc(3 * (size_t)P, 8), *gq = calloc(4 * (size_t)P, 8);
            double *glg = calloc((size_t)P, 8), *gsh = calloc(3 * (size_t)NK * P, 8), *gst = calloc(9 * (size_t)P, 8);
            orc_backward_f64(&s64, &c64, W, H, &o64, st64, iv64, v64, r64, dL, gm, gls, gq, glg, gsh, gst);
            int finite = 1;
            for (int i = 0; i < 3 * P; ++i) finite &= isfinite(gm[i]) && isfinite(gls[i]);
            check(finite, "finite gradients");
            free(dL), free(gm), free(gls), free(gq), free(glg), free(gsh), free(gst);
        }
        free(st64), free(st32), free(iv64), free(iv32), free(t64), free(v64), free(t32), free(v32);
        free(r64), free(r32), free(rgb), free(T), free(rgbb), free(Tb), free(rgb32), free(T32);
        free(last), free(lastb), free(last32);
    }
    free(p64);
    free(p32);
    if (failures) {
        fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    printf("oracle sanitize ok\n");
    return 0;
}
