/*
 * FlashGS rasterizer oracle: a plain, slow CPU implementation of what the
 * rendering path computes, written from the paper (FlashGS, arXiv 2408.07967).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  The product library never
 * links, loads or calls it, and the two share no code, header or table.
 *
 * This file is compiled twice:
 *   -DORC_FP64  every quantity is binary64 and exp/log come from libm.  This
 *               is the plain definition the images are judged against.
 *   -DORC_FP32  every quantity is binary32; each + - * / sqrt written below is
 *               one correctly rounded binary32 operation in the written order
 *               (built with -ffp-contract=off, SSE arithmetic, no fast-math),
 *               and exp / log are the canonical binary64 routines of
 *               orc_math.c rounded once.  This is the reference for the
 *               bit-exact comparison of per-Gaussian state, Gaussian-tile pairs
 *               and sorted order.
 *
 * Steps (the paper's order, Alg. 1 and Alg. 4):
 *   activations -> view transform -> near-plane and opacity cull (Alg. 4) ->
 *   pinhole projection (project + ndc2Pix) -> 3D covariance (computeCov3D) ->
 *   EWA 2D covariance (computeCov2D) -> conic -> opacity-aware extent (Eq. 1-3)
 *   -> tight axis-aligned box tangent to the ellipse (Sec. 4.1) -> exact
 *   ellipse/tile test (Alg. 3 with the division-free form of Eq. 7) ->
 *   SH colour for surviving Gaussians (Alg. 4) -> key (tile | depth), value
 *   (Gaussian index) -> sort (Sec. 2.2) -> per-tile front-to-back blending
 *   with early termination (Sec. 2.2, Sec. 5.2).
 *
 * Readings where the paper is silent (scale/rotation parameterisation, the
 * 0.3 px^2 low-pass dilation, the Jacobian clamp, the per-pixel contribution
 * rule q <= k^2, the 0.99 alpha clamp, the termination order, the pixel
 * sample at (i+1/2, j+1/2), the garbled Eq. 4 / Eq. 5 and the missing
 * discriminant guard in Eq. 7) are listed with their reasons in the project's
 * design notes; each is marked "reading" where it is used below.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#if defined(ORC_FP32)
typedef float REAL;
#define FN(name) name##_f32
#define TYPE(name) name##_f32
double orc_exp_d(double x);
double orc_log_d(double x);
#define R_EXP(x) ((float)orc_exp_d((double)(x)))
/* logistic function evaluated in binary64 and rounded once */
#define R_SIGMOID(x) ((float)(1.0 / (1.0 + orc_exp_d(-(double)(x)))))
/* 2 ln(o / tau) in binary64, optionally capped at 9 (3 sigma), rounded once */
#define R_EXTENT(o, tau, cap) orc_extent_f32((o), (tau), (cap))
static float orc_extent_f32(float o, float tau, int cap)
{
    double k2 = 2.0 * orc_log_d((double)o / (double)tau);
    if (cap && k2 > 9.0) k2 = 9.0;
    return (float)k2;
}
#define R_SQRT(x) sqrtf(x)
#define R_CEIL(x) ceilf(x)
#define R_FLOOR(x) floorf(x)
#define R_ISFINITE(x) isfinite(x)
#elif defined(ORC_FP64)
typedef double REAL;
#define FN(name) name##_f64
#define TYPE(name) name##_f64
#define R_EXP(x) exp(x)
#define R_SIGMOID(x) (1.0 / (1.0 + exp(-(x))))
static double orc_extent_f64(double o, double tau, int cap)
{
    double k2 = 2.0 * log(o / tau);
    if (cap && k2 > 9.0) k2 = 9.0;
    return k2;
}
#define R_EXTENT(o, tau, cap) orc_extent_f64((o), (tau), (cap))
#define R_SQRT(x) sqrt(x)
#define R_CEIL(x) ceil(x)
#define R_FLOOR(x) floor(x)
#define R_ISFINITE(x) isfinite(x)
#else
#error "define ORC_FP32 or ORC_FP64"
#endif

#define TILE 16

#include "orc_types.h"

/* Real spherical harmonics, orthonormal, with the Condon-Shortley phase,
 * index k = l^2 + l + m, evaluated at the unit direction (x, y, z).
 * Y_lm = sqrt(2) K_l^|m| P_l^|m|(z) cos(m phi)    (m > 0)
 *      = K_l^0 P_l^0(z)                             (m = 0)
 *      = sqrt(2) K_l^|m| P_l^|m|(z) sin(|m| phi)   (m < 0)
 * K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).  The polynomial forms below are
 * those expressions multiplied out (reading: the paper names
 * computeColorFromSH only). */
static void FN(orc_sh_basis)(REAL x, REAL y, REAL z, REAL *Y)
{
    const double pi = 3.14159265358979323846;
    const double k00 = sqrt(1.0 / (4.0 * pi));
    const double k1 = sqrt(3.0 / (4.0 * pi));
    const double k2a = sqrt(15.0 / (4.0 * pi));  /* |m| = 1, 2 (xy form) */
    const double k20 = sqrt(5.0 / (16.0 * pi));
    const double k22 = sqrt(15.0 / (16.0 * pi));
    const double k33 = sqrt(35.0 / (32.0 * pi));
    const double k32 = sqrt(105.0 / (4.0 * pi));
    const double k31 = sqrt(21.0 / (32.0 * pi));
    const double k30 = sqrt(7.0 / (16.0 * pi));
    const double k32b = sqrt(105.0 / (16.0 * pi));
    REAL xx = x * x, yy = y * y, zz = z * z;
    Y[0] = (REAL)k00;
    Y[1] = -(REAL)k1 * y;
    Y[2] = (REAL)k1 * z;
    Y[3] = -(REAL)k1 * x;
    Y[4] = (REAL)k2a * (x * y);
    Y[5] = -(REAL)k2a * (y * z);
    Y[6] = (REAL)k20 * ((REAL)3 * zz - (REAL)1);
    Y[7] = -(REAL)k2a * (x * z);
    Y[8] = (REAL)k22 * (xx - yy);
    Y[9] = -(REAL)k33 * (y * ((REAL)3 * xx - yy));
    Y[10] = (REAL)k32 * (x * y * z);
    Y[11] = -(REAL)k31 * (y * ((REAL)5 * zz - (REAL)1));
    Y[12] = (REAL)k30 * (z * ((REAL)5 * zz - (REAL)3));
    Y[13] = -(REAL)k31 * (x * ((REAL)5 * zz - (REAL)1));
    Y[14] = (REAL)k32b * (z * (xx - yy));
    Y[15] = -(REAL)k33 * (x * (xx - (REAL)3 * yy));
}

/* Exact ellipse / tile test (Alg. 3; the division- and square-root-free
 * chord-overlap condition of Eq. 7).
 *
 * The rectangle is the tile's pixel-sample hull, [16 tx + 1/2, min(16 tx + 16,
 * W) - 1/2] x (same in y) (reading: every pixel sample of the tile lies in
 * it, so the test stays exact for the per-pixel rule).  The ellipse is
 * E = { d : A dx^2 + 2 B dx dy + C dy^2 <= k^2 }, d relative to the 2D mean.
 *
 * Centre inside the rectangle -> hit.  Otherwise, for each edge line, the
 * line meets E in a chord [r-, r+] (roots of a quadratic a X^2 + b X + c = 0
 * with a = A or C > 0) and the tile is hit iff the chord overlaps the edge
 * segment [lo, hi]:  lo <= r+ and hi >= r-  (Eq. 4 / Eq. 5 with the garbled
 * indices read as max(a_i, a_j) and a_j <= b_i).  With e1 = 2 a lo + b and
 * e2 = 2 a hi + b this is (e1 <= 0 or e1^2 <= Delta) and (e2 >= 0 or
 * e2^2 <= Delta), Delta = b^2 - 4 a c (Eq. 7), guarded by Delta >= 0 (the
 * line must meet E at all; Eq. 7 omits the guard, Alg. 3 states it). */
static int FN(orc_tile_hit)(const REAL *s, int tx, int ty, int W, int H)
{
    REAL u = s[S_U], v = s[S_V], A = s[S_A], B = s[S_B], C = s[S_C], k2 = s[S_K2];
    int xe = TILE * tx + TILE; if (xe > W) xe = W;
    int ye = TILE * ty + TILE; if (ye > H) ye = H;
    REAL x0 = ((REAL)(TILE * tx) + (REAL)0.5) - u;
    REAL x1 = ((REAL)xe - (REAL)0.5) - u;
    REAL y0 = ((REAL)(TILE * ty) + (REAL)0.5) - v;
    REAL y1 = ((REAL)ye - (REAL)0.5) - v;
    if (x0 <= (REAL)0 && (REAL)0 <= x1 && y0 <= (REAL)0 && (REAL)0 <= y1) return 1;
    /* horizontal edges y = y0, y = y1: A x^2 + (2 B y) x + (C y^2 - k^2) = 0 */
    for (int e = 0; e < 2; ++e) {
        REAL ye_ = e ? y1 : y0;
        REAL bq = ((REAL)2 * B) * ye_;
        REAL cq = (C * ye_) * ye_ - k2;
        REAL delta = bq * bq - ((REAL)4 * A) * cq;
        if (delta >= (REAL)0) {
            REAL e1 = ((REAL)2 * A) * x0 + bq;
            REAL e2 = ((REAL)2 * A) * x1 + bq;
            if ((e1 <= (REAL)0 || e1 * e1 <= delta) && (e2 >= (REAL)0 || e2 * e2 <= delta)) return 1;
        }
    }
    /* vertical edges x = x0, x = x1: C y^2 + (2 B x) y + (A x^2 - k^2) = 0 */
    for (int e = 0; e < 2; ++e) {
        REAL xe2 = e ? x1 : x0;
        REAL bq = ((REAL)2 * B) * xe2;
        REAL cq = (A * xe2) * xe2 - k2;
        REAL delta = bq * bq - ((REAL)4 * C) * cq;
        if (delta >= (REAL)0) {
            REAL e1 = ((REAL)2 * C) * y0 + bq;
            REAL e2 = ((REAL)2 * C) * y1 + bq;
            if ((e1 <= (REAL)0 || e1 * e1 <= delta) && (e2 >= (REAL)0 || e2 * e2 <= delta)) return 1;
        }
    }
    return 0;
}

int FN(orc_tile_hit_api)(const REAL *state16, int tx, int ty, int W, int H)
{
    return FN(orc_tile_hit)(state16, tx, ty, W, H);
}

static REAL FN(orc_clamp)(REAL x, REAL lo, REAL hi)
{
    return x < lo ? lo : (x > hi ? hi : x);
}

/* Per-Gaussian preprocessing of one Gaussian g (Alg. 4, first half, plus the
 * colour of its last step).  Writes S_N reals and I_N ints; returns validity. */
static int FN(orc_gauss)(const TYPE(orc_scene) *sc, int64_t g, const TYPE(orc_camera) *cam,
                         int W, int H, const TYPE(orc_options) *op, REAL *s, int32_t *iv)
{
    memset(s, 0, sizeof(REAL) * S_N);
    memset(iv, 0, sizeof(int32_t) * I_N);
    const int64_t st = sc->stride;
    REAL mx = sc->means[g], my = sc->means[st + g], mz = sc->means[2 * st + g];
    REAL ls0 = sc->log_scales[g], ls1 = sc->log_scales[st + g], ls2 = sc->log_scales[2 * st + g];
    REAL qw = sc->quats[g], qx = sc->quats[st + g], qy = sc->quats[2 * st + g], qz = sc->quats[3 * st + g];
    REAL logit = sc->logits[g];
    if (!(R_ISFINITE(mx) && R_ISFINITE(my) && R_ISFINITE(mz) && R_ISFINITE(ls0) && R_ISFINITE(ls1) &&
          R_ISFINITE(ls2) && R_ISFINITE(qw) && R_ISFINITE(qx) && R_ISFINITE(qy) && R_ISFINITE(qz) &&
          R_ISFINITE(logit)))
        return 0;
    const REAL *R = cam->R;
    /* view transform (p_view of Alg. 1 / Alg. 4) */
    REAL tx = ((R[0] * mx + R[1] * my) + R[2] * mz) + cam->t[0];
    REAL ty = ((R[3] * mx + R[4] * my) + R[5] * mz) + cam->t[1];
    REAL tz = ((R[6] * mx + R[7] * my) + R[8] * mz) + cam->t[2];
    /* near plane (Alg. 4: p_view.z > 0.2) */
    if (!(tz > cam->near_z)) return 0;
    /* opacity prefilter (Alg. 4: opacity > 1/255); opacity = sigmoid(logit), reading */
    REAL o = R_SIGMOID(logit);
    if (!(o > op->alpha_min)) return 0;
    /* scale = exp(log-scale), rotation from the normalised quaternion (reading) */
    REAL s0 = R_EXP(ls0), s1 = R_EXP(ls1), s2 = R_EXP(ls2);
    REAL n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    if (!(n2 > (REAL)0) || !R_ISFINITE(n2)) return 0;
    REAL qn = R_SQRT(n2);
    REAL w = qw / qn, x = qx / qn, y = qy / qn, z = qz / qn;
    /* pinhole projection (project + ndc2Pix) */
    REAL xt = tx / tz, yt = ty / tz;
    REAL u = cam->fx * xt + cam->cx;
    REAL v = cam->fy * yt + cam->cy;
    /* EWA Jacobian of the perspective map, with the view-direction clamp
     * at jac_clip times the half-width of the image plane (reading) */
    REAL limx = op->jac_clip * (((REAL)0.5 * (REAL)W) / cam->fx);
    REAL limy = op->jac_clip * (((REAL)0.5 * (REAL)H) / cam->fy);
    REAL xc = FN(orc_clamp)(xt, -limx, limx);
    REAL yc = FN(orc_clamp)(yt, -limy, limy);
    REAL J00 = cam->fx / tz, J02 = -((cam->fx * xc) / tz);
    REAL J11 = cam->fy / tz, J12 = -((cam->fy * yc) / tz);
    /* computeCov3D: Sigma = M M^T, M = R_q diag(s) */
    REAL r00 = (REAL)1 - (REAL)2 * (y * y + z * z);
    REAL r01 = (REAL)2 * (x * y - w * z);
    REAL r02 = (REAL)2 * (x * z + w * y);
    REAL r10 = (REAL)2 * (x * y + w * z);
    REAL r11 = (REAL)1 - (REAL)2 * (x * x + z * z);
    REAL r12 = (REAL)2 * (y * z - w * x);
    REAL r20 = (REAL)2 * (x * z - w * y);
    REAL r21 = (REAL)2 * (y * z + w * x);
    REAL r22 = (REAL)1 - (REAL)2 * (x * x + y * y);
    REAL M00 = r00 * s0, M01 = r01 * s1, M02 = r02 * s2;
    REAL M10 = r10 * s0, M11 = r11 * s1, M12 = r12 * s2;
    REAL M20 = r20 * s0, M21 = r21 * s1, M22 = r22 * s2;
    REAL S00 = (M00 * M00 + M01 * M01) + M02 * M02;
    REAL S01 = (M00 * M10 + M01 * M11) + M02 * M12;
    REAL S02 = (M00 * M20 + M01 * M21) + M02 * M22;
    REAL S11 = (M10 * M10 + M11 * M11) + M12 * M12;
    REAL S12 = (M10 * M20 + M11 * M21) + M12 * M22;
    REAL S22 = (M20 * M20 + M21 * M21) + M22 * M22;
    /* computeCov2D: Sigma' = T Sigma T^T with T = J R_cam (2 x 3) */
    REAL T00 = J00 * R[0] + J02 * R[6], T01 = J00 * R[1] + J02 * R[7], T02 = J00 * R[2] + J02 * R[8];
    REAL T10 = J11 * R[3] + J12 * R[6], T11 = J11 * R[4] + J12 * R[7], T12 = J11 * R[5] + J12 * R[8];
    REAL U00 = (T00 * S00 + T01 * S01) + T02 * S02;
    REAL U01 = (T00 * S01 + T01 * S11) + T02 * S12;
    REAL U02 = (T00 * S02 + T01 * S12) + T02 * S22;
    REAL U10 = (T10 * S00 + T11 * S01) + T12 * S02;
    REAL U11 = (T10 * S01 + T11 * S11) + T12 * S12;
    REAL U12 = (T10 * S02 + T11 * S12) + T12 * S22;
    /* low-pass dilation of 0.3 px^2 on the diagonal (reading) */
    REAL ca = ((U00 * T00 + U01 * T01) + U02 * T02) + op->dilation;
    REAL cb = (U00 * T10 + U01 * T11) + U02 * T12;
    REAL cc = ((U10 * T10 + U11 * T11) + U12 * T12) + op->dilation;
    /* conic = inverse of Sigma' */
    REAL det = ca * cc - cb * cb;
    if (!(det > (REAL)0)) return 0;
    REAL A = cc / det, B = (-cb) / det, C = ca / det;
    /* opacity-aware extent: alpha(r) = o exp(-r^2 / 2 lambda) falls to tau at
     * r^2 = 2 ln(o / tau) lambda (Eq. 2, Eq. 3), capped at the 3 sigma rule
     * r^2 = 9 lambda (Eq. 1) when that is smaller (o > e^4.5 / 255 ~ 0.353) */
    REAL k2 = R_EXTENT(o, op->alpha_min, op->cap_3sigma);
    /* rectangle tightly tangent to the ellipse (Sec. 4.1): half-extents
     * k sqrt(Sigma'_xx), k sqrt(Sigma'_yy), taken over pixel samples */
    REAL hx, hy;
    if (op->binning == 2) {
        /* comparison mode: the square box of the circle of radius
         * ceil(3 sqrt(lambda_max)) of Sigma' (Alg. 1, Eq. 1), every tile of it
         * (Alg. 2); the per-pixel rule, and so the image, is unchanged
         * (reading: the box is taken over pixel samples like the tight one) */
        REAL mid = (REAL)0.5 * (ca + cc);
        REAL disc = mid * mid - det;
        if (disc < (REAL)0) disc = (REAL)0;
        REAL lam = mid + R_SQRT(disc);
        hx = R_CEIL((REAL)3 * R_SQRT(lam));
        hy = hx;
    } else {
        hx = R_SQRT(k2 * ca);
        hy = R_SQRT(k2 * cc);
    }
    REAL xlo = FN(orc_clamp)((u - hx) - (REAL)0.5, (REAL)-1, (REAL)W);
    REAL xhi = FN(orc_clamp)((u + hx) - (REAL)0.5, (REAL)-1, (REAL)W);
    REAL ylo = FN(orc_clamp)((v - hy) - (REAL)0.5, (REAL)-1, (REAL)H);
    REAL yhi = FN(orc_clamp)((v + hy) - (REAL)0.5, (REAL)-1, (REAL)H);
    int i0 = (int)R_CEIL(xlo), i1 = (int)R_FLOOR(xhi);
    int j0 = (int)R_CEIL(ylo), j1 = (int)R_FLOOR(yhi);
    if (i0 < 0) i0 = 0;
    if (j0 < 0) j0 = 0;
    if (i1 > W - 1) i1 = W - 1;
    if (j1 > H - 1) j1 = H - 1;
    if (i0 > i1 || j0 > j1) return 0; /* box holds no pixel sample (Alg. 4: bounding box is non-zero) */
    /* SH colour, computed only for Gaussians that survived (Alg. 4) */
    int D = sc->D;
    int nk = (D + 1) * (D + 1);
    REAL dxw = mx - cam->eye[0], dyw = my - cam->eye[1], dzw = mz - cam->eye[2];
    REAL dn = R_SQRT((dxw * dxw + dyw * dyw) + dzw * dzw);
    REAL Y[16];
    FN(orc_sh_basis)(dxw / dn, dyw / dn, dzw / dn, Y);
    REAL col[3];
    for (int ch = 0; ch < 3; ++ch) {
        REAL acc = (REAL)0;
        for (int k = 0; k < nk; ++k) acc = acc + sc->sh[(int64_t)(3 * k + ch) * st + g] * Y[k];
        acc = acc + (REAL)0.5; /* offset and clamp at zero (reading) */
        if (!R_ISFINITE(acc)) return 0; /* non-finite SH inputs are culled (reading) */
        col[ch] = acc > (REAL)0 ? acc : (REAL)0;
    }
    s[S_U] = u; s[S_V] = v; s[S_A] = A; s[S_B] = B; s[S_C] = C; s[S_K2] = k2;
    s[S_O] = o; s[S_DEPTH] = tz;
    s[S_R] = col[0]; s[S_G] = col[1]; s[S_BL] = col[2];
    s[S_COVA] = ca; s[S_COVB] = cb; s[S_COVC] = cc; s[S_HX] = hx; s[S_HY] = hy;
    iv[I_VALID] = 1;
    iv[I_I0] = i0; iv[I_I1] = i1; iv[I_J0] = j0; iv[I_J1] = j1;
    iv[I_TX0] = i0 / TILE; iv[I_TX1] = i1 / TILE; iv[I_TY0] = j0 / TILE; iv[I_TY1] = j1 / TILE;
    /* exact count of tiles of the rectangle that meet the ellipse (Alg. 3) */
    int cnt = 0;
    for (int ty_ = iv[I_TY0]; ty_ <= iv[I_TY1]; ++ty_)
        for (int tx_ = iv[I_TX0]; tx_ <= iv[I_TX1]; ++tx_)
            cnt += (op->binning != 0) ? 1 : FN(orc_tile_hit)(s, tx_, ty_, W, H);
    iv[I_COUNT] = cnt;
    return 1;
}

/* Preprocess every Gaussian.  state: [P][S_N]; ints: [P][I_N].
 * Returns the total number of Gaussian-tile pairs. */
int64_t FN(orc_preprocess)(const TYPE(orc_scene) *sc, const TYPE(orc_camera) *cam, int W, int H,
                           const TYPE(orc_options) *op, REAL *state, int32_t *ints)
{
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : total)
    for (int64_t g = 0; g < sc->P; ++g) {
        FN(orc_gauss)(sc, g, cam, W, H, op, state + g * S_N, ints + g * I_N);
        total += ints[g * I_N + I_COUNT];
    }
    return total;
}

typedef struct {
    uint32_t tile;
    uint32_t g;
    REAL depth;
} FN(orc_pair);

static int FN(orc_pair_cmp)(const void *pa, const void *pb)
{
    const FN(orc_pair) *a = (const FN(orc_pair) *)pa, *b = (const FN(orc_pair) *)pb;
    if (a->depth < b->depth) return -1;
    if (a->depth > b->depth) return 1;
    return (a->g < b->g) ? -1 : (a->g > b->g);
}

/* Key/value pairs sorted by (tile, depth, index) (Sec. 2.2: key = tile index
 * and depth, value = Gaussian index; ties between equal keys in ascending
 * index, reading), with per-tile ranges [range[2t], range[2t+1]).
 * Buckets the pairs by tile (Gaussians visited in index order), then sorts
 * each bucket by (depth, index).  tiles/vals: [npairs]; range: [2 * ntiles]. */
void FN(orc_pairs)(const TYPE(orc_scene) *sc, int W, int H, const TYPE(orc_options) *op,
                   const REAL *state, const int32_t *ints, int64_t npairs,
                   uint32_t *tiles_out, uint32_t *vals_out, int64_t *range)
{
    int tiles_x = (W + TILE - 1) / TILE, tiles_y = (H + TILE - 1) / TILE;
    int64_t ntiles = (int64_t)tiles_x * tiles_y;
    int64_t *cnt = (int64_t *)calloc((size_t)ntiles + 1, sizeof(int64_t));
    for (int64_t g = 0; g < sc->P; ++g) {
        const int32_t *iv = ints + g * I_N;
        if (!iv[I_VALID]) continue;
        for (int ty = iv[I_TY0]; ty <= iv[I_TY1]; ++ty)
            for (int tx = iv[I_TX0]; tx <= iv[I_TX1]; ++tx)
                if (op->binning != 0 || FN(orc_tile_hit)(state + g * S_N, tx, ty, W, H))
                    cnt[(int64_t)ty * tiles_x + tx + 1]++;
    }
    for (int64_t t = 0; t < ntiles; ++t) cnt[t + 1] += cnt[t];
    FN(orc_pair) *pr = (FN(orc_pair) *)malloc(sizeof(FN(orc_pair)) * (size_t)(npairs > 0 ? npairs : 1));
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ntiles > 0 ? ntiles : 1));
    for (int64_t t = 0; t < ntiles; ++t) cur[t] = cnt[t];
    for (int64_t g = 0; g < sc->P; ++g) {
        const int32_t *iv = ints + g * I_N;
        if (!iv[I_VALID]) continue;
        for (int ty = iv[I_TY0]; ty <= iv[I_TY1]; ++ty)
            for (int tx = iv[I_TX0]; tx <= iv[I_TX1]; ++tx)
                if (op->binning != 0 || FN(orc_tile_hit)(state + g * S_N, tx, ty, W, H)) {
                    int64_t t = (int64_t)ty * tiles_x + tx;
                    int64_t at = cur[t]++;
                    if (at < npairs) {
                        pr[at].tile = (uint32_t)t;
                        pr[at].g = (uint32_t)g;
                        pr[at].depth = state[g * S_N + S_DEPTH];
                    }
                }
    }
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < ntiles; ++t) {
        int64_t a = cnt[t], b = cnt[t + 1];
        if (b > npairs) b = npairs;
        if (b - a > 1) qsort(pr + a, (size_t)(b - a), sizeof(FN(orc_pair)), FN(orc_pair_cmp));
    }
    for (int64_t i = 0; i < npairs; ++i) {
        tiles_out[i] = pr[i].tile;
        vals_out[i] = pr[i].g;
    }
    for (int64_t t = 0; t < ntiles; ++t) {
        range[2 * t] = cnt[t];
        range[2 * t + 1] = cnt[t + 1];
    }
    free(pr);
    free(cur);
    free(cnt);
}

/* Quadratic form of the conic at pixel-sample offset (dx, dy) */
static REAL FN(orc_q)(const REAL *s, REAL dx, REAL dy)
{
    return (s[S_A] * dx * dx + (REAL)2 * s[S_B] * dx * dy) + s[S_C] * dy * dy;
}

/* Front-to-back blending of one pixel over an ordered list of Gaussians
 * (Sec. 2.2 rendering; early termination on transmittance, Sec. 5.2).
 * Contribution rule (reading): Gaussian g contributes at sample s iff
 * q_g(s) <= k_g^2; alpha = min(alpha_max, o exp(-q/2)); if T (1 - alpha) would
 * fall below T_stop the pixel stops before blending that Gaussian. */
static void FN(orc_blend_pixel)(const REAL *state, const uint32_t *list, int64_t n, REAL px, REAL py,
                                const TYPE(orc_options) *op, REAL *rgb, REAL *T_out, uint32_t *last_out)
{
    REAL T = (REAL)1, c0 = 0, c1 = 0, c2 = 0;
    uint32_t last = 0;
    for (int64_t i = 0; i < n; ++i) {
        const REAL *s = state + (int64_t)list[i] * S_N;
        REAL dx = px - s[S_U], dy = py - s[S_V];
        REAL q = FN(orc_q)(s, dx, dy);
        if (!(q <= s[S_K2])) continue;
        REAL alpha = s[S_O] * R_EXP(-(REAL)0.5 * q);
        if (alpha > op->alpha_max) alpha = op->alpha_max;
        REAL Tn = T * ((REAL)1 - alpha);
        if (Tn < op->T_stop) break;
        REAL wgt = alpha * T;
        c0 = c0 + s[S_R] * wgt;
        c1 = c1 + s[S_G] * wgt;
        c2 = c2 + s[S_BL] * wgt;
        T = Tn;
        last = (uint32_t)(i + 1);
    }
    rgb[0] = c0 + T * op->bg[0];
    rgb[1] = c1 + T * op->bg[1];
    rgb[2] = c2 + T * op->bg[2];
    *T_out = T;
    *last_out = last;
}

/* Tiled render: every pixel of tile t blends the tile's sorted list.
 * rgb: [3][H][W]; T: [H][W]; last: [H][W] (1 + list position of the last
 * contributor within its tile's list, 0 if none). */
void FN(orc_blend_tiled)(const REAL *state, int W, int H, const TYPE(orc_options) *op, const uint32_t *vals,
                         const int64_t *range, REAL *rgb, REAL *Tout, uint32_t *last)
{
    int tiles_x = (W + TILE - 1) / TILE, tiles_y = (H + TILE - 1) / TILE;
    int64_t HW = (int64_t)H * W;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t t = 0; t < (int64_t)tiles_x * tiles_y; ++t) {
        int tx = (int)(t % tiles_x), ty = (int)(t / tiles_x);
        const uint32_t *list = vals + range[2 * t];
        int64_t n = range[2 * t + 1] - range[2 * t];
        for (int j = ty * TILE; j < ty * TILE + TILE && j < H; ++j)
            for (int i = tx * TILE; i < tx * TILE + TILE && i < W; ++i) {
                REAL c[3];
                int64_t p = (int64_t)j * W + i;
                FN(orc_blend_pixel)(state, list, n, (REAL)i + (REAL)0.5, (REAL)j + (REAL)0.5, op, c, Tout + p,
                                    last + p);
                rgb[p] = c[0];
                rgb[HW + p] = c[1];
                rgb[2 * HW + p] = c[2];
            }
    }
}

/* Brute force without tiles: every pixel blends all valid Gaussians in
 * (depth, index) order.  For tiny scenes only. */
void FN(orc_blend_brute)(const REAL *state, const int32_t *ints, int64_t P, int W, int H,
                         const TYPE(orc_options) *op, REAL *rgb, REAL *Tout, uint32_t *last)
{
    FN(orc_pair) *pr = (FN(orc_pair) *)malloc(sizeof(FN(orc_pair)) * (size_t)(P > 0 ? P : 1));
    int64_t n = 0;
    for (int64_t g = 0; g < P; ++g)
        if (ints[g * I_N + I_VALID]) {
            pr[n].tile = 0;
            pr[n].g = (uint32_t)g;
            pr[n].depth = state[g * S_N + S_DEPTH];
            n++;
        }
    qsort(pr, (size_t)n, sizeof(FN(orc_pair)), FN(orc_pair_cmp));
    uint32_t *list = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) list[i] = pr[i].g;
    int64_t HW = (int64_t)H * W;
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            REAL c[3];
            int64_t p = (int64_t)j * W + i;
            FN(orc_blend_pixel)(state, list, n, (REAL)i + (REAL)0.5, (REAL)j + (REAL)0.5, op, c, Tout + p, last + p);
            rgb[p] = c[0];
            rgb[HW + p] = c[1];
            rgb[2 * HW + p] = c[2];
        }
    free(list);
    free(pr);
}

/* Real SH basis at a direction, for the tests' independent check. */
void FN(orc_sh_eval)(REAL x, REAL y, REAL z, REAL *Y16)
{
    FN(orc_sh_basis)(x, y, z, Y16);
}
