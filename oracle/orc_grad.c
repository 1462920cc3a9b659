/*
 * Reverse-mode derivative of the oracle's binary64 rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of oracle/: the product library
 * never links, loads or calls it.
 *
 * The paper calls its rasterizer differentiable and gives no adjoint, so
 * this file is the derivative of the image defined in orc_core.c (binary64
 * mode) with respect to the raw Gaussian parameters, written out by the chain
 * rule.  The discrete structure is held fixed: which Gaussians survive the
 * culls, each pixel's contributors (q <= k^2) and stopping point, which
 * alphas are clamped at alpha_max, which colour channels are clamped at 0 and
 * which view directions are clamped in the Jacobian.  Through a clamped
 * quantity the derivative is zero (the derivative of the clamp away from its
 * kink).  The contribution boundary q = k^2 moves with the opacity; that
 * boundary term only matters for a pixel sample lying exactly on the
 * ellipse, and it is not differentiated.
 *
 * Blend, per pixel, contributors n = 1..m front to back (colour c_n, alpha
 * a_n, transmittance T_n before n):
 *     C = sum_n c_n a_n T_n + T_{m+1} bg,      T_{n+1} = T_n (1 - a_n)
 *     dC/dc_n = a_n T_n
 *     dC/da_n = T_n (c_n - R_n),
 * where R_n is the colour the contributors after n composite over the
 * background with the transmittance restarted at 1:
 *     R_m = bg,   R_{n-1} = c_n a_n + (1 - a_n) R_n.
 * This is the product rule on the front-to-back sum; it divides by nothing.
 * Then a = o exp(-q/2) (unclamped): da/do = exp(-q/2), da/dq = -a/2, and
 * q = A dx^2 + 2 B dx dy + C dy^2 with (dx, dy) = sample - (u, v).
 *
 * Per Gaussian, the preprocessing steps of orc_core.c are recomputed in
 * binary64 and differentiated in reverse order: conic = inverse of Sigma',
 * Sigma' = T Sigma T^T + dilation I with T = J R_cam, Sigma = M M^T with
 * M = R(q / |q|) diag(exp(log-scale)), J and (u, v) from the camera-space
 * mean, opacity = sigmoid(logit), colour = max(0, sum_k sh_k Y_k(d) + 1/2)
 * with d the unit direction from the camera centre to the mean.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double REAL;
#define TYPE(name) name##_f64
#include "orc_types.h"

#define TILE 16

void orc_sh_eval_f64(double x, double y, double z, double *Y16);

/* Per-Gaussian gradient of the loss with respect to the blended state. */
enum { G_U, G_V, G_A, G_B, G_C, G_O, G_R, G_G, G_BL, G_N = 9 };

/* Gradient of each real SH basis polynomial of orc_core.c with respect to
 * (x, y, z), the polynomials taken as functions on R^3.  Only the component
 * tangent to the unit sphere is used (the direction is normalised), and that
 * component does not depend on how the polynomial is extended off the
 * sphere. */
static void sh_basis_grad(double x, double y, double z, double dY[16][3])
{
    const double pi = 3.14159265358979323846;
    const double k1 = sqrt(3.0 / (4.0 * pi));
    const double k2a = sqrt(15.0 / (4.0 * pi));
    const double k20 = sqrt(5.0 / (16.0 * pi));
    const double k22 = sqrt(15.0 / (16.0 * pi));
    const double k33 = sqrt(35.0 / (32.0 * pi));
    const double k32 = sqrt(105.0 / (4.0 * pi));
    const double k31 = sqrt(21.0 / (32.0 * pi));
    const double k30 = sqrt(7.0 / (16.0 * pi));
    const double k32b = sqrt(105.0 / (16.0 * pi));
    memset(dY, 0, sizeof(double) * 48);
    /* Y1 = -k1 y, Y2 = k1 z, Y3 = -k1 x */
    dY[1][1] = -k1;
    dY[2][2] = k1;
    dY[3][0] = -k1;
    /* Y4 = k2a x y */
    dY[4][0] = k2a * y; dY[4][1] = k2a * x;
    /* Y5 = -k2a y z */
    dY[5][1] = -k2a * z; dY[5][2] = -k2a * y;
    /* Y6 = k20 (3 z^2 - 1) */
    dY[6][2] = 6.0 * k20 * z;
    /* Y7 = -k2a x z */
    dY[7][0] = -k2a * z; dY[7][2] = -k2a * x;
    /* Y8 = k22 (x^2 - y^2) */
    dY[8][0] = 2.0 * k22 * x; dY[8][1] = -2.0 * k22 * y;
    /* Y9 = -k33 (3 x^2 y - y^3) */
    dY[9][0] = -6.0 * k33 * x * y; dY[9][1] = -k33 * (3.0 * x * x - 3.0 * y * y);
    /* Y10 = k32 x y z */
    dY[10][0] = k32 * y * z; dY[10][1] = k32 * x * z; dY[10][2] = k32 * x * y;
    /* Y11 = -k31 y (5 z^2 - 1) */
    dY[11][1] = -k31 * (5.0 * z * z - 1.0); dY[11][2] = -10.0 * k31 * y * z;
    /* Y12 = k30 (5 z^3 - 3 z) */
    dY[12][2] = k30 * (15.0 * z * z - 3.0);
    /* Y13 = -k31 x (5 z^2 - 1) */
    dY[13][0] = -k31 * (5.0 * z * z - 1.0); dY[13][2] = -10.0 * k31 * x * z;
    /* Y14 = k32b z (x^2 - y^2) */
    dY[14][0] = 2.0 * k32b * x * z; dY[14][1] = -2.0 * k32b * y * z; dY[14][2] = k32b * (x * x - y * y);
    /* Y15 = -k33 (x^3 - 3 x y^2) */
    dY[15][0] = -k33 * (3.0 * x * x - 3.0 * y * y); dY[15][1] = 6.0 * k33 * x * y;
}

/* ---- small dense helpers (row-major) ------------------------------------ */

static void matmul(const double *a, const double *b, double *c, int n, int k, int m)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j) {
            double s = 0.0;
            for (int l = 0; l < k; ++l) s += a[i * k + l] * b[l * m + j];
            c[i * m + j] = s;
        }
}

static void transpose(const double *a, double *t, int n, int m)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < m; ++j) t[j * n + i] = a[i * m + j];
}

/* ---- blend adjoint -------------------------------------------------------- */

typedef struct {
    uint32_t g;
    double a, T, G, dx, dy;
    int clamped;
} contrib;

/* Accumulates dL/d(state) of every Gaussian (gs: [P][G_N]) from dL/dRGB
 * (dL: [3][H][W]), walking each pixel's tile list exactly as the forward
 * blend does (same contribution, clamp and stopping rules). */
static void blend_adjoint(const double *state, int W, int H, const orc_options_f64 *op, const uint32_t *vals,
                          const int64_t *range, const double *dL, int64_t P, double *gs)
{
    int tiles_x = (W + TILE - 1) / TILE, tiles_y = (H + TILE - 1) / TILE;
    int64_t ntiles = (int64_t)tiles_x * tiles_y, HW = (int64_t)H * W;
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *part = (double *)calloc((size_t)nth * (size_t)P * G_N + 1, sizeof(double));
#pragma omp parallel
    {
        int th = 0;
#ifdef _OPENMP
        th = omp_get_thread_num();
#endif
        double *acc = part + (size_t)th * (size_t)P * G_N;
        int64_t cap = 0;
        contrib *cs = NULL;
        double *Rr = NULL;
        /* static schedule: for a given thread count every thread sums the
         * same tiles in the same order, so the result is reproducible */
#pragma omp for schedule(static)
        for (int64_t t = 0; t < ntiles; ++t) {
            int64_t n = range[2 * t + 1] - range[2 * t];
            const uint32_t *list = vals + range[2 * t];
            if (n > cap) {
                cap = n;
                cs = (contrib *)realloc(cs, sizeof(contrib) * (size_t)cap);
                Rr = (double *)realloc(Rr, sizeof(double) * 3 * (size_t)(cap + 1));
            }
            int tx = (int)(t % tiles_x), ty = (int)(t / tiles_x);
            for (int j = ty * TILE; j < ty * TILE + TILE && j < H; ++j)
                for (int i = tx * TILE; i < tx * TILE + TILE && i < W; ++i) {
                    int64_t p = (int64_t)j * W + i;
                    double px = i + 0.5, py = j + 0.5;
                    /* forward walk: contributors, their alpha and T */
                    double T = 1.0;
                    int64_t m = 0;
                    for (int64_t k = 0; k < n; ++k) {
                        const double *s = state + (int64_t)list[k] * S_N;
                        double dx = px - s[S_U], dy = py - s[S_V];
                        double q = (s[S_A] * dx * dx + 2.0 * s[S_B] * dx * dy) + s[S_C] * dy * dy;
                        if (!(q <= s[S_K2])) continue;
                        double G = exp(-0.5 * q);
                        double a = s[S_O] * G;
                        int clamped = 0;
                        if (a > op->alpha_max) {
                            a = op->alpha_max;
                            clamped = 1;
                        }
                        double Tn = T * (1.0 - a);
                        if (Tn < op->T_stop) break;
                        cs[m].g = list[k];
                        cs[m].a = a;
                        cs[m].T = T;
                        cs[m].G = G;
                        cs[m].dx = dx;
                        cs[m].dy = dy;
                        cs[m].clamped = clamped;
                        ++m;
                        T = Tn;
                    }
                    /* R_n, back to front: Rr[3 n + ch] is R after contributor n (0-based) */
                    if (m == 0) continue;
                    for (int ch = 0; ch < 3; ++ch) Rr[3 * (m - 1) + ch] = op->bg[ch];
                    for (int64_t k = m - 1; k >= 1; --k) {
                        const double *s = state + (int64_t)cs[k].g * S_N;
                        for (int ch = 0; ch < 3; ++ch)
                            Rr[3 * (k - 1) + ch] = s[S_R + ch] * cs[k].a + (1.0 - cs[k].a) * Rr[3 * k + ch];
                    }
                    double gC[3] = {dL[p], dL[HW + p], dL[2 * HW + p]};
                    for (int64_t k = 0; k < m; ++k) {
                        const double *s = state + (int64_t)cs[k].g * S_N;
                        double *ga = acc + (int64_t)cs[k].g * G_N;
                        double w = cs[k].a * cs[k].T;
                        double galpha = 0.0;
                        for (int ch = 0; ch < 3; ++ch) {
                            ga[G_R + ch] += gC[ch] * w;
                            galpha += gC[ch] * cs[k].T * (s[S_R + ch] - Rr[3 * k + ch]);
                        }
                        if (cs[k].clamped) continue;
                        double gq = -0.5 * cs[k].a * galpha;
                        ga[G_O] += galpha * cs[k].G;
                        double dx = cs[k].dx, dy = cs[k].dy;
                        ga[G_A] += gq * dx * dx;
                        ga[G_B] += gq * 2.0 * dx * dy;
                        ga[G_C] += gq * dy * dy;
                        /* dq/du = -(2 A dx + 2 B dy), dq/dv = -(2 B dx + 2 C dy) */
                        ga[G_U] += gq * -(2.0 * s[S_A] * dx + 2.0 * s[S_B] * dy);
                        ga[G_V] += gq * -(2.0 * s[S_B] * dx + 2.0 * s[S_C] * dy);
                    }
                }
        }
        free(cs);
        free(Rr);
    }
    for (int th = 0; th < nth; ++th) {
        const double *a = part + (size_t)th * (size_t)P * G_N;
        for (int64_t i = 0; i < P * G_N; ++i) gs[i] += a[i];
    }
    free(part);
}

/* ---- preprocess adjoint ----------------------------------------------------- */

/* Gradients of one valid Gaussian g's raw parameters from gsg = dL/d(u, v,
 * A, B, C, o, colour).  Outputs are planar with stride P. */
static void gauss_adjoint(const orc_scene_f64 *sc, int64_t g, const orc_camera_f64 *cam, int W, int H,
                          const orc_options_f64 *op, const double *gsg, double *gm, double *gls, double *gq,
                          double *glogit, double *gsh)
{
    const int64_t st = sc->stride, P = sc->P;
    double m[3] = {sc->means[g], sc->means[st + g], sc->means[2 * st + g]};
    double ls[3] = {sc->log_scales[g], sc->log_scales[st + g], sc->log_scales[2 * st + g]};
    double qr[4] = {sc->quats[g], sc->quats[st + g], sc->quats[2 * st + g], sc->quats[3 * st + g]};
    double logit = sc->logits[g];
    const double *Rc = cam->R;
    double fx = cam->fx, fy = cam->fy;

    /* forward recomputation */
    double t[3];
    for (int r = 0; r < 3; ++r) t[r] = Rc[3 * r] * m[0] + Rc[3 * r + 1] * m[1] + Rc[3 * r + 2] * m[2] + cam->t[r];
    double o = 1.0 / (1.0 + exp(-logit));
    double s[3] = {exp(ls[0]), exp(ls[1]), exp(ls[2])};
    double qn = sqrt(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
    double w = qr[0] / qn, x = qr[1] / qn, y = qr[2] / qn, z = qr[3] / qn;
    double xt = t[0] / t[2], yt = t[1] / t[2];
    double limx = op->jac_clip * (0.5 * W / fx), limy = op->jac_clip * (0.5 * H / fy);
    int clipx = xt < -limx || xt > limx, clipy = yt < -limy || yt > limy;
    double xc = clipx ? (xt < 0 ? -limx : limx) : xt;
    double yc = clipy ? (yt < 0 ? -limy : limy) : yt;
    double J[6] = {fx / t[2], 0.0, -fx * xc / t[2], 0.0, fy / t[2], -fy * yc / t[2]};
    double Rq[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                    2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                    2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    double M[9], Mt[9], Sig[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[3 * i + j] = Rq[3 * i + j] * s[j];
    transpose(M, Mt, 3, 3);
    matmul(M, Mt, Sig, 3, 3, 3);
    double T[6], Tt[6], TS[6], Sp[4];
    matmul(J, Rc, T, 2, 3, 3);
    transpose(T, Tt, 2, 3);
    matmul(T, Sig, TS, 2, 3, 3);
    matmul(TS, Tt, Sp, 2, 3, 2);
    double a = Sp[0] + op->dilation, b = Sp[1], c = Sp[3] + op->dilation;
    double det = a * c - b * b;
    double Y2[4] = {c / det, -b / det, -b / det, a / det}; /* conic as a 2 x 2 matrix */

    /* conic: dL/dY with the off-diagonal scalar B split over both entries */
    double gY[4] = {gsg[G_A], 0.5 * gsg[G_B], 0.5 * gsg[G_B], gsg[G_C]};
    /* Y = X^{-1}: dL/dX = -Y^T dL/dY Y^T; X = Sigma' + dilation I */
    double tmp[4], gSp[4];
    matmul(Y2, gY, tmp, 2, 2, 2);
    matmul(tmp, Y2, gSp, 2, 2, 2);
    for (int i = 0; i < 4; ++i) gSp[i] = -gSp[i];
    /* Sigma' = T Sigma T^T: dL/dSigma = T^T gSp T, dL/dT = gSp T Sigma^T + gSp^T T Sigma */
    double gSig[9], tmp23[6], gT[6], gSpt[4], tmp23b[6];
    double gSpT[6];
    matmul(gSp, T, gSpT, 2, 2, 3);
    matmul(Tt, gSpT, gSig, 3, 2, 3);
    double Sigt[9];
    transpose(Sig, Sigt, 3, 3);
    matmul(gSpT, Sigt, tmp23, 2, 3, 3);
    transpose(gSp, gSpt, 2, 2);
    double gSptT[6];
    matmul(gSpt, T, gSptT, 2, 2, 3);
    matmul(gSptT, Sig, tmp23b, 2, 3, 3);
    for (int i = 0; i < 6; ++i) gT[i] = tmp23[i] + tmp23b[i];
    /* T = J R_cam: dL/dJ = gT R_cam^T */
    double Rct[9], gJ[6];
    transpose(Rc, Rct, 3, 3);
    matmul(gT, Rct, gJ, 2, 3, 3);
    /* Sigma = M M^T: dL/dM = (gSig + gSig^T) M */
    double gSigS[9], gM[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) gSigS[3 * i + j] = gSig[3 * i + j] + gSig[3 * j + i];
    matmul(gSigS, M, gM, 3, 3, 3);
    /* M = Rq diag(s) */
    double gR[9], gs[3] = {0, 0, 0};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            gR[3 * i + j] = gM[3 * i + j] * s[j];
            gs[j] += gM[3 * i + j] * Rq[3 * i + j];
        }
    for (int j = 0; j < 3; ++j) gls[j * P + g] = gs[j] * s[j];
    /* rotation matrix of the unit quaternion (w, x, y, z) */
    double gw = 2 * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
    double gx = 2 * (y * gR[1] + z * gR[2] + y * gR[3] - 2 * x * gR[4] - w * gR[5] + z * gR[6] + w * gR[7] -
                     2 * x * gR[8]);
    double gy = 2 * (-2 * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] + z * gR[7] -
                     2 * y * gR[8]);
    double gz = 2 * (-2 * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2 * z * gR[4] + y * gR[5] + x * gR[6] +
                     y * gR[7]);
    /* normalisation q / |q| */
    double qh[4] = {w, x, y, z}, gqh[4] = {gw, gx, gy, gz};
    double dot = qh[0] * gqh[0] + qh[1] * gqh[1] + qh[2] * gqh[2] + qh[3] * gqh[3];
    for (int i = 0; i < 4; ++i) gq[i * P + g] = (gqh[i] - qh[i] * dot) / qn;
    /* J from the camera-space mean (J01 and J10 are constant zero) */
    double gt[3] = {0, 0, 0};
    gt[2] += gJ[0] * (-fx / (t[2] * t[2])) + gJ[4] * (-fy / (t[2] * t[2]));
    gt[2] += gJ[2] * (fx * xc / (t[2] * t[2])) + gJ[5] * (fy * yc / (t[2] * t[2]));
    double gxt = clipx ? 0.0 : gJ[2] * (-fx / t[2]);
    double gyt = clipy ? 0.0 : gJ[5] * (-fy / t[2]);
    /* u = fx x~ + cx, v = fy y~ + cy */
    gxt += gsg[G_U] * fx;
    gyt += gsg[G_V] * fy;
    /* x~ = t_x / t_z, y~ = t_y / t_z */
    gt[0] += gxt / t[2];
    gt[1] += gyt / t[2];
    gt[2] += -gxt * t[0] / (t[2] * t[2]) - gyt * t[1] / (t[2] * t[2]);
    /* t = R_cam m + t_cam */
    double gmean[3];
    for (int j = 0; j < 3; ++j) gmean[j] = Rc[j] * gt[0] + Rc[3 + j] * gt[1] + Rc[6 + j] * gt[2];
    /* opacity */
    glogit[g] = gsg[G_O] * o * (1.0 - o);
    /* colour from SH at the view direction */
    int nk = (sc->D + 1) * (sc->D + 1);
    double dw[3] = {m[0] - cam->eye[0], m[1] - cam->eye[1], m[2] - cam->eye[2]};
    double dn = sqrt(dw[0] * dw[0] + dw[1] * dw[1] + dw[2] * dw[2]);
    double d[3] = {dw[0] / dn, dw[1] / dn, dw[2] / dn};
    double Y[16], dY[16][3];
    orc_sh_eval_f64(d[0], d[1], d[2], Y);
    sh_basis_grad(d[0], d[1], d[2], dY);
    double gd[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ++ch) {
        double raw = 0.5;
        for (int k = 0; k < nk; ++k) raw += sc->sh[(int64_t)(3 * k + ch) * st + g] * Y[k];
        double gcol = raw > 0.0 ? gsg[G_R + ch] : 0.0;
        for (int k = 0; k < nk; ++k) {
            gsh[(int64_t)(3 * k + ch) * P + g] = gcol * Y[k];
            double shv = sc->sh[(int64_t)(3 * k + ch) * st + g];
            for (int e = 0; e < 3; ++e) gd[e] += gcol * shv * dY[k][e];
        }
    }
    /* d = dw / |dw|: dL/d(dw) = (gd - d (d . gd)) / |dw| */
    double dd = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
    for (int e = 0; e < 3; ++e) gmean[e] += (gd[e] - d[e] * dd) / dn;
    for (int e = 0; e < 3; ++e) gm[e * P + g] = gmean[e];
}

/* dL/d(raw parameters) for dL/dRGB = dL ([3][H][W]), given the binary64
 * forward's per-Gaussian state and ints (orc_preprocess_f64) and its sorted
 * lists (orc_pairs_f64).  Gradient planes have stride P and are overwritten;
 * culled Gaussians get zero.  gstate ([P][9], may be NULL) receives
 * dL/d(u, v, A, B, C, o, r, g, b). */
void orc_backward_f64(const orc_scene_f64 *sc, const orc_camera_f64 *cam, int W, int H, const orc_options_f64 *op,
                      const double *state, const int32_t *ints, const uint32_t *vals, const int64_t *range,
                      const double *dL, double *gm, double *gls, double *gq, double *glogit, double *gsh,
                      double *gstate)
{
    int64_t P = sc->P;
    int nk = (sc->D + 1) * (sc->D + 1);
    double *gs = (double *)calloc((size_t)P * G_N + 1, sizeof(double));
    blend_adjoint(state, W, H, op, vals, range, dL, P, gs);
    memset(gm, 0, sizeof(double) * (size_t)(3 * P));
    memset(gls, 0, sizeof(double) * (size_t)(3 * P));
    memset(gq, 0, sizeof(double) * (size_t)(4 * P));
    memset(glogit, 0, sizeof(double) * (size_t)P);
    memset(gsh, 0, sizeof(double) * (size_t)(3 * nk) * (size_t)P);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t g = 0; g < P; ++g)
        if (ints[g * I_N + I_VALID])
            gauss_adjoint(sc, g, cam, W, H, op, gs + g * G_N, gm, gls, gq, glogit, gsh);
    if (gstate) memcpy(gstate, gs, sizeof(double) * (size_t)P * G_N);
    free(gs);
}
