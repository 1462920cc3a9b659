/*
 * Types shared by the oracle's translation units (test infrastructure only;
 * never included by the product library).  The including file defines REAL
 * (float or double) and TYPE(name) (name_f32 / name_f64) first.  The struct
 * typedefs may be included once per (REAL, TYPE) pair in one file; the state
 * indices once in all.
 */
#include <stdint.h>

/* ---- inputs ------------------------------------------------------------ */

/* Gaussian parameters (Alg. 1 / Alg. 4 inputs), planar: plane c of an
 * attribute lives at ptr + c * stride.  sh has 3 (D+1)^2 planes, plane
 * 3 k + channel, k = l^2 + l + m. */
typedef struct {
    int64_t P, stride;
    int32_t D, pad_;
    const REAL *means, *log_scales, *quats, *logits, *sh;
} TYPE(orc_scene);

/* world -> camera x_cam = R x + t (row-major R); camera x right, y down,
 * z forward; eye = camera centre in world; focal lengths and principal point
 * in pixels. */
typedef struct {
    REAL R[9], t[3], eye[3];
    REAL fx, fy, cx, cy, near_z;
} TYPE(orc_camera);

typedef struct {
    REAL alpha_min; /* tau = 1/255 (Sec. 4.1) */
    REAL T_stop;    /* 1e-4 */
    REAL alpha_max; /* 0.99, reading */
    REAL dilation;  /* 0.3 px^2, reading */
    REAL jac_clip;  /* 1.3, reading */
    REAL bg[3];
    int32_t cap_3sigma; /* 1: k^2 = min(9, 2 ln(o/tau)) (Sec. 4.1) */
    int32_t binning;    /* 0 exact (Alg. 3), 1 tight box only, 2 3 sigma square box (Alg. 1) */
} TYPE(orc_options);

/* ---- per-Gaussian state ------------------------------------------------ */
#ifndef ORC_STATE_INDICES
#define ORC_STATE_INDICES

enum {
    S_U, S_V, S_A, S_B, S_C, S_K2, S_O, S_DEPTH, S_R, S_G, S_BL,
    S_COVA, S_COVB, S_COVC, S_HX, S_HY, S_N = 16
};
enum { I_VALID, I_COUNT, I_I0, I_I1, I_J0, I_J1, I_TX0, I_TX1, I_TY0, I_TY1, I_N = 10 };

#endif
