// Per-pixel evaluation shared by the blend and its adjoint.  Both must take
// the same contribution and clamp decisions bit for bit, so the quadratic
// form and the alpha are written once, with explicit multiply-adds.
#pragma once

#include <hip/hip_runtime.h>

namespace fgs {

constexpr float kNegHalfLog2e = -0.72134752044448170f;  // -log2(e) / 2

// Conservative ellipse / rectangle test used only to skip work: the
// rectangle [X0, X1] x [Y0, Y1] in pixel-sample coordinates (Alg. 3 with the
// chord-overlap condition of Eq. 7).  Callers inflate k2 slightly so that no
// contributor is ever skipped.
__device__ __forceinline__ bool rect_hit(float u, float v, float A, float B, float C, float k2, float X0, float X1,
                                         float Y0, float Y1) {
    const float x0 = X0 - u, x1 = X1 - u, y0 = Y0 - v, y1 = Y1 - v;
    if (x0 <= 0.0f && 0.0f <= x1 && y0 <= 0.0f && 0.0f <= y1) return true;
    bool hit = false;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float ye_ = e ? y1 : y0;
        const float bq = 2.0f * B * ye_;
        const float cq = C * ye_ * ye_ - k2;
        const float delta = bq * bq - 4.0f * A * cq;
        const float e1 = 2.0f * A * x0 + bq, e2 = 2.0f * A * x1 + bq;
        hit |= (delta >= 0.0f) && (e1 <= 0.0f || e1 * e1 <= delta) && (e2 >= 0.0f || e2 * e2 <= delta);
    }
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const float xe_ = e ? x1 : x0;
        const float bq = 2.0f * B * xe_;
        const float cq = A * xe_ * xe_ - k2;
        const float delta = bq * bq - 4.0f * C * cq;
        const float e1 = 2.0f * C * y0 + bq, e2 = 2.0f * C * y1 + bq;
        hit |= (delta >= 0.0f) && (e1 <= 0.0f || e1 * e1 <= delta) && (e2 >= 0.0f || e2 * e2 <= delta);
    }
    return hit;
}

// q = A dx^2 + 2B dx dy + C dy^2 with twoB = 2B, as C dy^2 + dx (A dx + 2B dy).
__device__ __forceinline__ float conic_q(float A, float twoB, float C, float dx, float dy) {
    const float t = fmaf(A, dx, twoB * dy);
    return fmaf(C * dy, dy, dx * t);
}

// o exp(-q/2) = 2^(log2 o - q log2(e) / 2) (Sec. 5.3.2: exponent in log form),
// before the alpha_max clamp.
__device__ __forceinline__ float gauss_alpha(float q, float log2o) {
    return __builtin_amdgcn_exp2f(fmaf(q, kNegHalfLog2e, log2o));
}

}  // namespace fgs
