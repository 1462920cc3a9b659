// Per-pixel evaluation shared by the blend and its adjoint.  Both must take
// the same contribution and clamp decisions bit for bit, so the staged
// coefficients and the exponent are written once, with explicit multiply-adds.
#pragma once

#include <hip/hip_runtime.h>

#include "fgs_internal.hpp"

namespace fgs {

constexpr float kHalfLog2e = 0.72134752044448170f;  // log2(e) / 2

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

// Staged form of a Gaussian for the pixel loop.  With c = log2(e) / 2 the
// base-2 exponent of o exp(-q/2) is (Sec. 5.3.2, exponent in log form)
//     E = log2 o - c q = log2 o + A' dx^2 + B2' dx dy + C' dy^2,
// A' = -c A, B2' = -2 c B, C' = -c C, and the pixel lies in the opacity-aware
// extent (q <= k^2) iff E >= thr = log2 o - c k^2.
//   f0 = (u, v, A', B2')   f1 = (C', thr, log2 o, r)   f2 = (g, b)
__device__ __forceinline__ void stage_gauss(const GaussState &s, float4 &f0, float4 &f1, float2 &f2) {
    const float log2o = s.f1.z;
    f0 = make_float4(s.f0.x, s.f0.y, -kHalfLog2e * s.f0.z, -2.0f * kHalfLog2e * s.f0.w);
    f1 = make_float4(-kHalfLog2e * s.f1.x, fmaf(-kHalfLog2e, s.f1.y, log2o), log2o, s.f1.w);
    f2 = make_float2(s.f2.x, s.f2.y);
}

// Row terms shared by the pixels of one row (same dy).
struct RowTerms {
    float b2dy;  // B2' dy
    float base;  // C' dy^2 + log2 o
};

__device__ __forceinline__ RowTerms row_terms(const float4 &f0, const float4 &f1, float py) {
    const float dy = py - f0.y;
    RowTerms r;
    r.b2dy = f0.w * dy;
    r.base = fmaf(f1.x * dy, dy, f1.z);
    return r;
}

// E at pixel-sample x for the row terms r: dx (A' dx + B2' dy) + C' dy^2 + log2 o.
__device__ __forceinline__ float exponent_at(const float4 &f0, const RowTerms &r, float px) {
    const float dx = px - f0.x;
    return fmaf(dx, fmaf(f0.z, dx, r.b2dy), r.base);
}

}  // namespace fgs
