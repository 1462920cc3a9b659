// Real orthonormal spherical-harmonic basis (Condon-Shortley phase, index
// k = l^2 + l + m, degrees 0..3) and its gradient, for the view-dependent
// colour of each Gaussian.  The preprocess includes it in a translation unit
// built without multiply-add contraction, the backward in one built with it.
#pragma once

#include <hip/hip_runtime.h>

namespace fgs {

namespace shc {
constexpr float c0 = 0.28209479177387814f;    // 1 / (2 sqrt(pi))
constexpr float c1 = 0.48860251190291992f;    // sqrt(3 / (4 pi))
constexpr float c2a = 1.0925484305920792f;    // sqrt(15 / (4 pi))
constexpr float c20 = 0.31539156525252005f;   // sqrt(5 / (16 pi))
constexpr float c22 = 0.54627421529603959f;   // sqrt(15 / (16 pi))
constexpr float c33 = 0.59004358992664352f;   // sqrt(35 / (32 pi))
constexpr float c32 = 2.8906114426405538f;    // sqrt(105 / (4 pi))
constexpr float c31 = 0.45704579946446572f;   // sqrt(21 / (32 pi))
constexpr float c30 = 0.37317633259011546f;   // sqrt(7 / (16 pi))
constexpr float c32b = 1.4453057213202769f;   // sqrt(105 / (16 pi))
}  // namespace shc

// Y[k] for k < (D + 1)^2 at the unit direction (x, y, z).
__device__ __forceinline__ void sh_basis(float x, float y, float z, int D, float *Y) {
    using namespace shc;
    Y[0] = c0;
    if (D < 1) return;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    if (D < 2) return;
    const float xx = x * x, yy = y * y, zz = z * z;
    Y[4] = c2a * (x * y);
    Y[5] = -c2a * (y * z);
    Y[6] = c20 * (3.0f * zz - 1.0f);
    Y[7] = -c2a * (x * z);
    Y[8] = c22 * (xx - yy);
    if (D < 3) return;
    Y[9] = -c33 * (y * (3.0f * xx - yy));
    Y[10] = c32 * (x * y * z);
    Y[11] = -c31 * (y * (5.0f * zz - 1.0f));
    Y[12] = c30 * (z * (5.0f * zz - 3.0f));
    Y[13] = -c31 * (x * (5.0f * zz - 1.0f));
    Y[14] = c32b * (z * (xx - yy));
    Y[15] = -c33 * (x * (xx - 3.0f * yy));
}

// g = sum_k w[k] grad Y_k at (x, y, z), with each Y_k taken as the polynomial
// above on R^3.  Callers project g onto the tangent plane of the unit sphere
// (the direction is normalised), which removes the dependence on how the
// polynomials extend off the sphere.
__device__ __forceinline__ void sh_basis_grad(float x, float y, float z, int D, const float *w, float *g) {
    using namespace shc;
    float gx = 0.0f, gy = 0.0f, gz = 0.0f;
    if (D >= 1) {
        gy -= c1 * w[1];
        gz += c1 * w[2];
        gx -= c1 * w[3];
    }
    if (D >= 2) {
        gx += c2a * y * w[4];
        gy += c2a * x * w[4];
        gy -= c2a * z * w[5];
        gz -= c2a * y * w[5];
        gz += 6.0f * c20 * z * w[6];
        gx -= c2a * z * w[7];
        gz -= c2a * x * w[7];
        gx += 2.0f * c22 * x * w[8];
        gy -= 2.0f * c22 * y * w[8];
    }
    if (D >= 3) {
        const float xx = x * x, yy = y * y, zz = z * z;
        gx -= 6.0f * c33 * x * y * w[9];
        gy -= 3.0f * c33 * (xx - yy) * w[9];
        gx += c32 * y * z * w[10];
        gy += c32 * x * z * w[10];
        gz += c32 * x * y * w[10];
        gy -= c31 * (5.0f * zz - 1.0f) * w[11];
        gz -= 10.0f * c31 * y * z * w[11];
        gz += c30 * (15.0f * zz - 3.0f) * w[12];
        gx -= c31 * (5.0f * zz - 1.0f) * w[13];
        gz -= 10.0f * c31 * x * z * w[13];
        gx += 2.0f * c32b * x * z * w[14];
        gy -= 2.0f * c32b * y * z * w[14];
        gz += c32b * (xx - yy) * w[14];
        gx -= 3.0f * c33 * (xx - yy) * w[15];
        gy += 6.0f * c33 * x * y * w[15];
    }
    g[0] = gx;
    g[1] = gy;
    g[2] = gz;
}

}  // namespace fgs
