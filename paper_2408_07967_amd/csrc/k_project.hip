// Per-Gaussian preprocessing with the exact ellipse/tile test, and key
// emission in depth order (FlashGS Alg. 4, Alg. 3, Eq. 1-3, Eq. 7, Sec. 4.2).
//
// This translation unit is compiled with -ffp-contract=off: every binary32
// + - * / and sqrt below is one correctly rounded IEEE operation in the
// written order, so the per-Gaussian state and the tile test give the same
// bits as the canonical FP32 evaluation of the method; exp and ln are
// evaluated in binary64 by a fixed operation sequence and rounded once.
#include <algorithm>

#include "fgs_internal.hpp"
#include "sh_basis.hpp"

namespace fgs {
namespace {

constexpr int kWave = 64;

// ---- canonical binary64 exp / ln (Cody-Waite reduction + Taylor; atanh series)

#define FGS_LN2_HI 0x1.62e42fee00000p-1
#define FGS_LN2_LO 0x1.a39ef35793c76p-33
#define FGS_INV_LN2 0x1.71547652b82fep+0

__device__ __forceinline__ double pow2i(int k) {
    return __longlong_as_double((long long)(k + 1023) << 52);
}

__device__ __forceinline__ double floor_exact(double x) {
    double t = (double)(long long)x;
    return (t > x) ? t - 1.0 : t;
}

__device__ double canon_exp(double x) {
    if (x != x) return x;
    if (x > 709.8) return __longlong_as_double(0x7ff0000000000000LL);
    if (x < -745.2) return 0.0;
    double k = floor_exact(x * FGS_INV_LN2 + 0.5);
    double r = (x - k * FGS_LN2_HI) - k * FGS_LN2_LO;
    double p = 1.0 / 6227020800.0;
    p = p * r + 1.0 / 479001600.0;
    p = p * r + 1.0 / 39916800.0;
    p = p * r + 1.0 / 3628800.0;
    p = p * r + 1.0 / 362880.0;
    p = p * r + 1.0 / 40320.0;
    p = p * r + 1.0 / 5040.0;
    p = p * r + 1.0 / 720.0;
    p = p * r + 1.0 / 120.0;
    p = p * r + 1.0 / 24.0;
    p = p * r + 1.0 / 6.0;
    p = p * r + 0.5;
    p = p * r + 1.0;
    p = p * r + 1.0;
    int ki = (int)k;
    int k1 = ki / 2;
    int k2 = ki - k1;
    return (p * pow2i(k1)) * pow2i(k2);
}

// ln x for finite x >= 1 (the only use: ln(o / tau) with o > tau)
__device__ double canon_log(double x) {
    unsigned long long bits = (unsigned long long)__double_as_longlong(x);
    int e = (int)((bits >> 52) & 0x7ff) - 1023;
    double m = __longlong_as_double((long long)((bits & 0x000fffffffffffffULL) | 0x3ff0000000000000ULL));
    if (m > 1.4142135623730951) {
        m = m * 0.5;
        e = e + 1;
    }
    double s = (m - 1.0) / (m + 1.0);
    double z = s * s;
    double p = 1.0 / 23.0;
    p = p * z + 1.0 / 21.0;
    p = p * z + 1.0 / 19.0;
    p = p * z + 1.0 / 17.0;
    p = p * z + 1.0 / 15.0;
    p = p * z + 1.0 / 13.0;
    p = p * z + 1.0 / 11.0;
    p = p * z + 1.0 / 9.0;
    p = p * z + 1.0 / 7.0;
    p = p * z + 1.0 / 5.0;
    p = p * z + 1.0 / 3.0;
    double lnm = (2.0 * s) + (2.0 * s) * (z * p);
    double de = (double)e;
    return de * FGS_LN2_HI + (lnm + de * FGS_LN2_LO);
}

__device__ __forceinline__ float clampf_(float x, float lo, float hi) {
    return x < lo ? lo : (x > hi ? hi : x);
}

__device__ __forceinline__ float bcast(float x, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}
__device__ __forceinline__ int bcast(int x, int lane) { return __builtin_amdgcn_readlane(x, lane); }
__device__ __forceinline__ uint32_t bcast(uint32_t x, int lane) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, lane);
}

// Exact test of the ellipse { d : A dx^2 + 2 B dx dy + C dy^2 <= k2 } around
// (u, v) against the pixel-sample hull of tile (tx, ty) (Alg. 3; Eq. 7 with
// the discriminant guard).  Centre inside -> hit; otherwise each edge line
// meets the ellipse in a chord whose overlap with the edge segment is decided
// without division or square root.
//
// The test splits into terms of the tile's column alone and of its row alone,
// so that the tiles of one rectangle can share them; tile_hit is the two
// halves combined, with the same binary32 operations in the same order.
//
// Column terms (hull x-range [x0, x1] relative to u):
//   a = (2A x0, 2A x1, bq(x0), delta(x0)), b = (bq(x1), delta(x1), flag, 0)
// with bq(x) = 2B x and delta(x) = bq^2 - 4C (A x^2 - k2) for the vertical
// edge at x (quadratic in y), and flag = 1 if x0 <= 0 <= x1.
__device__ __forceinline__ void tile_col_terms(float u, float A, float B, float C, float k2, int tx, int W,
                                               float4 &a, float4 &b) {
    int xe = kTile * tx + kTile;
    xe = xe > W ? W : xe;
    const float x0 = ((float)(kTile * tx) + 0.5f) - u;
    const float x1 = ((float)xe - 0.5f) - u;
    const float A2 = 2.0f * A, B2 = 2.0f * B, C4 = 4.0f * C;
    const float bq0 = B2 * x0, bq1 = B2 * x1;
    const float cq0 = (A * x0) * x0 - k2, cq1 = (A * x1) * x1 - k2;
    a = make_float4(A2 * x0, A2 * x1, bq0, bq0 * bq0 - C4 * cq0);
    b = make_float4(bq1, bq1 * bq1 - C4 * cq1, (x0 <= 0.0f && 0.0f <= x1) ? 1.0f : 0.0f, 0.0f);
}

// Row terms (hull y-range [y0, y1] relative to v):
//   a = (bq(y0), delta(y0), bq(y1), delta(y1)), b = (2C y0, 2C y1, flag, 0)
// with bq(y) = 2B y and delta(y) = bq^2 - 4A (C y^2 - k2) for the horizontal
// edge at y (quadratic in x), and flag = 1 if y0 <= 0 <= y1.
__device__ __forceinline__ void tile_row_terms(float v, float A, float B, float C, float k2, int ty, int H,
                                               float4 &a, float4 &b) {
    int ye = kTile * ty + kTile;
    ye = ye > H ? H : ye;
    const float y0 = ((float)(kTile * ty) + 0.5f) - v;
    const float y1 = ((float)ye - 0.5f) - v;
    const float B2 = 2.0f * B, C2 = 2.0f * C, A4 = 4.0f * A;
    const float bq0 = B2 * y0, bq1 = B2 * y1;
    const float cq0 = (C * y0) * y0 - k2, cq1 = (C * y1) * y1 - k2;
    a = make_float4(bq0, bq0 * bq0 - A4 * cq0, bq1, bq1 * bq1 - A4 * cq1);
    b = make_float4(C2 * y0, C2 * y1, (y0 <= 0.0f && 0.0f <= y1) ? 1.0f : 0.0f, 0.0f);
}

// One edge: the chord [r-, r+] of the quadratic with discriminant d overlaps
// the edge segment, given e1 = 2a s0 + bq and e2 = 2a s1 + bq at its ends.
// (Bitwise, not short-circuit, so that the test compiles to straight-line
// code.)
__device__ __forceinline__ bool edge_hit(float e1, float e2, float d) {
    return (d >= 0.0f) & ((e1 <= 0.0f) | (e1 * e1 <= d)) & ((e2 >= 0.0f) | (e2 * e2 <= d));
}

__device__ __forceinline__ bool tile_hit_terms(const float4 ca, const float4 cb, const float4 ra, const float4 rb) {
    const bool inside = (cb.z != 0.0f) & (rb.z != 0.0f);  // centre inside the hull
    // horizontal edges y = y0, y1, then vertical edges x = x0, x1
    return inside | edge_hit(ca.x + ra.x, ca.y + ra.x, ra.y) | edge_hit(ca.x + ra.z, ca.y + ra.z, ra.w) |
           edge_hit(rb.x + ca.z, rb.y + ca.z, ca.w) | edge_hit(rb.x + cb.x, rb.y + cb.x, cb.y);
}

__device__ __forceinline__ bool tile_hit(float u, float v, float A, float B, float C, float k2, int tx, int ty,
                                         int W, int H) {
    float4 ca, cb, ra, rb;
    tile_col_terms(u, A, B, C, k2, tx, W, ca, cb);
    tile_row_terms(v, A, B, C, k2, ty, H, ra, rb);
    return tile_hit_terms(ca, cb, ra, rb);
}

// Row and column of row-major position idx in rows of ntx (idx < 2^24,
// rcpn = reciprocal of ntx): the rounded quotient estimate is off by at most
// one and is corrected, so this equals integer division.
__device__ __forceinline__ void row_col(int idx, int ntx, float rcpn, int &ry, int &rx) {
    ry = (int)((float)idx * rcpn);
    rx = idx - ry * ntx;
    const int below = rx < 0, above = rx >= ntx;
    ry += above - below;
    rx += (below - above) * ntx;
}

// (tx0, tx1, ty0, ty1) of an emission record's packed rectangle
__device__ __forceinline__ uint4 unpack_rect(const uint4 &r) {
    return make_uint4(r.x & 0xffffu, r.x >> 16, r.y & 0xffffu, r.y >> 16);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, d, kWave);
        if (lane >= d) x += y;
    }
    return x;
}

// Largest lane L with s[L] <= item, for s non-decreasing over 64 lanes with
// s[0] = 0: the owner of flattened item `item` (lanes with no items are
// skipped because the next lane has the same start).
__device__ __forceinline__ int owner_lane(const uint32_t *s, uint32_t item) {
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1)
        if (s[lo + step] <= item) lo += step;
    return lo;
}

// k / n for 0 <= k < 64 and 1 <= n <= 64: (k + 1/2) / n is at least 1/128
// away from an integer, far more than the reciprocal's error.
__device__ __forceinline__ int small_div(uint32_t k, int n) {
    return (int)(((float)k + 0.5f) * __builtin_amdgcn_rcpf((float)n));
}

// Scales exp(log-scale) and the unit quaternion q / |q| (computeCov3D's
// inputs), as the binary32 values of the canonical evaluation.  False for a
// non-finite scale or a quaternion of zero or non-finite norm.
__device__ __forceinline__ bool scale_rot(float ls0, float ls1, float ls2, const float *q4, float *s3, float *qu) {
    const float qw = q4[0], qx = q4[1], qy = q4[2], qz = q4[3];
    s3[0] = (float)canon_exp((double)ls0);
    s3[1] = (float)canon_exp((double)ls1);
    s3[2] = (float)canon_exp((double)ls2);
    const float n2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    const bool fin = isfinite(ls0) && isfinite(ls1) && isfinite(ls2) && isfinite(n2);
    if (!(fin && n2 > 0.0f)) return false;
    const float qn = sqrtf(n2);
    qu[0] = qw / qn;
    qu[1] = qx / qn;
    qu[2] = qy / qn;
    qu[3] = qz / qn;
    return true;
}

// 3D covariance Sigma = M M^T with M = R(q) diag(s) (computeCov3D), upper
// triangle S00, S01, S02, S11, S12, S22, in binary32.
__device__ __forceinline__ void sigma3(const float *s3, const float *qu, float *S) {
    const float s0 = s3[0], s1 = s3[1], s2 = s3[2];
    const float w = qu[0], x = qu[1], y = qu[2], z = qu[3];
    const float r00 = 1.0f - 2.0f * (y * y + z * z);
    const float r01 = 2.0f * (x * y - w * z);
    const float r02 = 2.0f * (x * z + w * y);
    const float r10 = 2.0f * (x * y + w * z);
    const float r11 = 1.0f - 2.0f * (x * x + z * z);
    const float r12 = 2.0f * (y * z - w * x);
    const float r20 = 2.0f * (x * z - w * y);
    const float r21 = 2.0f * (y * z + w * x);
    const float r22 = 1.0f - 2.0f * (x * x + y * y);
    const float M00 = r00 * s0, M01 = r01 * s1, M02 = r02 * s2;
    const float M10 = r10 * s0, M11 = r11 * s1, M12 = r12 * s2;
    const float M20 = r20 * s0, M21 = r21 * s1, M22 = r22 * s2;
    S[0] = (M00 * M00 + M01 * M01) + M02 * M02;
    S[1] = (M00 * M10 + M01 * M11) + M02 * M12;
    S[2] = (M00 * M20 + M01 * M21) + M02 * M22;
    S[3] = (M10 * M10 + M11 * M11) + M12 * M12;
    S[4] = (M10 * M20 + M11 * M21) + M12 * M22;
    S[5] = (M20 * M20 + M21 * M21) + M22 * M22;
}

// Conic of the dilated EWA covariance in binary64, rounded once to binary32
// (the blend's conic, see GaussState).  The inputs are the binary32 scales,
// unit quaternion, mean and camera, promoted to binary64 (c: the camera and
// its Jacobian clamp limits in binary64); the Jacobian clamp is the same.
// With M = R(q) diag(s) and T = J R_cam, Sigma' = T M M^T T^T + dilation I =
// N N^T + dilation I for N = T M, accumulated one column of M at a time (the
// product the canonical evaluation forms as T Sigma T^T).  The binary32
// determinant of Sigma' cancels badly for long thin footprints; in binary64
// the narrow axis keeps its accuracy.  False if the binary64 determinant is
// not positive.
__device__ bool conic_b64(const float *s3, const float *qu, float mx, float my, float mz, const DevCam64 &c,
                          double dil, float *Ab, float *Bb, float *Cb) {
    const double px = mx, py = my, pz = mz;
    const double tx = c.R[0] * px + c.R[1] * py + c.R[2] * pz + c.t[0];
    const double ty = c.R[3] * px + c.R[4] * py + c.R[5] * pz + c.t[1];
    const double tz = c.R[6] * px + c.R[7] * py + c.R[8] * pz + c.t[2];
    const double iz = 1.0 / tz;
    double xc = tx * iz, yc = ty * iz;
    xc = xc < -c.limx ? -c.limx : (xc > c.limx ? c.limx : xc);
    yc = yc < -c.limy ? -c.limy : (yc > c.limy ? c.limy : yc);
    const double J00 = c.fx * iz, J02 = -(c.fx * xc) * iz, J11 = c.fy * iz, J12 = -(c.fy * yc) * iz;
    double T0[3], T1[3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        T0[j] = J00 * c.R[j] + J02 * c.R[6 + j];
        T1[j] = J11 * c.R[3 + j] + J12 * c.R[6 + j];
    }
    const double w = qu[0], x = qu[1], y = qu[2], z = qu[3];
    double a = 0.0, b = 0.0, cc = 0.0;
    auto column = [&](double r0, double r1, double r2, double sj) {
        const double n0 = (T0[0] * r0 + T0[1] * r1 + T0[2] * r2) * sj;
        const double n1 = (T1[0] * r0 + T1[1] * r1 + T1[2] * r2) * sj;
        a += n0 * n0;
        b += n0 * n1;
        cc += n1 * n1;
    };
    column(1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y + w * z), 2.0 * (x * z - w * y), (double)s3[0]);
    column(2.0 * (x * y - w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z + w * x), (double)s3[1]);
    column(2.0 * (x * z + w * y), 2.0 * (y * z - w * x), 1.0 - 2.0 * (x * x + y * y), (double)s3[2]);
    a += dil;
    cc += dil;
    const double det = a * cc - b * b;
    if (!(det > 0.0)) return false;
    const double inv = 1.0 / det;
    *Ab = (float)(cc * inv);
    *Bb = (float)(-b * inv);
    *Cb = (float)(a * inv);
    return true;
}

// Opacity-aware extent (Eq. 3), capped by the 3 sigma rule (Eq. 1).
__device__ __forceinline__ float extent_k2(float o, const DevOptions &op) {
    double k2d = 2.0 * canon_log((double)o / (double)op.alpha_min);
    if (op.cap_3sigma && k2d > 9.0) k2d = 9.0;
    return (float)k2d;
}

// View-independent precompute of a resident scene (Sec. 5.3.1: preprocessing
// shared by the viewpoints of one scene): per Gaussian (x, y, z, opacity) with
// opacity 0 for a Gaussian that can never be visible, the scales, the unit
// quaternion and k^2, the trace of the 3D covariance with k^2 (the cull's
// extent bound), and the SH coefficients Gaussian-major.  The same operations
// as the per-frame path, so frames render bit for bit the same.  Slot i holds
// Gaussian perm[i] (a spatial order, so that the candidates of a frame's cull
// are read as few contiguous runs), and orig[i] = perm[i].
__global__ __launch_bounds__(kBlock) void k_prepare(DevScene sc, DevOptions op, const uint32_t *__restrict__ perm,
                                                    float4 *__restrict__ pos_o, float4 *__restrict__ cov,
                                                    float *__restrict__ sh_out, float2 *__restrict__ bnd,
                                                    uint32_t *__restrict__ orig, int sh_stride) {
    const int64_t st = sc.stride;
    const int ncoef = 3 * (sc.D + 1) * (sc.D + 1);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < sc.P;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t g = perm[i];
        orig[i] = (uint32_t)g;
        const float mx = sc.means[g], my = sc.means[st + g], mz = sc.means[2 * st + g];
        const float logit = sc.logits[g];
        const float o = (float)(1.0 / (1.0 + canon_exp(-(double)logit)));
        float S[6] = {0, 0, 0, 0, 0, 0}, s3[3] = {0, 0, 0}, qu[4] = {0, 0, 0, 0};
        float k2 = 0.0f;
        bool ok = isfinite(logit) && o > op.alpha_min;
        if (ok) {
            const float q4[4] = {sc.quats[g], sc.quats[st + g], sc.quats[2 * st + g], sc.quats[3 * st + g]};
            ok = scale_rot(sc.log_scales[g], sc.log_scales[st + g], sc.log_scales[2 * st + g], q4, s3, qu);
        }
        if (ok) {
            sigma3(s3, qu, S);
            k2 = extent_k2(o, op);
        }
        pos_o[i] = make_float4(mx, my, mz, ok ? o : 0.0f);
        cov[2 * i] = make_float4(s3[0], s3[1], s3[2], k2);
        cov[2 * i + 1] = make_float4(qu[0], qu[1], qu[2], qu[3]);
        // trace(Sigma) >= its largest eigenvalue: bounds the screen extent
        bnd[i] = make_float2(S[0] + S[3] + S[5], k2);
    }
    // SH: planar in, Gaussian-major out, transposed through LDS so that the
    // writes (the workgroup's slots, one contiguous range) are coalesced
    __shared__ float s_t[kBlock * (48 + 1)];
    for (int64_t i0 = (int64_t)blockIdx.x * kBlock; i0 < sc.P; i0 += (int64_t)gridDim.x * kBlock) {
        const int64_t i = i0 + threadIdx.x;
        const int n = sc.P - i0 < kBlock ? (int)(sc.P - i0) : kBlock;
        const int64_t g = i < sc.P ? (int64_t)perm[i] : 0;
        __syncthreads();
        for (int j = 0; j < sh_stride; ++j)
            s_t[threadIdx.x * (48 + 1) + j] = (j < ncoef && i < sc.P) ? sc.sh[(int64_t)j * st + g] : 0.0f;
        __syncthreads();
        float *dst = sh_out + i0 * sh_stride;
        for (int e = threadIdx.x; e < n * sh_stride; e += kBlock) {
            const int r = e / sh_stride, j = e - r * sh_stride;
            dst[e] = s_t[r * (48 + 1) + j];
        }
    }
}

// A binary32 value as an unsigned integer of the same order (for atomic
// min / max), and back.
__device__ __forceinline__ uint32_t float_order(float f) {
    const uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float order_float(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// Box of the finite means: per workgroup a reduction over its Gaussians,
// then one atomic min / max per axis into bounds (order-mapped, see
// float_order).
__global__ __launch_bounds__(kBlock) void k_spatial_bounds(DevScene sc, uint32_t *__restrict__ bounds) {
    const int64_t st = sc.stride;
    uint32_t lo[3] = {0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[3] = {0u, 0u, 0u};
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < sc.P; g += (int64_t)gridDim.x * blockDim.x) {
        const float m[3] = {sc.means[g], sc.means[st + g], sc.means[2 * st + g]};
        if (!(isfinite(m[0]) && isfinite(m[1]) && isfinite(m[2]))) continue;
        for (int a = 0; a < 3; ++a) {
            const uint32_t u = float_order(m[a]);
            lo[a] = u < lo[a] ? u : lo[a];
            hi[a] = u > hi[a] ? u : hi[a];
        }
    }
    __shared__ uint32_t s_lo[3][kBlock / kWave], s_hi[3][kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int a = 0; a < 3; ++a) {
        uint32_t l = lo[a], h = hi[a];
        for (int d = kWave / 2; d > 0; d >>= 1) {
            const uint32_t l2 = (uint32_t)__shfl_xor((int)l, d, kWave), h2 = (uint32_t)__shfl_xor((int)h, d, kWave);
            l = l2 < l ? l2 : l;
            h = h2 > h ? h2 : h;
        }
        if (lane == 0) {
            s_lo[a][wave] = l;
            s_hi[a][wave] = h;
        }
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const int a = threadIdx.x;
        uint32_t l = 0xffffffffu, h = 0u;
        for (int w = 0; w < kBlock / kWave; ++w) {
            l = s_lo[a][w] < l ? s_lo[a][w] : l;
            h = s_hi[a][w] > h ? s_hi[a][w] : h;
        }
        if (l != 0xffffffffu) atomicMin(&bounds[a], l);
        if (h != 0u) atomicMax(&bounds[3 + a], h);
    }
}

__global__ void k_spatial_bounds_init(uint32_t *bounds) {
    if (threadIdx.x < 6) bounds[threadIdx.x] = threadIdx.x < 3 ? 0xffffffffu : 0u;
}

// Ten bits of x spread to every third bit (bit b to bit 3b).
__device__ __forceinline__ uint32_t spread3(uint32_t x) {
    x &= 0x3ffu;
    x = (x | (x << 16)) & 0x030000ffu;
    x = (x | (x << 8)) & 0x0300f00fu;
    x = (x | (x << 4)) & 0x030c30c3u;
    x = (x | (x << 2)) & 0x09249249u;
    return x;
}

// Morton code of each mean quantised to 1024 cells per axis of the box.
__global__ __launch_bounds__(kBlock) void k_spatial_keys(DevScene sc, const uint32_t *__restrict__ bounds,
                                                         uint32_t *__restrict__ keys) {
    const int64_t st = sc.stride;
    float lo[3], sc3[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = order_float(bounds[a]);
        const float ext = order_float(bounds[3 + a]) - lo[a];
        sc3[a] = ext > 0.0f ? 1024.0f / ext : 0.0f;
    }
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < sc.P; g += (int64_t)gridDim.x * blockDim.x) {
        const float m[3] = {sc.means[g], sc.means[st + g], sc.means[2 * st + g]};
        uint32_t key = 0xffffffffu;
        if (isfinite(m[0]) && isfinite(m[1]) && isfinite(m[2]) && bounds[0] != 0xffffffffu) {
            uint32_t q[3];
            for (int a = 0; a < 3; ++a) {
                const float c = (m[a] - lo[a]) * sc3[a];
                q[a] = c <= 0.0f ? 0u : (c >= 1023.0f ? 1023u : (uint32_t)c);
            }
            key = spread3(q[0]) | (spread3(q[1]) << 1) | (spread3(q[2]) << 2);
        }
        keys[g] = key;
    }
}

// Gaussians [lo, hi) of cull workgroup b of kCullBlocks: whole 256-Gaussian
// batches split evenly.
__device__ __forceinline__ void cull_range(int64_t P, uint32_t b, int64_t *lo, int64_t *hi) {
    const int64_t batches = (P + kBlock - 1) / kBlock;
    *lo = batches * b / kCullBlocks * kBlock;
    const int64_t h = batches * (b + 1) / kCullBlocks * kBlock;
    *hi = h < P ? h : P;
    if (*lo > *hi) *lo = *hi;
}

// The cull's keep test of one Gaussian (position and opacity p4, extent
// terms b) for one camera.  Evaluated without branches, so that a caller's
// loads of p4 and b are all issued together.
__device__ __forceinline__ bool cull_keep(const float4 &p4, const float2 &b, const DevCamera &cam,
                                          const DevOptions &op, int W, int H) {
    const float *R = cam.R;
    const float tx = ((R[0] * p4.x + R[1] * p4.y) + R[2] * p4.z) + cam.t[0];
    const float ty = ((R[3] * p4.x + R[4] * p4.y) + R[5] * p4.z) + cam.t[1];
    const float tz = ((R[6] * p4.x + R[7] * p4.y) + R[8] * p4.z) + cam.t[2];
    const bool front = (tz > cam.near_z) & (p4.w > op.alpha_min) & isfinite(p4.x) & isfinite(p4.y) & isfinite(p4.z);
    const float iz = 1.0f / tz;
    const float xt = tx * iz, yt = ty * iz;
    const float limx = op.jac_clip * (0.5f * (float)W / cam.fx);
    const float limy = op.jac_clip * (0.5f * (float)H / cam.fy);
    const float xc = fminf(fmaxf(xt, -limx), limx), yc = fminf(fmaxf(yt, -limy), limy);
    const float J00 = cam.fx * iz, J02 = -cam.fx * xc * iz, J11 = cam.fy * iz, J12 = -cam.fy * yc * iz;
    float n0 = 0.0f, n1 = 0.0f;
    for (int j = 0; j < 3; ++j) {
        const float t0 = J00 * R[j] + J02 * R[6 + j], t1 = J11 * R[3 + j] + J12 * R[6 + j];
        n0 += t0 * t0;
        n1 += t1 * t1;
    }
    float hx, hy;
    if (op.binning == 2) {
        // square of radius ceil(3 sqrt(lambda_max(Sigma'))), lambda_max <= trace
        hx = sqrtf(9.0f * ((n0 + n1) * b.x + op.dilation)) * 1.001f + 3.0f;
        hy = hx;
    } else {
        hx = sqrtf(b.y * (n0 * b.x + op.dilation)) * 1.001f + 3.0f;
        hy = sqrtf(b.y * (n1 * b.x + op.dilation)) * 1.001f + 3.0f;
    }
    const float u = cam.fx * xt + cam.cx, v = cam.fy * yt + cam.cy;
    // drop only what is certainly off the image (a NaN keeps it)
    const bool out = (u + hx < 0.0f) | (u - hx > (float)W) | (v + hy < 0.0f) | (v - hy > (float)H);
    return front & !out;
}

// Whether the cull would drop every member of a batch whose bounds are
// (lo, hi, kx) (DevPrepared::blk), for one camera.  A member is dropped if
// its opacity is at most alpha_min, its view depth is not past the near
// plane, or its screen extent bound is off the image (cull_keep).  Over the
// batch: the opacity is at most lo.w; the view depth is affine in the mean,
// so over the box of means it lies between the corners' depths; in front of
// the camera the projection is linear-fractional with a positive
// denominator, so the means' screen coordinates also lie between the
// corners'; and each member's extent bound sqrt(k^2 (|t0|^2 trace +
// dilation)) grows with k^2, trace and |t0|^2 = (fx / z)^2 |R_0 - xc R_2|^2
// <= (fx / z_min)^2 (|R_0| + limx |R_2|)^2 (|xc| <= limx; the 3 sigma square
// likewise).  Margins (a relative 1e-5 on the depths, 1 % and 8 pixels on
// the extent) cover the rounding of either evaluation.
__device__ bool batch_culled(const float4 &lo, const float4 &hi, const float4 &kx, const DevCamera &cam,
                             const DevOptions &op, int W, int H) {
    if (!(lo.w > op.alpha_min)) return true;  // every opacity too low (or no member)
    const float *R = cam.R;
    bool behind = true, front = true;
    float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY, zmin = INFINITY;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const float x = (c & 1) ? hi.x : lo.x, y = (c & 2) ? hi.y : lo.y, z = (c & 4) ? hi.z : lo.z;
        const float tx = ((R[0] * x + R[1] * y) + R[2] * z) + cam.t[0];
        const float ty = ((R[3] * x + R[4] * y) + R[5] * z) + cam.t[1];
        const float tz = ((R[6] * x + R[7] * y) + R[8] * z) + cam.t[2];
        const float mag = ((fabsf(R[6] * x) + fabsf(R[7] * y)) + fabsf(R[8] * z)) + fabsf(cam.t[2]);
        behind = behind && tz < cam.near_z - 1e-5f * mag;
        front = front && tz > 1e-5f * mag && tz > 1e-20f;
        const float iz = 1.0f / tz;
        umin = fminf(umin, cam.fx * (tx * iz) + cam.cx);
        umax = fmaxf(umax, cam.fx * (tx * iz) + cam.cx);
        vmin = fminf(vmin, cam.fy * (ty * iz) + cam.cy);
        vmax = fmaxf(vmax, cam.fy * (ty * iz) + cam.cy);
        zmin = fminf(zmin, tz);
    }
    if (behind) return true;   // every member's depth is at most the near plane
    if (!front) return false;  // the box reaches behind the camera: test each member
    const float r0 = sqrtf((R[0] * R[0] + R[1] * R[1]) + R[2] * R[2]);
    const float r1 = sqrtf((R[3] * R[3] + R[4] * R[4]) + R[5] * R[5]);
    const float r2 = sqrtf((R[6] * R[6] + R[7] * R[7]) + R[8] * R[8]);
    const float limx = op.jac_clip * (0.5f * (float)W / cam.fx);
    const float limy = op.jac_clip * (0.5f * (float)H / cam.fy);
    const float ax = (cam.fx / zmin) * (r0 + limx * r2), ay = (cam.fy / zmin) * (r1 + limy * r2);
    const float n0 = ax * ax, n1 = ay * ay;
    float hx, hy;
    if (op.binning == 2) {
        hx = sqrtf(9.0f * ((n0 + n1) * hi.w + op.dilation));
        hy = hx;
    } else {
        hx = sqrtf(kx.x * (n0 * hi.w + op.dilation));
        hy = sqrtf(kx.x * (n1 * hi.w + op.dilation));
    }
    hx = hx * 1.01f + 8.0f;
    hy = hy * 1.01f + 8.0f;
    // (a NaN anywhere keeps the batch)
    return (umax + hx < 0.0f) || (umin - hx > (float)W) || (vmax + hy < 0.0f) || (vmin - hy > (float)H);
}

// Bounds of each batch of kBlock slots (one workgroup per batch) over its
// members that can be visible (see DevPrepared::blk).
__global__ __launch_bounds__(kBlock) void k_block_bounds(const float4 *__restrict__ pos_o,
                                                         const float2 *__restrict__ bnd, int64_t P,
                                                         float4 *__restrict__ blk) {
    __shared__ float s_r[kBlock / kWave][8];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    float4 p = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    float2 b = make_float2(0.0f, 0.0f);
    if (i < P) {
        p = pos_o[i];
        b = bnd[i];
    }
    const bool use = i < P && p.w > 0.0f && isfinite(p.x) && isfinite(p.y) && isfinite(p.z);
    // maxima as minima of negatives (a slot without a member adds +inf to
    // every minimum); a NaN trace or k^2 counts as +inf
    float r[8] = {use ? p.x : INFINITY, use ? p.y : INFINITY, use ? p.z : INFINITY,
                  use ? -p.x : INFINITY, use ? -p.y : INFINITY, use ? -p.z : INFINITY,
                  use ? -p.w : INFINITY, 0.0f};
    const float tr = isnan(b.x) ? INFINITY : b.x, k2 = isnan(b.y) ? INFINITY : b.y;
    float mtr = use ? tr : 0.0f, mk2 = use ? k2 : 0.0f;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
#pragma unroll
        for (int q = 0; q < 7; ++q) r[q] = fminf(r[q], __shfl_xor(r[q], d, kWave));
        mtr = fmaxf(mtr, __shfl_xor(mtr, d, kWave));
        mk2 = fmaxf(mk2, __shfl_xor(mk2, d, kWave));
    }
    r[7] = mtr;
    if (lane == 0) {
        for (int q = 0; q < 7; ++q) s_r[wv][q] = r[q];
        s_r[wv][7] = mtr;
    }
    __shared__ float s_k2[kBlock / kWave];
    if (lane == 0) s_k2[wv] = mk2;
    __syncthreads();
    if (threadIdx.x == 0) {
        float o[8];
        float k2m = s_k2[0];
        for (int q = 0; q < 8; ++q) o[q] = s_r[0][q];
        for (int w = 1; w < kBlock / kWave; ++w) {
            for (int q = 0; q < 7; ++q) o[q] = fminf(o[q], s_r[w][q]);
            o[7] = fmaxf(o[7], s_r[w][7]);
            k2m = fmaxf(k2m, s_k2[w]);
        }
        blk[3 * blockIdx.x] = make_float4(o[0], o[1], o[2], -o[6]);
        blk[3 * blockIdx.x + 1] = make_float4(-o[3], -o[4], -o[5], o[7]);
        blk[3 * blockIdx.x + 2] = make_float4(k2m, 0.0f, 0.0f, 0.0f);
    }
}

// Cull of a prepared scene: reads 24 bytes per Gaussian and keeps those in
// front of the near plane, above the opacity threshold and whose extent may
// reach a pixel sample.  The extent test is conservative: Sigma'_xx =
// t0^T Sigma t0 <= |t0|^2 trace(Sigma) for the row t0 of T = J R_cam, so
// sqrt(k^2 (|t0|^2 trace + dilation)) (or the 3 sigma radius plus one for the
// square box) bounds the half-width of the box, and a 0.1 % + 3 px margin
// covers rounding.  Everything it drops the exact path would cull too.
// kMulti: the union over the cameras of mo, whose counters it clears.  Each
// workgroup owns a contiguous range of Gaussians and lists its candidates in
// index order at the start of that range (no global atomics).
template <bool kMulti>
__global__ __launch_bounds__(kBlock) void k_cull(DevScene sc, DevPrepared pp, DevCamera cam, DevOptions op, int W,
                                                 int H, uint32_t *__restrict__ cand, uint32_t *__restrict__ seg_count,
                                                 FrameCounters *fc, MultiOut mo) {
    __shared__ uint32_t s_w[kBlock / kWave];
    // the frame's counters start at zero (the preprocess, next on the
    // stream, is their first user)
    static_assert(sizeof(FrameCounters) / 4 <= kBlock, "counters cleared by one workgroup");
    if constexpr (kMulti) {
        if (blockIdx.x == 0 && threadIdx.x < sizeof(FrameCounters) / 4)
            for (int c = 0; c < mo.n; ++c) reinterpret_cast<uint32_t *>(mo.c[c].fc)[threadIdx.x] = 0;
    } else {
        if (blockIdx.x == 0 && threadIdx.x < sizeof(FrameCounters) / 4) reinterpret_cast<uint32_t *>(fc)[threadIdx.x] = 0;
    }
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    int64_t lo, hi;
    cull_range(sc.P, blockIdx.x, &lo, &hi);
    uint32_t n = 0;     // candidates of this workgroup so far (uniform)
    uint32_t read = 0;  // batches read (uniform)
    // The batch bounds of the workgroup's range are tested first, one batch
    // per thread, into a mask (a batch that the test below would drop
    // entirely is not read); then the kept batches are read in turn.
    __shared__ uint32_t s_skip[kBlock / 32];
    const int64_t b_lo = lo / kBlock, b_hi = (hi + kBlock - 1) / kBlock;
    for (int64_t cb = b_lo; cb < b_hi; cb += kBlock) {
        {
            const int64_t bt = cb + threadIdx.x;
            bool skip = false;
            if (bt < b_hi) {
                const float4 *const bb = pp.blk + 3 * bt;
                const float4 blo = bb[0], bhi = bb[1], bkx = bb[2];
                skip = true;
                if constexpr (kMulti) {
                    for (int c = 0; c < mo.n && skip; ++c)
                        skip = batch_culled(blo, bhi, bkx, mo.c[c].cam, op, mo.c[c].W, mo.c[c].H);
                } else {
                    skip = batch_culled(blo, bhi, bkx, cam, op, W, H);
                }
            }
            const uint64_t bal = __ballot(skip);
            if (lane == 0) {
                s_skip[2 * wave] = (uint32_t)bal;
                s_skip[2 * wave + 1] = (uint32_t)(bal >> 32);
            }
            __syncthreads();
        }
        const int nq = (int)((cb + kBlock < b_hi ? cb + kBlock : b_hi) - cb);
        // the first kept batch of the chunk at or after q (nq if none)
        auto next_kept = [&](int q) {
            while (q < nq) {
                const uint32_t w = ~s_skip[q >> 5] >> (q & 31);
                if (w) return min(q + (int)__builtin_ctz(w), nq);
                q = (q | 31) + 1;
            }
            return nq;
        };
        // member threadIdx.x of kept batch q: its position, opacity and
        // extent terms.  The index is clamped into the range (some member's
        // data past its end or for q = nq, unused): the loads are issued
        // unconditionally, so that nothing waits on a pending one.
        auto load = [&](int q, float4 &p4, float2 &bd) {
            int64_t g = (cb + (q < nq ? q : 0)) * kBlock + threadIdx.x;
            g = g < hi ? g : hi - 1;
            p4 = pp.pos_o[g];
            bd = pp.bnd[g];
        };
        // test and compact kept batch q, members' data p4 and bd
        auto batch = [&](int q, const float4 &p4, const float2 &bd) {
            ++read;
            const int64_t g = (cb + q) * kBlock + threadIdx.x;
            bool keep;
            if constexpr (kMulti) {
                // union of the cameras' candidates: the exact path of each
                // camera culls the rest
                keep = cull_keep(p4, bd, mo.c[0].cam, op, mo.c[0].W, mo.c[0].H);
                for (int c = 1; c < mo.n && !keep; ++c) keep = cull_keep(p4, bd, mo.c[c].cam, op, mo.c[c].W, mo.c[c].H);
            } else {
                keep = cull_keep(p4, bd, cam, op, W, H);
            }
            keep = keep && g < hi;
            // ordered compaction into this workgroup's own segment
            const uint64_t bal = __ballot(keep);
            if (lane == 0) s_w[wave] = (uint32_t)__popcll(bal);
            __syncthreads();
            uint32_t before = 0, tot = 0;
#pragma unroll
            for (int w = 0; w < kBlock / kWave; ++w) {
                before += w < wave ? s_w[w] : 0u;
                tot += s_w[w];
            }
            if (keep) cand[lo + n + before + (uint32_t)__popcll(bal & ((1ull << lane) - 1ull))] = (uint32_t)g;
            n += tot;
            __syncthreads();
        };
        // two buffers in turn: the next kept batch's loads are in flight
        // during this one's test, with no copy between them
        float4 pa, pb;
        float2 ba, bb;
        int q = next_kept(0);
        load(q, pa, ba);
        while (q < nq) {
            int qn = next_kept(q + 1);
            load(qn, pb, bb);
            batch(q, pa, ba);
            q = qn;
            if (q >= nq) break;
            qn = next_kept(q + 1);
            load(qn, pa, ba);
            batch(q, pb, bb);
            q = qn;
        }
        __syncthreads();  // every thread has read the mask before it is replaced
    }
    if (threadIdx.x == 0) {
        seg_count[blockIdx.x] = n;
        seg_count[kCullBlocks + blockIdx.x] = read;
    }
}

// kMulti (with kPrep): every camera of mo in turn over the union candidate
// list, each with its own outputs and counters (the camera and output
// arguments are then unused); the repeated reads of a Gaussian's precompute
// for the second and later cameras follow the first within the same
// wavefront and hit the caches.
template <bool kPrep, bool kMulti = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_preprocess(DevScene sc, DevPrepared pp, DevCamera cam, DevCam64 cam64, DevOptions op,
                                                       int W_arg, int H_arg, GaussState *__restrict__ gs,
                                                       float4 *__restrict__ conic,
                                                       uint4 *__restrict__ rect, uint32_t *__restrict__ count,
                                                       uint8_t *__restrict__ count8, uint4 *__restrict__ erec,
                                                       uint32_t *__restrict__ dkey,
                                                       const uint32_t *__restrict__ cand,
                                                       const uint32_t *__restrict__ seg_count,
                                                       uint32_t *__restrict__ gmap, uint2 *__restrict__ chunks,
                                                       uint32_t chunk_cap, FrameCounters *fc,
                                                       uint32_t *__restrict__ gsum_clear, int full, MultiOut mo) {
    static_assert(!kMulti || kPrep, "a batch walks a union candidate list");
    // the first depth pass's group sums start at zero
    if constexpr (kMulti) {
        for (int c = 0; c < mo.n; ++c)
            for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < (uint32_t)kGsumWords; i += gridDim.x * kBlock)
                mo.c[c].gsum_clear[i] = 0;
    } else {
        for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < (uint32_t)kGsumWords; i += gridDim.x * kBlock)
            gsum_clear[i] = 0;
    }
    // Persistent grid: each workgroup walks batches of 256 Gaussians.  Every
    // wavefront keeps its own visible count and pending chunk reservations
    // (LDS), so the batch loop has no workgroup barrier and global atomics
    // are per wavefront flush, not per batch.
    constexpr int kWaveBig = kBigList / (kBlock / kWave);  // pending large Gaussians per wavefront
    __shared__ uint32_t s_bg[kBlock / kWave][kWaveBig], s_boff[kBlock / kWave][kWaveBig],
        s_bn[kBlock / kWave][kWaveBig], s_bx[kBlock / kWave][kWaveBig], s_by[kBlock / kWave][kWaveBig];
    __shared__ uint32_t s_excl[kBlock / kWave][kWave], s_mlo[kBlock / kWave][kWave], s_mhi[kBlock / kWave][kWave];
    const int wv = threadIdx.x / kWave;  // this lane's wavefront
    uint32_t w_nbig = 0, w_nch = 0;      // wave-uniform: pending entries and their chunks
    uint32_t w_vis = 0;                  // wave-uniform: visible Gaussians so far
    uint32_t l_pairs = 0;                // this lane's small-rectangle hits so far
    __shared__ uint32_t s_vis[kMulti ? kBlock / kWave : 1][kMulti ? kMaxCams : 1];  // per camera (kMulti)
    __shared__ uint32_t s_pairs[kMulti ? kBlock / kWave : 1][kMulti ? kMaxCams : 1];
    // kMulti: the pending list holds entries of every camera, each tagged
    // with its camera; chunks are counted per camera, and a flush reserves
    // each camera's share of its own chunk list
    constexpr int kMB = kMulti ? kWaveBig : 1;
    constexpr int kMC = kMulti ? kMaxCams : 1;
    __shared__ uint32_t s_bc[kBlock / kWave][kMB], s_nch[kBlock / kWave][kMC], s_cbase[kBlock / kWave][kMC];
    __shared__ uint2 *s_chunks[kMC];
    __shared__ uint4 *s_erec[kMC];
    if constexpr (kMulti) {
        if ((threadIdx.x & (kWave - 1)) == 0)
            for (int c = 0; c < kMaxCams; ++c) {
                s_vis[wv][c] = 0;
                s_pairs[wv][c] = 0;
                s_nch[wv][c] = 0;
            }
        if (threadIdx.x == 0)
            for (int c = 0; c < mo.n; ++c) {
                s_chunks[c] = mo.c[c].chunks;
                s_erec[c] = mo.c[c].erec;
            }
        __syncthreads();
    }

    // reserve chunk-list space for the wavefront's pending large Gaussians
    // and write their entries (g, first chunk); on overflow only flag it
    // (the host resizes the list and renders the frame again)
    auto flush_big = [&](int ln, FrameCounters *fc, uint2 *__restrict__ chunks, uint32_t chunk_cap,
                         uint4 *__restrict__ erec) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        uint32_t base = 0;
        if (ln == 0) base = atomicAdd(&fc->nchunks, w_nch);
        base = (uint32_t)__shfl((int)base, 0, kWave);
        const bool ok = (uint64_t)base + w_nch <= chunk_cap;
        if (!ok && ln == 0) atomicOr(&fc->error, kErrChunkOverflow);
        for (uint32_t e = (uint32_t)ln; e < w_nbig; e += kWave) {
            const uint32_t gg = s_bg[wv][e], first = base + s_boff[wv][e], n = s_bn[wv][e];
            if (ok)
                for (uint32_t c = 0; c < n; ++c) chunks[first + c] = make_uint2(gg, first);
            // (on overflow the record still marks the rectangle as chunked, so
            // that the emission of this frame reads no record of an earlier one)
            erec[gg] = make_uint4(s_bx[wv][e], s_by[wv][e], 0u, ok ? first : 0u);
        }
        // every lane has read the list before it is refilled
        __builtin_amdgcn_wave_barrier();
        w_nbig = 0;
        w_nch = 0;
    };
    constexpr uint32_t kNoBase = 0xffffffffu;
    auto flush_big_multi = [&](int ln) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (ln == 0)
            for (int c = 0; c < mo.n; ++c) {
                const uint32_t n = s_nch[wv][c];
                uint32_t base = kNoBase;
                if (n) {
                    base = atomicAdd(&mo.c[c].fc->nchunks, n);
                    if ((uint64_t)base + n > mo.c[c].chunk_cap) {
                        atomicOr(&mo.c[c].fc->error, kErrChunkOverflow);
                        base = kNoBase;
                    }
                }
                s_cbase[wv][c] = base;
                s_nch[wv][c] = 0;
            }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (uint32_t e = (uint32_t)ln; e < w_nbig; e += kWave) {
            const uint32_t c = s_bc[wv][e], base = s_cbase[wv][c];
            const uint32_t gg = s_bg[wv][e];
            if (base == kNoBase) {
                // overflow: still mark the rectangle as chunked (no stale record)
                s_erec[c][gg] = make_uint4(s_bx[wv][e], s_by[wv][e], 0u, 0u);
                continue;
            }
            const uint32_t first = base + s_boff[wv][e], n = s_bn[wv][e];
            uint2 *const ck = s_chunks[c];
            for (uint32_t k = 0; k < n; ++k) ck[first + k] = make_uint2(gg, first);
            s_erec[c][gg] = make_uint4(s_bx[wv][e], s_by[wv][e], 0u, first);
        }
        __builtin_amdgcn_wave_barrier();
        w_nbig = 0;
    };

    const int lane = threadIdx.x & (kWave - 1);
    // A prepared scene walks the cull's candidates as one list: the exclusive
    // prefix of the segment counts maps a list position to its segment, and
    // workgroups take 256-position batches in turn, so every workgroup gets
    // the same share whatever the segment sizes.  Raw parameters walk every
    // Gaussian.  g = sc.P marks an idle lane.
    static_assert((kCullBlocks & (kCullBlocks - 1)) == 0 && kCullBlocks % kBlock == 0, "segment prefix layout");
    __shared__ uint32_t s_pref[kPrep ? kCullBlocks : 1];
    __shared__ uint32_t s_wtot[kBlock / kWave];
    uint32_t ncand = 0;
    if constexpr (kPrep) {
        constexpr int kPer = kCullBlocks / kBlock;
        uint32_t c[kPer], sum = 0;
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            c[j] = seg_count[threadIdx.x * kPer + j];
            sum += c[j];
        }
        const int wave = threadIdx.x / kWave;
        const uint32_t incl = wave_incl_scan(sum, lane);
        if (lane == kWave - 1) s_wtot[wave] = incl;
        __syncthreads();
        uint32_t run = incl - sum;
        for (int w = 0; w < kBlock / kWave; ++w) {
            if (w < wave) run += s_wtot[w];
            ncand += s_wtot[w];
        }
#pragma unroll
        for (int j = 0; j < kPer; ++j) {
            s_pref[threadIdx.x * kPer + j] = run;
            run += c[j];
        }
        __syncthreads();
    }
    if constexpr (kPrep) {
        // the batches the cull read (its workgroups' counts), for the stats
        if (blockIdx.x == 0) {
            constexpr int kPer = kCullBlocks / kBlock;
            uint32_t r = 0;
#pragma unroll
            for (int j = 0; j < kPer; ++j) r += seg_count[kCullBlocks + threadIdx.x * kPer + j];
            const uint32_t incl = wave_incl_scan(r, lane);
            __syncthreads();  // s_wtot is free again
            if (lane == kWave - 1) s_wtot[threadIdx.x / kWave] = incl;
            __syncthreads();
            if (threadIdx.x == 0) {
                uint32_t tot = 0;
                for (int w = 0; w < kBlock / kWave; ++w) tot += s_wtot[w];
                if constexpr (kMulti) {
                    for (int c = 0; c < mo.n; ++c) {
                        mo.c[c].fc->ncand = ncand;
                        mo.c[c].fc->cull_read = tot;
                    }
                } else {
                    fc->ncand = ncand;
                    fc->cull_read = tot;
                }
            }
        }
    }
    // outputs of a prepared scene go to the candidate's list position (dense,
    // contiguous per wavefront), of raw parameters to the Gaussian's index
    int64_t batch = blockIdx.x;  // batch of 256 list positions (prepared) or Gaussians (raw)
    for (;;) {
    int64_t g = sc.P;
    uint32_t ii = 0;  // prepared: position in the candidate list
    if constexpr (kPrep) {
        if ((uint64_t)batch * kBlock >= ncand) break;
        ii = (uint32_t)batch * kBlock + threadIdx.x;
        if (ii < ncand) {
            // last segment whose prefix is <= ii: it holds position ii
            uint32_t sg = 0;
#pragma unroll
            for (uint32_t step = kCullBlocks / 2; step > 0; step >>= 1)
                if (s_pref[sg + step] <= ii) sg += step;
            int64_t lo, hi;
            cull_range(sc.P, sg, &lo, &hi);
            g = (int64_t)cand[lo + (ii - s_pref[sg])];
        }
        batch += gridDim.x;
    } else {
        if (batch * kBlock >= sc.P) break;
        const int64_t ii = batch * kBlock + threadIdx.x;
        if (ii < sc.P) g = ii;
        batch += gridDim.x;
    }
    const int ncams = kMulti ? mo.n : 1;
    for (int ci = 0; ci < ncams; ++ci) {
    // this camera, its image size and its outputs
    const DevCamera &cm = kMulti ? mo.c[ci].cam : cam;
    const int W = kMulti ? mo.c[ci].W : W_arg, H = kMulti ? mo.c[ci].H : H_arg;
    const DevCam64 &cm64 = kMulti ? mo.c[ci].cam64 : cam64;
    GaussState *__restrict__ const gs_c = kMulti ? mo.c[ci].gs : gs;
    float4 *__restrict__ const conic_c = kMulti ? mo.c[ci].conic : conic;
    uint4 *__restrict__ const rect_c = kMulti ? mo.c[ci].rect : rect;
    uint32_t *__restrict__ const count_c = kMulti ? mo.c[ci].count : count;
    uint8_t *__restrict__ const count8_c = kMulti ? mo.c[ci].count8 : count8;
    uint4 *__restrict__ const erec_c = kMulti ? mo.c[ci].erec : erec;
    uint32_t *__restrict__ const dkey_c = kMulti ? mo.c[ci].dkey : dkey;
    const int64_t st = sc.stride;
    bool valid = false;
    float u = 0, v = 0, A = 0, B = 0, C = 0, k2 = 0, o = 0, tz = 0, l2o = 0;
    float Ab = 0, Bb = 0, Cb = 0;  // the blend's conic (see GaussState)
    int tx0 = 0, tx1 = -1, ty0 = 0, ty1 = -1;
    float col[3] = {0, 0, 0};

    if (g < sc.P) {
        float mx, my, mz, po = 0.0f;
        if constexpr (kPrep) {
            const float4 p4 = pp.pos_o[g];
            mx = p4.x;
            my = p4.y;
            mz = p4.z;
            po = p4.w;
        } else {
            mx = sc.means[g];
            my = sc.means[st + g];
            mz = sc.means[2 * st + g];
        }
        const float *R = cm.R;
        // view transform (p_view)
        const float tx = ((R[0] * mx + R[1] * my) + R[2] * mz) + cm.t[0];
        const float ty = ((R[3] * mx + R[4] * my) + R[5] * mz) + cm.t[1];
        tz = ((R[6] * mx + R[7] * my) + R[8] * mz) + cm.t[2];
        // near plane (Alg. 4: p_view.z > 0.2); the remaining attributes are
        // read only for Gaussians in front of the camera
        if (tz > cm.near_z && isfinite(mx) && isfinite(my) && isfinite(mz)) {
            bool ok = false;
            float S[6] = {0, 0, 0, 0, 0, 0}, s3[3] = {0, 0, 0}, qu[4] = {0, 0, 0, 0};
            float log2o = 0.0f;
            if constexpr (kPrep) {
                // view-independent part precomputed once (Sec. 5.3.1); an
                // invalid Gaussian has opacity 0
                o = po;
                ok = o > op.alpha_min;
                if (ok) {
                    const float4 c0 = pp.cov[2 * g], c1 = pp.cov[2 * g + 1];
                    s3[0] = c0.x; s3[1] = c0.y; s3[2] = c0.z;
                    k2 = c0.w;
                    qu[0] = c1.x; qu[1] = c1.y; qu[2] = c1.z; qu[3] = c1.w;
                }
            } else {
                const float logit = sc.logits[g];
                o = (float)(1.0 / (1.0 + canon_exp(-(double)logit)));
                // opacity prefilter (Alg. 4: opacity > 1/255)
                if (o > op.alpha_min && isfinite(logit)) {
                    const float ls0 = sc.log_scales[g], ls1 = sc.log_scales[st + g],
                                ls2 = sc.log_scales[2 * st + g];
                    const float q4[4] = {sc.quats[g], sc.quats[st + g], sc.quats[2 * st + g], sc.quats[3 * st + g]};
                    ok = scale_rot(ls0, ls1, ls2, q4, s3, qu);
                    if (ok) k2 = extent_k2(o, op);
                }
            }
            if (ok) {
                sigma3(s3, qu, S);
                log2o = log2f(o);
                // the blend's conic (binary64, rounded once)
                const bool have_b64 = conic_b64(s3, qu, mx, my, mz, cm64, (double)op.dilation, &Ab, &Bb, &Cb);
                const float S00 = S[0], S01 = S[1], S02 = S[2], S11 = S[3], S12 = S[4], S22 = S[5];
                {
                    // pinhole projection (project + ndc2Pix)
                    const float xt = tx / tz, yt = ty / tz;
                    u = cm.fx * xt + cm.cx;
                    v = cm.fy * yt + cm.cy;
                    // EWA Jacobian with the view-direction clamp
                    const float limx = op.jac_clip * ((0.5f * (float)W) / cm.fx);
                    const float limy = op.jac_clip * ((0.5f * (float)H) / cm.fy);
                    const float xc = clampf_(xt, -limx, limx);
                    const float yc = clampf_(yt, -limy, limy);
                    const float J00 = cm.fx / tz, J02 = -((cm.fx * xc) / tz);
                    const float J11 = cm.fy / tz, J12 = -((cm.fy * yc) / tz);
                    // 2D covariance Sigma' = T Sigma T^T, T = J R_cam
                    const float T00 = J00 * R[0] + J02 * R[6], T01 = J00 * R[1] + J02 * R[7],
                                T02 = J00 * R[2] + J02 * R[8];
                    const float T10 = J11 * R[3] + J12 * R[6], T11 = J11 * R[4] + J12 * R[7],
                                T12 = J11 * R[5] + J12 * R[8];
                    const float U00 = (T00 * S00 + T01 * S01) + T02 * S02;
                    const float U01 = (T00 * S01 + T01 * S11) + T02 * S12;
                    const float U02 = (T00 * S02 + T01 * S12) + T02 * S22;
                    const float U10 = (T10 * S00 + T11 * S01) + T12 * S02;
                    const float U11 = (T10 * S01 + T11 * S11) + T12 * S12;
                    const float U12 = (T10 * S02 + T11 * S12) + T12 * S22;
                    const float ca = ((U00 * T00 + U01 * T01) + U02 * T02) + op.dilation;
                    const float cb = (U00 * T10 + U01 * T11) + U02 * T12;
                    const float cc = ((U10 * T10 + U11 * T11) + U12 * T12) + op.dilation;
                    const float det = ca * cc - cb * cb;
                    if (det > 0.0f) {
                        A = cc / det;
                        B = (-cb) / det;
                        C = ca / det;
                        // the blend's conic: the binary32 one if the binary64
                        // determinant was not positive
                        if (!have_b64) {
                            Ab = A;
                            Bb = B;
                            Cb = C;
                        }
                        // rectangle tangent to the ellipse (Sec. 4.1), in pixel samples;
                        // binning 2: the square of the 3 sigma circle of 3DGS
                        // (Alg. 1: radius ceil(3 sqrt(lambda_max)) of Sigma')
                        float hx, hy;
                        if (op.binning == 2) {
                            const float mid = 0.5f * (ca + cc);
                            float disc = mid * mid - det;
                            disc = disc > 0.0f ? disc : 0.0f;
                            const float lam = mid + sqrtf(disc);
                            hx = ceilf(3.0f * sqrtf(lam));
                            hy = hx;
                        } else {
                            hx = sqrtf(k2 * ca);
                            hy = sqrtf(k2 * cc);
                        }
                        const float xlo = clampf_((u - hx) - 0.5f, -1.0f, (float)W);
                        const float xhi = clampf_((u + hx) - 0.5f, -1.0f, (float)W);
                        const float ylo = clampf_((v - hy) - 0.5f, -1.0f, (float)H);
                        const float yhi = clampf_((v + hy) - 0.5f, -1.0f, (float)H);
                        int i0 = (int)ceilf(xlo), i1 = (int)floorf(xhi);
                        int j0 = (int)ceilf(ylo), j1 = (int)floorf(yhi);
                        i0 = i0 < 0 ? 0 : i0;
                        j0 = j0 < 0 ? 0 : j0;
                        i1 = i1 > W - 1 ? W - 1 : i1;
                        j1 = j1 > H - 1 ? H - 1 : j1;
                        if (i0 <= i1 && j0 <= j1) {
                            tx0 = i0 / kTile;
                            tx1 = i1 / kTile;
                            ty0 = j0 / kTile;
                            ty1 = j1 / kTile;
                            // SH colour for surviving Gaussians only (Alg. 4)
                            const float dxw = mx - cm.eye[0], dyw = my - cm.eye[1], dzw = mz - cm.eye[2];
                            const float dn = sqrtf((dxw * dxw + dyw * dyw) + dzw * dzw);
                            float Y[16];
                            sh_basis(dxw / dn, dyw / dn, dzw / dn, sc.D, Y);
                            const int nk = (sc.D + 1) * (sc.D + 1);
                            float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
                            // every coefficient load is issued before the first
                            // use (one memory round trip, not one per coefficient)
                            const int ncoef = 3 * nk;
                            float shv[48];
                            if constexpr (kPrep) {
                                // Gaussian-major coefficients: one contiguous read
                                const float4 *shg = reinterpret_cast<const float4 *>(pp.sh + (int64_t)g * pp.sh_stride);
#pragma unroll
                                for (int j = 0; j < 12; ++j) {
                                    const float4 q4 = 4 * j < ncoef ? shg[j] : make_float4(0.f, 0.f, 0.f, 0.f);
                                    shv[4 * j] = q4.x;
                                    shv[4 * j + 1] = q4.y;
                                    shv[4 * j + 2] = q4.z;
                                    shv[4 * j + 3] = q4.w;
                                }
                            } else {
#pragma unroll
                                for (int j = 0; j < 48; ++j) shv[j] = j < ncoef ? sc.sh[(int64_t)j * st + g] : 0.0f;
                            }
#pragma unroll
                            for (int k = 0; k < 16; ++k) {
                                if (k < nk) {
                                    a0 = a0 + shv[3 * k + 0] * Y[k];
                                    a1 = a1 + shv[3 * k + 1] * Y[k];
                                    a2 = a2 + shv[3 * k + 2] * Y[k];
                                }
                            }
                            a0 = a0 + 0.5f;
                            a1 = a1 + 0.5f;
                            a2 = a2 + 0.5f;
                            // non-finite SH inputs cull the Gaussian
                            valid = isfinite(a0) && isfinite(a1) && isfinite(a2);
                            col[0] = a0 > 0.0f ? a0 : 0.0f;
                            col[1] = a1 > 0.0f ? a1 : 0.0f;
                            col[2] = a2 > 0.0f ? a2 : 0.0f;
                            l2o = log2o;
                        }
                    }
                }
            }
        }
    }

    // ---- exact tile count (Alg. 3 over the rectangle) -------------------------
    const int ntx = tx1 - tx0 + 1, nty = ty1 - ty0 + 1;
    const int nt = valid ? ntx * nty : 0;
    uint32_t cnt = 0;
    uint64_t hm = 0;
    // rectangles of more than kBigTiles tiles go to the chunk list, where
    // wavefronts across the GPU test them kChunkTiles tiles at a time
    const bool chunked = valid && nt > kBigTiles;
    {
        const uint64_t bm = __ballot(chunked);
        if (bm) {  // uniform
            const uint32_t nch = chunked ? (uint32_t)((nt + kChunkTiles - 1) / kChunkTiles) : 0u;
            const uint32_t incl = wave_incl_scan(nch, lane);
            // chunks pending before these (this camera's, kMulti)
            uint32_t cbase = w_nch;
            if constexpr (kMulti) cbase = s_nch[wv][ci];
            if (chunked) {
                const uint32_t slot = w_nbig + (uint32_t)__popcll(bm & ((1ull << lane) - 1ull));
                if constexpr (kMulti) s_bc[wv][slot] = (uint32_t)ci;
                s_bg[wv][slot] = kPrep ? ii : (uint32_t)g;
                s_bn[wv][slot] = nch;
                s_bx[wv][slot] = (uint32_t)tx0 | ((uint32_t)tx1 << 16);
                s_by[wv][slot] = (uint32_t)ty0 | ((uint32_t)ty1 << 16);
                s_boff[wv][slot] = cbase + incl - nch;
            }
            w_nbig += (uint32_t)__popcll(bm);
            const uint32_t tot = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
            if constexpr (kMulti) {
                if (lane == 0) s_nch[wv][ci] = cbase + tot;
            } else {
                w_nch += tot;
            }
        }
    }
    const bool small = valid && !chunked;  // rectangle of at most kBigTiles tiles
    if (op.binning != 0) {
        // every tile of the rectangle (test and comparison modes)
        if (small) {
            cnt = (uint32_t)nt;
            hm = nt >= 64 ? ~0ull : ((1ull << nt) - 1ull);
        }
    } else {
        // The wavefront flattens its (Gaussian, rectangle tile) items so that
        // every lane tests one tile per step whatever the mix of rectangle
        // sizes (Sec. 5.1.2 size-aware scheduling, balanced across wave64).
        const int wave = threadIdx.x / kWave;
        uint32_t *sx = s_excl[wave];
        const uint32_t items = small ? (uint32_t)nt : 0u;
        const uint32_t incl = wave_incl_scan(items, lane);
        const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
        sx[lane] = incl - items;
        s_mlo[wave][lane] = 0u;
        s_mhi[wave][lane] = 0u;
        for (uint32_t b0 = 0; b0 < total; b0 += kWave) {
            const uint32_t item = b0 + (uint32_t)lane;
            const int L = owner_lane(sx, item < total ? item : total - 1u);
            const uint32_t k = item - sx[L];
            const float su = __shfl(u, L, kWave), sv = __shfl(v, L, kWave), sA = __shfl(A, L, kWave),
                        sB = __shfl(B, L, kWave), sC = __shfl(C, L, kWave), sk2 = __shfl(k2, L, kWave);
            const int stx0 = __shfl(tx0, L, kWave), sty0 = __shfl(ty0, L, kWave), sntx = __shfl(ntx, L, kWave);
            if (item < total) {
                const int ry = small_div(k, sntx), rx = (int)k - ry * sntx;
                if (tile_hit(su, sv, sA, sB, sC, sk2, stx0 + rx, sty0 + ry, W, H))
                    atomicOr(k < 32u ? &s_mlo[wave][L] : &s_mhi[wave][L], 1u << (k & 31u));
            }
        }
        hm = (uint64_t)s_mlo[wave][lane] | ((uint64_t)s_mhi[wave][lane] << 32);
        cnt = (uint32_t)__popcll(hm);
    }

    if (g < sc.P) {
        const uint32_t key = valid ? __float_as_uint(tz) : kInvalidKey;
        const int64_t oi = kPrep ? (int64_t)ii : g;  // output slot
        if constexpr (kPrep) {
            // the Gaussian of this list position, in the caller's indexing
            uint32_t *const gmap_c = kMulti ? mo.c[ci].gmap : gmap;
            gmap_c[ii] = pp.orig[g];
        }
        dkey_c[oi] = key;
        // entries: the overlapped super-tiles (at most 10 for a rectangle of
        // at most kBigTiles tiles)
        count8_c[oi] = chunked ? kCount8Big : (uint8_t)(valid ? super_span(tx0, tx1, ty0, ty1) : 0u);
        // the 4-byte count: a chunked rectangle's starts at 0 (k_big_count
        // adds its hits); the others are read from count8
        if (full || chunked) count_c[oi] = valid ? cnt : 0u;
        if (valid) {
            GaussState s;
            s.f0 = make_float4(u, v, Ab, Bb);
            s.f1 = make_float4(Cb, k2, l2o, col[0]);
            s.f2 = make_float4(col[1], col[2], tz, o);
            gs_c[oi] = s;
            // the canonical conic: the large rectangles' tile tests read it
            if (full || chunked) conic_c[oi] = make_float4(A, B, C, 0.0f);
            if (full) rect_c[oi] = make_uint4((uint32_t)tx0, (uint32_t)tx1, (uint32_t)ty0, (uint32_t)ty1);
            // emission record: rectangle (4 x 16 bits) and hit mask in one
            // 16-byte gather (a chunked one's is written at its flush)
            if (!chunked)
                erec_c[oi] = make_uint4((uint32_t)tx0 | ((uint32_t)tx1 << 16), (uint32_t)ty0 | ((uint32_t)ty1 << 16),
                                      (uint32_t)hm, (uint32_t)(hm >> 32));
        } else if (kPrep && full) {
            // a list slot is reused every frame: clear a culled candidate's
            // introspected state
            gs_c[oi] = GaussState{};
            conic_c[oi] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            rect_c[oi] = make_uint4(0u, 0u, 0u, 0u);
        }
    }
    if constexpr (kMulti) {
        const uint32_t nv = (uint32_t)__popcll(__ballot(valid));
        uint32_t np = small ? cnt : 0u;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) np += (uint32_t)__shfl_xor((int)np, d, kWave);
        if (lane == 0) {
            s_vis[wv][ci] += nv;
            s_pairs[wv][ci] += np;
        }
        if (w_nbig > (uint32_t)(kWaveBig - kWave)) flush_big_multi(lane);  // room for the next camera
    } else {
        l_pairs += small ? cnt : 0u;
        w_vis += (uint32_t)__popcll(__ballot(valid));
        if (w_nbig > (uint32_t)(kWaveBig - kWave))
            flush_big(lane, fc, chunks, chunk_cap, erec);  // room for the next batch
    }
    }  // camera loop
    }  // batch loop
    if constexpr (kMulti) {
        if (w_nbig) flush_big_multi(lane);
        if (lane == 0)
            for (int c = 0; c < mo.n; ++c) {
                if (s_vis[wv][c]) atomicAdd(&mo.c[c].fc->visible, s_vis[wv][c]);
                if (s_pairs[wv][c]) atomicAdd(&mo.c[c].fc->pairs, s_pairs[wv][c]);
            }
    } else {
        if (w_nbig) flush_big(lane, fc, chunks, chunk_cap, erec);
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) l_pairs += (uint32_t)__shfl_xor((int)l_pairs, d, kWave);
        if (lane == 0 && w_vis) atomicAdd(&fc->visible, w_vis);
        if (lane == 0 && l_pairs) atomicAdd(&fc->pairs, l_pairs);
    }
}

// Hit mask of a small rectangle (bit rx + ntx ry of its emission record)
// restricted to super-tile (sx, sy), in the super-tile's own layout (bit
// lx + kSuper ly): the rectangle's rows in the super-tile, each cut to the
// super-tile's columns and moved to its place.
__device__ __forceinline__ uint64_t super_mask(uint64_t hm, int tx0, int ty0, int ntx, int nty, int sx, int sy) {
    const int xs = sx * kSuper, ys = sy * kSuper;
    const int a = xs - tx0 > 0 ? xs - tx0 : 0, b = xs + kSuper - tx0 < ntx ? xs + kSuper - tx0 : ntx;
    const int c = ys - ty0 > 0 ? ys - ty0 : 0, d = ys + kSuper - ty0 < nty ? ys + kSuper - ty0 : nty;
    const uint64_t wm = (1ull << (b - a)) - 1ull;  // b - a <= kSuper
    const int lx0 = tx0 + a - xs;
    uint64_t m = 0;
    for (int ry = c; ry < d; ++ry)
        m |= ((hm >> (ry * ntx + a)) & wm) << ((ty0 + ry - ys) * kSuper + lx0);
    return m;
}

// Key emission at super-tile granularity (Alg. 2 with the offsets of a
// prefix scan, the pair (tile, Gaussian) replaced by (super-tile, Gaussian,
// hit mask); the tile test is reused from the preprocess through the hit
// mask).  The visible Gaussians are taken 64 at a time in (depth, index)
// order; the wavefront flattens the small rectangles' entries so that every
// lane builds one entry per step, written at its Gaussian's scanned offset
// plus its index among the Gaussian's entries (row-major over the
// overlapped super-tiles).  A chunked Gaussian only leaves (its output slot,
// its offset) at its first chunk's slot of `big` for k_big_entries.
__global__ __launch_bounds__(kBlock) void k_super_emit(int W, const uint32_t *__restrict__ order, uint32_t visible,
                                                       const uint32_t *__restrict__ visible_dev,
                                                       const uint32_t *__restrict__ offsets,
                                                       const uint4 *__restrict__ erec, uint2 *__restrict__ big,
                                                       uint32_t chunk_cap, uint16_t *__restrict__ skey,
                                                       uint32_t *__restrict__ gidx, uint64_t *__restrict__ smask,
                                                       uint32_t ecap, uint2 *__restrict__ sranges, uint32_t nsuper,
                                                       uint32_t *__restrict__ gsum_clear,
                                                       const FrameCounters *__restrict__ fc) {
    __shared__ uint32_t s_excl[kBlock / kWave][kWave];
    // an overflowed chunk list left the large rectangles untested: their
    // entries (k_big_entries writes them otherwise) are filled here with
    // super-tile 0, the Gaussian and an empty mask, so that the second half
    // of this frame, which the host discards and renders again, reads only
    // entries it wrote (every list value a valid Gaussian)
    const bool overflow = (fc->error & kErrChunkOverflow) != 0;
    // every super-tile's range starts empty, (0xffffffff, 0), for the last
    // sort pass to narrow (sranges NULL: no pass records them)
    if (sranges)
        for (uint32_t t = blockIdx.x * kBlock + threadIdx.x; t < nsuper; t += gridDim.x * kBlock)
            sranges[t] = make_uint2(0xffffffffu, 0u);
    // and the first sort pass's group sums start at zero
    if (gsum_clear)
        for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < (uint32_t)kGsumWords; i += gridDim.x * kBlock)
            gsum_clear[i] = 0;
    // the visible count comes from the device when the launch is sized by a
    // bound (graph-captured frames); it never exceeds the bound
    if (visible_dev) visible = min(visible, *visible_dev);
    const int tiles_x = (W + kTile - 1) / kTile;
    const uint32_t stx = (uint32_t)((tiles_x + kSuper - 1) >> kSuperShift);
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t *sx = s_excl[threadIdx.x / kWave];
    for (uint32_t r0 = blockIdx.x * kBlock; r0 < visible; r0 += gridDim.x * kBlock) {
        const uint32_t r = r0 + threadIdx.x;
        const bool act = r < visible;
        uint32_t g = 0, base = 0;
        uint4 er = make_uint4(0u, 0u, 0u, 0u);
        if (act) {
            g = order[r];
            base = offsets[r];
            er = erec[g];
        }
        const uint4 rc = unpack_rect(er);
        const int tx0 = (int)rc.x, ty0 = (int)rc.z;
        const int ntx = (int)rc.y - tx0 + 1, nty = (int)rc.w - ty0 + 1;
        const bool chunked = act && ntx * nty > kBigTiles;
        if (chunked && er.w < chunk_cap) big[er.w] = make_uint2(g, base);
        if (chunked && overflow) {  // (rare: one lane per Gaussian is enough)
            const uint32_t n = super_span(tx0, (int)rc.y, ty0, (int)rc.w);
            for (uint32_t k = 0; k < n && base + k < ecap; ++k) {
                skey[base + k] = 0;
                gidx[base + k] = g;
                smask[base + k] = 0ull;
            }
        }
        // flattened (Gaussian, super-tile) items of the small rectangles
        const uint32_t items = act && !chunked ? super_span(tx0, (int)rc.y, ty0, (int)rc.w) : 0u;
        const uint32_t incl = wave_incl_scan(items, lane);
        const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
        sx[lane] = incl - items;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t prect = (uint32_t)tx0 | ((uint32_t)ty0 << 16), psize = (uint32_t)ntx | ((uint32_t)nty << 8);
        for (uint32_t i0 = 0; i0 < total; i0 += kWave) {
            const uint32_t item = i0 + (uint32_t)lane;
            const int L = owner_lane(sx, item < total ? item : total - 1u);
            const uint32_t k = item < total ? item - sx[L] : 0u;  // (a spare lane redoes entry 0)
            const uint32_t gL = (uint32_t)__shfl((int)g, L, kWave), bL = (uint32_t)__shfl((int)base, L, kWave);
            const uint32_t pr = (uint32_t)__shfl((int)prect, L, kWave), ps = (uint32_t)__shfl((int)psize, L, kWave);
            const uint32_t hlo = (uint32_t)__shfl((int)er.z, L, kWave), hhi = (uint32_t)__shfl((int)er.w, L, kWave);
            const int ltx0 = (int)(pr & 0xffffu), lty0 = (int)(pr >> 16);
            const int lntx = (int)(ps & 0xffu), lnty = (int)(ps >> 8);
            const int sx0 = ltx0 >> kSuperShift, sy0 = lty0 >> kSuperShift;
            const int nsx = ((ltx0 + lntx - 1) >> kSuperShift) - sx0 + 1;  // at most 9 (k < 16)
            const int ey = small_div(k, nsx), ex = (int)k - ey * nsx;
            const uint64_t m = super_mask((uint64_t)hlo | ((uint64_t)hhi << 32), ltx0, lty0, lntx, lnty, sx0 + ex,
                                          sy0 + ey);
            const uint32_t at = bL + k;
            if (item < total && at < ecap) {  // never leave the entry buffers
                skey[at] = (uint16_t)((uint32_t)(sy0 + ey) * stx + (uint32_t)(sx0 + ex));
                gidx[at] = gL;
                smask[at] = m;
            }
        }
        // every lane has read the item starts before they are replaced
        __builtin_amdgcn_wave_barrier();
    }
}

// Entries of the chunked Gaussians.  Each wavefront takes 64 chunk slots,
// one per lane; a Gaussian's first chunk holds, in `big`, its output slot
// and entry offset.  The wavefront flattens the entries of its Gaussians so
// that every lane builds one entry per step: entry k of a Gaussian is
// super-tile k of its rectangle's overlap in row-major order.  The chunk
// masks of a Gaussian are one bit stream over its rectangle in row-major
// order, so each of the super-tile's (at most kSuper) rows is a run of at
// most kSuper consecutive bits, read from two words.
__global__ __launch_bounds__(kBlock) void k_big_entries(int W, const uint4 *__restrict__ erec, uint32_t ng,
                                                        const uint2 *__restrict__ chunks,
                                                        const uint2 *__restrict__ big, uint32_t chunk_cap,
                                                        const uint32_t *__restrict__ chunk_mask,
                                                        const FrameCounters *__restrict__ fc,
                                                        uint16_t *__restrict__ skey, uint32_t *__restrict__ gidx,
                                                        uint64_t *__restrict__ smask, uint32_t ecap) {
    __shared__ uint32_t s_excl[kBlock / kWave][kWave];
    // an overflowed list has entries this frame never wrote (the frame is
    // rendered again, or reported, by the host)
    if (fc->error & kErrChunkOverflow) return;
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t *sx = s_excl[threadIdx.x / kWave];
    const int tiles_x = (W + kTile - 1) / kTile;
    const uint32_t stx = (uint32_t)((tiles_x + kSuper - 1) >> kSuperShift);
    const uint32_t n = fc->nchunks < chunk_cap ? fc->nchunks : chunk_cap;
    const uint32_t nwaves = gridDim.x * (kBlock / kWave);
    constexpr uint32_t kWordsPerChunk = kChunkTiles / 32;
    const size_t wlast = (size_t)chunk_cap * kWordsPerChunk - 1;
    for (uint32_t c0 = (blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave) * kWave; c0 < n;
         c0 += nwaves * kWave) {
        const uint32_t c = c0 + (uint32_t)lane;
        bool first = false;
        uint2 gb = make_uint2(0u, 0u);
        if (c < n) {
            first = chunks[c].y == c;
            gb = big[c];
        }
        first = first && gb.x < ng;
        uint4 rc = make_uint4(0u, 0u, 0u, 0u);
        if (first) rc = unpack_rect(erec[gb.x]);
        const uint32_t items = first ? super_span((int)rc.x, (int)rc.y, (int)rc.z, (int)rc.w) : 0u;
        const uint32_t incl = wave_incl_scan(items, lane);
        const uint32_t total = (uint32_t)__shfl((int)incl, kWave - 1, kWave);
        sx[lane] = incl - items;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const uint32_t px = rc.x | (rc.y << 16), py = rc.z | (rc.w << 16);
        for (uint32_t i0 = 0; i0 < total; i0 += kWave) {
            const uint32_t item = i0 + (uint32_t)lane;
            const int L = owner_lane(sx, item < total ? item : total - 1u);
            const uint32_t k = item < total ? item - sx[L] : 0u;  // (a spare lane redoes entry 0)
            const uint32_t g = (uint32_t)__shfl((int)gb.x, L, kWave), base = (uint32_t)__shfl((int)gb.y, L, kWave);
            const uint32_t lx = (uint32_t)__shfl((int)px, L, kWave), ly = (uint32_t)__shfl((int)py, L, kWave);
            const int bx0 = (int)(lx & 0xffffu), bx1 = (int)(lx >> 16), by0 = (int)(ly & 0xffffu), by1 = (int)(ly >> 16);
            const int bntx = bx1 - bx0 + 1;
            const int sx0 = bx0 >> kSuperShift, sy0 = by0 >> kSuperShift;
            const int nsx = (bx1 >> kSuperShift) - sx0 + 1;
            int ey, ex;
            row_col((int)k, nsx, __builtin_amdgcn_rcpf((float)nsx), ey, ex);
            const int xs = (sx0 + ex) << kSuperShift, ys = (sy0 + ey) << kSuperShift;
            const int xa = xs > bx0 ? xs : bx0, xb = xs + kSuper - 1 < bx1 ? xs + kSuper - 1 : bx1;
            const int ya = ys > by0 ? ys : by0, yb = ys + kSuper - 1 < by1 ? ys + kSuper - 1 : by1;
            const uint64_t lmask = (1ull << (xb - xa + 1)) - 1ull;  // xb - xa + 1 <= kSuper
            const size_t wbase = (size_t)(c0 + (uint32_t)L) * kWordsPerChunk;
            // every row's two words are loaded (rows past yb repeat row yb)
            // before any is used: one memory round trip
            uint32_t lo[kSuper], hi[kSuper], sh[kSuper];
#pragma unroll
            for (int rr = 0; rr < kSuper; ++rr) {
                const int ty = ya + rr < yb ? ya + rr : yb;
                const uint32_t idx = (uint32_t)((ty - by0) * bntx + (xa - bx0));
                const size_t w0 = wbase + idx / 32 < wlast ? wbase + idx / 32 : wlast;
                const size_t w1 = w0 + 1 < wlast ? w0 + 1 : wlast;
                lo[rr] = chunk_mask[w0];
                hi[rr] = chunk_mask[w1];
                sh[rr] = idx % 32;
            }
            uint64_t m = 0;
#pragma unroll
            for (int rr = 0; rr < kSuper; ++rr) {
                const uint64_t bits = (((uint64_t)lo[rr] | ((uint64_t)hi[rr] << 32)) >> sh[rr]) & lmask;
                const int place = (ya + rr - ys) * kSuper + (xa - xs);
                m |= ya + rr <= yb ? bits << place : 0ull;
            }
            const uint32_t at = base + k;
            if (item < total && at < ecap) {
                skey[at] = (uint16_t)((uint32_t)(ys >> kSuperShift) * stx + (uint32_t)(xs >> kSuperShift));
                gidx[at] = g;
                smask[at] = m;
            }
        }
        // every lane has read the item starts before they are replaced
        __builtin_amdgcn_wave_barrier();
    }
}

// LDS visibility of this wavefront's own writes to its own later reads
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Exact tile tests of the chunked Gaussians.  A wavefront takes 64
// consecutive chunk slots: every lane loads one slot's descriptor and then
// its Gaussian's rectangle, centre, conic and k^2, so that the 64 chunks cost
// two memory round trips together; the chunks are then tested one after the
// other with their values read from the owning lane (kChunkTiles tiles, 4
// per lane, independent).  A chunk covers few tile rows, whose terms of the
// test (tile_row_terms) are computed once per row into LDS; each tile adds
// its column's terms and combines them (tile_hit_terms: the operations of
// tile_hit).  The 8 mask words of a chunk are written by four
// lanes, and the hits of a Gaussian's consecutive chunks are summed across
// the lanes before one atomic per Gaussian and wavefront.  A workgroup adds
// its hits to the frame's pair count once.  (With 64 slots per wavefront the
// kernel runs as fewer, longer wavefronts, which leaves the depth sort
// beside it more of each CU than one chunk per wavefront did.)
__global__ __launch_bounds__(kBlock) void k_big_count(int W, int H, int binning, const GaussState *__restrict__ gs,
                                                      const float4 *__restrict__ conic,
                                                      const uint4 *__restrict__ erec,
                                                      const uint2 *__restrict__ chunks, uint32_t chunk_cap,
                                                      uint32_t *__restrict__ chunk_mask, uint32_t *count,
                                                      FrameCounters *fc) {
    constexpr int kPer = kChunkTiles / kWave;
    static_assert(kPer == 4, "a chunk's mask is written as four 64-bit words");
    __shared__ uint32_t s_hits[kBlock / kWave];
    // the row terms of the chunk being tested (one lane per row)
    __shared__ float4 s_ra[kBlock / kWave][kWave], s_rb[kBlock / kWave][kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int wv = threadIdx.x / kWave;
    uint32_t whits = 0;  // wave-uniform
    // an overflowed list has entries this frame never wrote (the frame is
    // rendered again, or reported, by the host)
    if (!(fc->error & kErrChunkOverflow)) {
        const uint32_t n = fc->nchunks < chunk_cap ? fc->nchunks : chunk_cap;
        const uint32_t nwaves = gridDim.x * (kBlock / kWave);
        uint64_t *const mask64 = reinterpret_cast<uint64_t *>(chunk_mask);
        for (uint32_t c0 = (blockIdx.x * (kBlock / kWave) + (uint32_t)wv) * kWave; c0 < n; c0 += nwaves * kWave) {
            const uint32_t c = c0 + (uint32_t)lane;
            uint2 e = make_uint2(kNoChunk, 0u);
            if (c < n) e = chunks[c];
            const bool have = e.x != kNoChunk;
            // this lane's chunk: its Gaussian's record, centre, k^2 and conic
            uint4 rr = make_uint4(0u, 0u, 0u, 0u);
            float4 f0 = make_float4(0.0f, 0.0f, 0.0f, 0.0f), f1 = f0, cn = f0;
            if (have) {
                rr = erec[e.x];
                if (binning == 0) {
                    const float4 *sp = reinterpret_cast<const float4 *>(gs + e.x);
                    f0 = sp[0];
                    f1 = sp[1];
                    cn = conic[e.x];
                }
            }
            const uint32_t cidx = have ? c - e.y : 0u;  // chunk within its Gaussian
            uint32_t my_hits = 0;
            uint64_t todo = __ballot(have);
            while (todo) {
                const int j = __builtin_ctzll(todo);
                todo &= todo - 1ull;
                const uint32_t px = bcast(rr.x, j), py = bcast(rr.y, j), cc = bcast(cidx, j);
                const float u = bcast(f0.x, j), v = bcast(f0.y, j), k2 = bcast(f1.y, j);
                const float A = bcast(cn.x, j), B = bcast(cn.y, j), C = bcast(cn.z, j);
                const int tx0 = (int)(px & 0xffffu), ntx = (int)(px >> 16) - tx0 + 1;
                const int ty0 = (int)(py & 0xffffu), nt = ntx * ((int)(py >> 16) - ty0 + 1);
                const float rcpn = __builtin_amdgcn_rcpf((float)ntx);
                // the chunk's rows: their terms once each (a chunk over more
                // rows than a wavefront has lanes tests tile by tile)
                const int i0 = (int)cc * kChunkTiles;
                const int i1 = (i0 + kChunkTiles < nt ? i0 + kChunkTiles : nt) - 1;
                int ry_a, rx_a, ry_b, rx_b;
                row_col(i0, ntx, rcpn, ry_a, rx_a);
                row_col(i1, ntx, rcpn, ry_b, rx_b);
                const bool rows = binning == 0 && ry_b - ry_a < kWave;
                if (rows) {
                    wave_sync();  // every lane has read the previous chunk's terms
                    if (lane <= ry_b - ry_a) {
                        float4 ra, rb;
                        tile_row_terms(v, A, B, C, k2, ty0 + ry_a + lane, H, ra, rb);
                        s_ra[wv][lane] = ra;
                        s_rb[wv][lane] = rb;
                    }
                    wave_sync();
                }
                uint64_t bw[kPer];
#pragma unroll
                for (int q = 0; q < kPer; ++q) {
                    const int idx = i0 + q * kWave + lane;
                    bool h = false;
                    if (idx < nt) {
                        int ry, rx;
                        row_col(idx, ntx, rcpn, ry, rx);
                        if (rows) {
                            float4 ca, cb;
                            tile_col_terms(u, A, B, C, k2, tx0 + rx, W, ca, cb);
                            h = tile_hit_terms(ca, cb, s_ra[wv][ry - ry_a], s_rb[wv][ry - ry_a]);
                        } else {
                            h = binning != 0 || tile_hit(u, v, A, B, C, k2, tx0 + rx, ty0 + ry, W, H);
                        }
                    }
                    bw[q] = __ballot(h);
                }
                const uint32_t tot = (uint32_t)(__popcll(bw[0]) + __popcll(bw[1]) + __popcll(bw[2]) + __popcll(bw[3]));
                if (lane < kPer) {
                    const uint64_t w = lane == 0 ? bw[0] : lane == 1 ? bw[1] : lane == 2 ? bw[2] : bw[3];
                    mask64[(size_t)(c0 + (uint32_t)j) * kPer + (uint32_t)lane] = w;
                }
                my_hits = lane == j ? tot : my_hits;
                whits += tot;
            }
            // one atomic per run of lanes holding chunks of the same Gaussian
            // (a Gaussian's chunks are consecutive slots)
            const uint32_t incl = wave_incl_scan(my_hits, lane);
            const uint32_t gprev = (uint32_t)__shfl_up((int)e.x, 1, kWave);
            const uint32_t gnext = (uint32_t)__shfl_down((int)e.x, 1, kWave);
            const bool head = lane == 0 || gprev != e.x;
            const bool tail = lane == kWave - 1 || gnext != e.x;
            const uint64_t heads = __ballot(head);
            // the run's first lane: the highest head at or below this lane
            const int first = 63 - __builtin_clzll(heads & (lane == kWave - 1 ? ~0ull : ((2ull << lane) - 1ull)));
            const uint32_t before = (uint32_t)__shfl((int)incl, first > 0 ? first - 1 : 0, kWave);
            const uint32_t run = incl - (first > 0 ? before : 0u);
            if (have && tail && run) atomicAdd(&count[e.x], run);
        }
    }
    if (lane == 0) s_hits[wv] = whits;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
#pragma unroll
        for (int w = 0; w < kBlock / kWave; ++w) t += s_hits[w];
        if (t) atomicAdd(&fc->pairs, t);
    }
}

}  // namespace

// Workgroups that fit on the device at once for a kernel (its register and
// LDS use decide the occupancy): a persistent grid of exactly that size
// keeps every CU busy without a tail of late workgroups.
template <class K>
static unsigned resident_blocks(K kernel) {
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess || per_cu <= 0 ||
        cus <= 0)
        return kPersistentBlocks;
    const unsigned n = (unsigned)(per_cu * cus);
    return n < (unsigned)kPersistentBlocks ? n : (unsigned)kPersistentBlocks;
}

unsigned preprocess_grid(int64_t P) {
    static const unsigned cap = resident_blocks(k_preprocess<false>);
    const int64_t b = (P + kBlock - 1) / kBlock;
    return (unsigned)(b < (int64_t)cap ? (b > 0 ? b : 1) : cap);
}

unsigned emit_grid(uint32_t visible) {
    static const unsigned cap = resident_blocks(k_super_emit);
    const uint32_t b = (visible + kBlock - 1) / kBlock;
    return b < cap ? (b > 0 ? b : 1u) : cap;
}

void launch_preprocess(const DevScene &sc, const DevPrepared *pp, const DevCamera &cam, const DevCam64 &cam64,
                       const DevOptions &op, int W, int H, GaussState *gs, float4 *conic, uint4 *rect, uint32_t *count,
                       uint8_t *count8, uint4 *erec, uint32_t *dkey, uint32_t *cand, uint32_t *seg_count,
                       uint32_t *gmap, uint2 *chunks, uint32_t chunk_cap, FrameCounters *fc, uint32_t *gsum_clear,
                       bool full, hipStream_t s) {
    if (sc.P <= 0) return;
    if (pp) {
        hipLaunchKernelGGL(k_preprocess<true>, dim3(preprocess_grid(sc.P)), dim3(kBlock), 0, s, sc, *pp, cam, cam64, op,
                           W, H, gs, conic, rect, count, count8, erec, dkey, cand, seg_count, gmap, chunks, chunk_cap,
                           fc, gsum_clear, (int)full, MultiOut{});
    } else {
        hipLaunchKernelGGL(k_preprocess<false>, dim3(preprocess_grid(sc.P)), dim3(kBlock), 0, s, sc, DevPrepared{},
                           cam, cam64, op, W, H, gs, conic, rect, count, count8, erec, dkey, cand, seg_count, gmap,
                           chunks, chunk_cap, fc, gsum_clear, (int)full, MultiOut{});
    }
}

void launch_cull(const DevScene &sc, const DevPrepared &pp, const DevCamera &cam, const DevOptions &op, int W, int H,
                 uint32_t *cand, uint32_t *seg_count, FrameCounters *fc, hipStream_t s) {
    if (sc.P <= 0) return;
    hipLaunchKernelGGL(k_cull<false>, dim3(kCullBlocks), dim3(kBlock), 0, s, sc, pp, cam, op, W, H, cand, seg_count,
                       fc, MultiOut{});
}

void launch_preprocess_multi(const DevScene &sc, const DevPrepared &pp, const MultiOut &mo, const DevOptions &op,
                             uint32_t *cand, uint32_t *seg_count, uint32_t *gmap, hipStream_t s) {
    if (sc.P <= 0 || mo.n < 1 || mo.n > kMaxCams) return;
    const CamOut &c0 = mo.c[0];
    hipLaunchKernelGGL(k_cull<true>, dim3(kCullBlocks), dim3(kBlock), 0, s, sc, pp, c0.cam, op, c0.W, c0.H, cand,
                       seg_count, c0.fc, mo);
    hipLaunchKernelGGL((k_preprocess<true, true>), dim3(preprocess_grid(sc.P)), dim3(kBlock), 0, s, sc, pp, c0.cam,
                       c0.cam64, op, c0.W, c0.H, c0.gs, c0.conic, c0.rect, c0.count, c0.count8, c0.erec, c0.dkey, cand,
                       seg_count, gmap, c0.chunks, c0.chunk_cap, c0.fc, c0.gsum_clear, 0, mo);
}

void launch_prepare(const DevScene &sc, const DevOptions &op, const uint32_t *perm, float4 *pos_o, float4 *cov,
                    float *sh, float2 *bnd, uint32_t *orig, int sh_stride, hipStream_t s) {
    if (sc.P <= 0) return;
    const int64_t blocks = (sc.P + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_prepare, dim3((unsigned)(blocks < 8192 ? blocks : 8192)), dim3(kBlock), 0, s, sc, op, perm,
                       pos_o, cov, sh, bnd, orig, sh_stride);
}

void launch_block_bounds(const float4 *pos_o, const float2 *bnd, int64_t P, float4 *blk, hipStream_t s) {
    if (P <= 0) return;
    hipLaunchKernelGGL(k_block_bounds, dim3((unsigned)((P + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, pos_o, bnd, P,
                       blk);
}

void launch_spatial_keys(const DevScene &sc, uint32_t *bounds, uint32_t *keys, hipStream_t s) {
    hipLaunchKernelGGL(k_spatial_bounds_init, dim3(1), dim3(64), 0, s, bounds);
    if (sc.P <= 0) return;
    const int64_t blocks = (sc.P + kBlock - 1) / kBlock;
    const unsigned grid = (unsigned)(blocks < 4096 ? blocks : 4096);
    hipLaunchKernelGGL(k_spatial_bounds, dim3(grid), dim3(kBlock), 0, s, sc, bounds);
    hipLaunchKernelGGL(k_spatial_keys, dim3(grid), dim3(kBlock), 0, s, sc, bounds, keys);
}

void launch_big_count(int W, int H, int binning, const GaussState *gs, const float4 *conic, const uint4 *erec,
                      const uint2 *chunks, uint32_t chunk_cap, uint32_t *chunk_mask, uint32_t *count,
                      FrameCounters *fc, hipStream_t s) {
    if (chunk_cap == 0) return;
    hipLaunchKernelGGL(k_big_count, dim3(kPersistentBlocks), dim3(kBlock), 0, s, W, H, binning, gs, conic, erec,
                       chunks, chunk_cap, chunk_mask, count, fc);
}

void launch_super_emit(int W, int H, const uint32_t *order, uint32_t visible, const uint32_t *visible_dev,
                       const uint32_t *offsets, const uint4 *erec, uint32_t ng, const uint2 *chunks, uint2 *big,
                       const uint32_t *chunk_mask, uint32_t chunk_cap, const FrameCounters *fc, uint16_t *skey,
                       uint32_t *gidx, uint64_t *smask, uint32_t ecap, uint2 *sranges, uint32_t nsuper,
                       uint32_t *gsum_clear, hipStream_t s) {
    (void)H;
    if (visible == 0 && (!sranges || nsuper == 0) && !gsum_clear) return;
    unsigned grid = emit_grid(visible);
    if (sranges) grid = std::max(grid, std::min<unsigned>((nsuper + kBlock - 1) / kBlock, kPersistentBlocks));
    hipLaunchKernelGGL(k_super_emit, dim3(grid), dim3(kBlock), 0, s, W, order, visible, visible_dev, offsets, erec,
                       big, chunk_cap, skey, gidx, smask, ecap, sranges, nsuper, gsum_clear, fc);
    if (chunk_cap == 0 || visible == 0) return;
    hipLaunchKernelGGL(k_big_entries, dim3(kPersistentBlocks), dim3(kBlock), 0, s, W, erec, ng, chunks, big,
                       chunk_cap, chunk_mask, fc, skey, gidx, smask, ecap);
}

}  // namespace fgs
