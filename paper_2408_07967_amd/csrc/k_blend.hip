// Per-tile front-to-back alpha blending with early termination (Sec. 2.2
// rendering stage; Sec. 5.2 early stop on saturated transmittance, opacity
// checks moved out of the per-pixel loop, base-2 exponent in log form).
//
// One 256-thread workgroup per 16 x 16 tile; each wavefront owns an 8 x 8
// quadrant, one pixel per lane.  The tile's sorted list is walked in batches
// of 256 Gaussians: every thread stages one Gaussian's 48-byte state in LDS
// and tests the ellipse against the four quadrant hulls (the same exact
// test as the tile binning, with a slightly inflated extent so it never
// drops a contributor), so a wavefront skips Gaussians that miss its quadrant
// with one scalar branch.  Per pixel and Gaussian:
//   q = A dx^2 + 2B dx dy + C dy^2; contributes iff q <= k^2;
//   alpha = min(alpha_max, 2^(log2 o - q log2(e) / 2));
//   T' = T (1 - alpha); if T' < T_stop the pixel stops before blending it;
//   C += colour alpha T; T = T'.
// A stopped lane moves its sample point to +1e30 so that q overflows and the
// Gaussian never contributes again: the hot loop carries no done-flag.
#include "fgs_internal.hpp"

namespace fgs {
namespace {

constexpr int kWave = 64;
constexpr float kFar = 1e30f;

// Conservative ellipse / rectangle test used only to skip work: the
// rectangle [X0, X1] x [Y0, Y1] in pixel-sample coordinates.
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

template <bool kCountWork, bool kLast>
__global__ __launch_bounds__(kBlock) void k_blend(const GaussState *__restrict__ gs,
                                                  const uint32_t *__restrict__ values,
                                                  const uint2 *__restrict__ ranges, int W, int H, int tiles_x,
                                                  DevOptions op, float *__restrict__ rgb, float *__restrict__ Tout,
                                                  uint32_t *__restrict__ last_out, unsigned long long *work) {
    __shared__ float4 s_f0[kBlock], s_f1[kBlock];
    __shared__ float2 s_f2[kBlock];
    // s_rel[q][w]: bit i set iff entry 64 w + i of the batch meets quadrant q
    __shared__ uint32_t s_rel[4][kBlock / kWave][2];

    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);  // wave-uniform
    const int tile = blockIdx.x;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int qx = wave & 1, qy = wave >> 1;
    const int pi = tx * kTile + qx * 8 + (lane & 7);
    const int pj = ty * kTile + qy * 8 + (lane >> 3);
    const bool in_img = pi < W && pj < H;
    float px = in_img ? (float)pi + 0.5f : kFar;
    const float py = (float)pj + 0.5f;

    const uint2 rg = ranges[tile];
    const uint32_t start = rg.x, end = rg.y;
    float T = 1.0f, c0 = 0.0f, c1 = 0.0f, c2 = 0.0f;
    uint32_t last = 0;
    bool done = !in_img;
    bool wave_done = __ballot(!done) == 0;
    uint32_t examined = in_img ? (end - start) : 0u;  // entries this pixel must look at
    const float nl2e = -0.72134752044448170f;          // -log2(e) / 2
    // loop-invariant clamp as the result of an arithmetic op (a canonical
    // value, so the minimum needs no per-iteration canonicalisation)
    const float amax = op.alpha_max + 0.0f;
    const float tstop = op.T_stop;

    for (uint32_t b0 = start; b0 < end; b0 += kBlock) {
        const uint32_t nb = (end - b0) < (uint32_t)kBlock ? (end - b0) : (uint32_t)kBlock;
        uint32_t qm = 0;
        if ((uint32_t)tid < nb) {
            const GaussState s = gs[values[b0 + tid]];
            const float k2i = s.f1.y * 1.00002f + 1e-5f;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int X0i = tx * kTile + (q & 1) * 8, Y0i = ty * kTile + (q >> 1) * 8;
                int X1i = X0i + 8, Y1i = Y0i + 8;
                X1i = X1i > W ? W : X1i;
                Y1i = Y1i > H ? H : Y1i;
                if (X0i < X1i && Y0i < Y1i &&
                    rect_hit(s.f0.x, s.f0.y, s.f0.z, s.f0.w, s.f1.x, k2i, (float)X0i + 0.5f, (float)X1i - 0.5f,
                             (float)Y0i + 0.5f, (float)Y1i - 0.5f))
                    qm |= 1u << q;
            }
            // 2B in place of B for the pixel loop
            s_f0[tid] = make_float4(s.f0.x, s.f0.y, s.f0.z, 2.0f * s.f0.w);
            s_f1[tid] = s.f1;
            s_f2[tid] = make_float2(s.f2.x, s.f2.y);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint64_t bq = __ballot((qm >> q) & 1u);
            if (lane == 0) {
                s_rel[q][wave][0] = (uint32_t)bq;
                s_rel[q][wave][1] = (uint32_t)(bq >> 32);
            }
        }
        __syncthreads();
        if (!wave_done) {
            for (int wd = 0; wd < kBlock / kWave && !wave_done; ++wd) {
                uint64_t m = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)s_rel[wave][wd][0]) |
                             ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)s_rel[wave][wd][1]) << 32);
                while (m) {
                    const int j = wd * kWave + __builtin_ctzll(m);
                    m &= m - 1;
                    const float4 f0 = s_f0[j], f1 = s_f1[j];
                    const float2 f2 = s_f2[j];
                    const float dx = px - f0.x, dy = py - f0.y;
                    const float t = fmaf(f0.z, dx, f0.w * dy);
                    const float q = fmaf(f1.x * dy, dy, dx * t);
                    bool inq = q <= f1.y;
                    const float e = __builtin_amdgcn_exp2f(fmaf(q, nl2e, f1.z));
                    float a = inq ? fminf(e, amax) : 0.0f;
                    float Tn = fmaf(-a, T, T);
                    const bool stop = Tn < tstop;
                    if (__ballot(stop) != 0) {
                        // rare path: lanes that saturate stop before this Gaussian
                        if (stop) {
                            a = 0.0f;
                            Tn = T;
                            inq = false;
                            px = kFar;
                            done = true;
                            if (kCountWork) examined = b0 - start + (uint32_t)j + 1u;
                        }
                        wave_done = __ballot(!done) == 0;
                    }
                    const float wgt = a * T;
                    c0 = fmaf(wgt, f1.w, c0);
                    c1 = fmaf(wgt, f2.x, c1);
                    c2 = fmaf(wgt, f2.y, c2);
                    T = Tn;
                    if (kLast) last = inq ? (b0 - start + (uint32_t)j + 1u) : last;
                    if (wave_done) break;
                }
            }
        }
        // all 256 pixels finished: stop walking the list (also the barrier
        // that protects the staging buffers)
        if (__syncthreads_count(done ? 1 : 0) == kBlock) break;
    }

    if (kCountWork) {
        // a wave that skipped a Gaussian whose ellipse misses its quadrant
        // still counts it: the count is the method's, not this kernel's
        unsigned long long v = examined;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d, kWave);
        if (lane == 0) atomicAdd(work, v);
    }
    if (in_img) {
        const size_t hw = (size_t)W * H;
        const size_t p = (size_t)pj * W + pi;
        rgb[p] = c0 + T * op.bg[0];
        rgb[hw + p] = c1 + T * op.bg[1];
        rgb[2 * hw + p] = c2 + T * op.bg[2];
        if (Tout) Tout[p] = T;
        if (kLast && last_out) last_out[p] = last;
    }
}

}  // namespace

void launch_blend(const GaussState *gs, const uint32_t *values, const uint2 *ranges, int W, int H,
                  const DevOptions &op, float *rgb, float *T, uint32_t *last, unsigned long long *work,
                  hipStream_t s) {
    const int tiles_x = (W + kTile - 1) / kTile, tiles_y = (H + kTile - 1) / kTile;
    const dim3 grid((unsigned)(tiles_x * tiles_y)), block(kBlock);
    if (work)
        hipLaunchKernelGGL((k_blend<true, true>), grid, block, 0, s, gs, values, ranges, W, H, tiles_x, op, rgb, T,
                           last, work);
    else if (last)
        hipLaunchKernelGGL((k_blend<false, true>), grid, block, 0, s, gs, values, ranges, W, H, tiles_x, op, rgb, T,
                           last, work);
    else
        hipLaunchKernelGGL((k_blend<false, false>), grid, block, 0, s, gs, values, ranges, W, H, tiles_x, op, rgb,
                           T, last, work);
}

}  // namespace fgs
