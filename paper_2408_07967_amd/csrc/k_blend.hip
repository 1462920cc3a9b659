// Per-tile front-to-back alpha blending with early termination (Sec. 2.2
// rendering stage; Sec. 5.2 early stop on saturated transmittance, opacity
// checks moved out of the per-pixel loop; Sec. 5.3.2 exponent in log form).
//
// One 128-thread workgroup per 16 x 16 tile: each wavefront owns a 16 x 8
// half, each lane two horizontally adjacent pixels, so the row terms of the
// quadratic form, the LDS reads and the loop control are shared by two
// pixels.  The tile's sorted list is walked in batches of 128 Gaussians
// (6.4 KB of LDS per workgroup: eight wavefronts per SIMD fit):
// every thread stages one Gaussian (the coefficients of the exponent,
// opacity threshold and colour) in LDS and tests each ellipse against the two
// halves (the exact tile test with a slightly inflated extent, so it never
// drops a contributor); a wavefront walks only the set bits of its half's
// masks, in scalar code.  Per pixel and Gaussian:
//   E = log2 o - q log2(e) / 2; contributes iff E >= log2 o - k^2 log2(e) / 2;
//   alpha = min(alpha_max, 2^E);
//   T' = T (1 - alpha); if T' < T_stop the pixel stops before blending it;
//   C += colour alpha T; T = T'.
// A stopped pixel moves its sample point to +1e30 so that E becomes -inf and
// the Gaussian never contributes again: the hot loop carries no done-flag.
#include "fgs_internal.hpp"
#include "blend_common.hpp"

namespace fgs {
namespace {

constexpr int kWave = 64;
constexpr int kThreads = 128;        // two wavefronts per tile
constexpr int kBatch = 128;          // Gaussians staged per batch
constexpr int kWords = kBatch / kWave;
constexpr float kFar = 1e30f;

struct Pixel {
    float x;        // sample x, or kFar once stopped
    float T, c0, c1, c2;
    uint32_t last;
    uint32_t examined;
    bool done;
};

// Alpha and transmittance of one pixel for one Gaussian, before the
// termination check.
struct Step {
    float a, Tn;
    bool in, stop;
};

__device__ __forceinline__ Step step(const Pixel &p, float e, float thr, float amax, float tstop) {
    Step st;
    st.in = e >= thr;
    // min(2^E, amax) as a clamp to [0, amax] (2^E >= 0): one v_med3_f32, with
    // no per-iteration canonicalisation of amax that a minimum would bring
    st.a = st.in ? __builtin_amdgcn_fmed3f(__builtin_amdgcn_exp2f(e), 0.0f, amax) : 0.0f;
    st.Tn = fmaf(-st.a, p.T, p.T);
    st.stop = st.Tn < tstop;
    return st;
}

// The pixel saturates: it stops before this Gaussian (rare path).
template <bool kCountWork>
__device__ __forceinline__ void stop_before(Pixel &p, Step &st, uint32_t pos) {
    st.a = 0.0f;
    st.Tn = p.T;
    st.in = false;
    p.x = kFar;
    p.done = true;
    if (kCountWork) p.examined = pos + 1u;
}

template <bool kLast>
__device__ __forceinline__ void apply(Pixel &p, const Step &st, const float4 &f1, const float2 &f2, uint32_t pos) {
    const float w = st.a * p.T;
    p.c0 = fmaf(w, f1.w, p.c0);
    p.c1 = fmaf(w, f2.x, p.c1);
    p.c2 = fmaf(w, f2.y, p.c2);
    p.T = st.Tn;
    if (kLast) p.last = st.in ? pos + 1u : p.last;
}

template <bool kCountWork, bool kLast>
__global__ __launch_bounds__(kThreads) void k_blend(const GaussState *__restrict__ gs,
                                                    const uint32_t *__restrict__ values,
                                                    const uint2 *__restrict__ ranges, int W, int H, int tiles_x,
                                                    DevOptions op, float *__restrict__ rgb, float *__restrict__ Tout,
                                                    uint32_t *__restrict__ last_out, unsigned long long *work) {
    // one float4 stride for all three arrays: a single LDS address per Gaussian
    __shared__ float4 s_f0[kBatch], s_f1[kBatch], s_f2[kBatch];
    // s_rel[h][w]: bit i set iff entry 64 w + i of the batch meets half h
    __shared__ uint32_t s_rel[2][kWords][2];

    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);  // wave-uniform
    const int tile = blockIdx.x;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int pi0 = tx * kTile + 2 * (lane & 7);
    const int pj = ty * kTile + wave * 8 + (lane >> 3);
    const bool in0 = pi0 < W && pj < H, in1 = pi0 + 1 < W && pj < H;
    const float py = (float)pj + 0.5f;

    const uint2 rg = ranges[tile];
    const uint32_t start = rg.x, end = rg.y > rg.x ? rg.y : rg.x;  // an empty tile may hold start > end
    Pixel p0{in0 ? (float)pi0 + 0.5f : kFar, 1.0f, 0.0f, 0.0f, 0.0f, 0u, in0 ? end - start : 0u, !in0};
    Pixel p1{in1 ? (float)pi0 + 1.5f : kFar, 1.0f, 0.0f, 0.0f, 0.0f, 0u, in1 ? end - start : 0u, !in1};
    bool wave_done = __ballot(!(p0.done && p1.done)) == 0;
    // loop-invariant clamp as the result of an arithmetic op (a canonical
    // value, so the minimum needs no per-iteration canonicalisation)
    const float amax = op.alpha_max + 0.0f;
    const float tstop = op.T_stop;
    uint32_t wsteps = 0;  // kCountWork: entries this wavefront evaluates (uniform)

    for (uint32_t b0 = start; b0 < end; b0 += kBatch) {
        const uint32_t nb = (end - b0) < (uint32_t)kBatch ? (end - b0) : (uint32_t)kBatch;
#pragma unroll
        for (int r = 0; r < kBatch / kThreads; ++r) {
            const uint32_t i = (uint32_t)(r * kThreads + tid);
            uint32_t hm = 0;
            if (i < nb) {
                const GaussState s = gs[values[b0 + i]];
                const float k2i = s.f1.y * 1.00002f + 1e-5f;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int X0i = tx * kTile, Y0i = ty * kTile + h * 8;
                    int X1i = X0i + kTile, Y1i = Y0i + 8;
                    X1i = X1i > W ? W : X1i;
                    Y1i = Y1i > H ? H : Y1i;
                    if (Y0i < Y1i && rect_hit(s.f0.x, s.f0.y, s.f0.z, s.f0.w, s.f1.x, k2i, (float)X0i + 0.5f,
                                              (float)X1i - 0.5f, (float)Y0i + 0.5f, (float)Y1i - 0.5f))
                        hm |= 1u << h;
                }
                float4 f0, f1;
                float2 f2;
                stage_gauss(s, f0, f1, f2);
                s_f0[i] = f0;
                s_f1[i] = f1;
                s_f2[i] = make_float4(f2.x, f2.y, 0.0f, 0.0f);
            }
            // entry i = 128 r + 64 wave + lane: word 2 r + wave, bit lane
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const uint64_t bq = __ballot((hm >> h) & 1u);
                if (lane == 0) {
                    s_rel[h][2 * r + wave][0] = (uint32_t)bq;
                    s_rel[h][2 * r + wave][1] = (uint32_t)(bq >> 32);
                }
            }
        }
        __syncthreads();
        if (!wave_done) {
            for (int wd = 0; wd < kWords && !wave_done; ++wd) {
                uint64_t m = (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)s_rel[wave][wd][0]) |
                             ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)s_rel[wave][wd][1]) << 32);
                // one staged Gaussian for both pixels of the lane; true once
                // every pixel of the wavefront has stopped
                auto blend_one = [&](int j) {
                    if (kCountWork) ++wsteps;
                    const float4 f0 = s_f0[j], f1 = s_f1[j];
                    const float2 f2 = *reinterpret_cast<const float2 *>(&s_f2[j]);
                    const RowTerms rt = row_terms(f0, f1, py);
                    const float e0 = exponent_at(f0, rt, p0.x);
                    const float e1 = exponent_at(f0, rt, p1.x);
                    const uint32_t pos = b0 - start + (uint32_t)j;
                    Step s0 = step(p0, e0, f1.y, amax, tstop);
                    Step s1 = step(p1, e1, f1.y, amax, tstop);
                    if (__ballot(s0.stop || s1.stop) != 0) {
                        if (s0.stop) stop_before<kCountWork>(p0, s0, pos);
                        if (s1.stop) stop_before<kCountWork>(p1, s1, pos);
                        wave_done = __ballot(!(p0.done && p1.done)) == 0;
                    }
                    apply<kLast>(p0, s0, f1, f2, pos);
                    apply<kLast>(p1, s1, f1, f2, pos);
                    return wave_done;
                };
                // two Gaussians per trip (the loop-carried state alternates
                // between register sets instead of being copied back)
                while (m) {
                    const int ja = wd * kWave + __builtin_ctzll(m);
                    m &= m - 1;
                    if (blend_one(ja) || !m) break;
                    const int jb = wd * kWave + __builtin_ctzll(m);
                    m &= m - 1;
                    if (blend_one(jb)) break;
                }
            }
        }
        // all 256 pixels finished: stop walking the list (also the barrier
        // that protects the staging buffers)
        if (__syncthreads_count((p0.done && p1.done) ? 1 : 0) == kThreads) break;
    }

    if (kCountWork) {
        // a wave that skipped a Gaussian whose ellipse misses its half still
        // counts it: the count is the method's, not this kernel's
        unsigned long long v = (unsigned long long)p0.examined + p1.examined;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d, kWave);
        if (lane == 0) {
            atomicAdd(work, v);
            atomicAdd(work + 1, (unsigned long long)wsteps);
        }
    }
    const size_t hw = (size_t)W * H;
    const size_t q = (size_t)pj * W + pi0;
    if (in0) {
        rgb[q] = p0.c0 + p0.T * op.bg[0];
        rgb[hw + q] = p0.c1 + p0.T * op.bg[1];
        rgb[2 * hw + q] = p0.c2 + p0.T * op.bg[2];
        if (Tout) Tout[q] = p0.T;
        if (kLast && last_out) last_out[q] = p0.last;
    }
    if (in1) {
        rgb[q + 1] = p1.c0 + p1.T * op.bg[0];
        rgb[hw + q + 1] = p1.c1 + p1.T * op.bg[1];
        rgb[2 * hw + q + 1] = p1.c2 + p1.T * op.bg[2];
        if (Tout) Tout[q + 1] = p1.T;
        if (kLast && last_out) last_out[q + 1] = p1.last;
    }
}

// Variant of the blend (selected per context): each wavefront walks its
// tile's whole list on its own with a software prefetch pipeline, the form
// of the paper's render loop (Sec. 5.3.2): while entry i is blended, the
// state of entry i + 1 and the index of entry i + 2 are in flight (vector
// buffer loads, which complete in order, so the wait for entry i's state
// leaves the later loads outstanding).  Nothing is staged in LDS and no half
// mask is kept: every entry is evaluated for the wavefront's 128 pixels; an
// entry whose ellipse misses a pixel gives it alpha 0, which leaves colour,
// transmittance and last contributor exactly as they were, so the image is
// bit for bit the one of k_blend.
template <bool kLast>
__global__ __launch_bounds__(kThreads) void k_blend_prefetch(const GaussState *__restrict__ gs,
                                                             const uint32_t *__restrict__ values,
                                                             const uint2 *__restrict__ ranges, int W, int H,
                                                             int tiles_x, uint32_t nvalues, uint32_t ngs,
                                                             DevOptions op, float *__restrict__ rgb,
                                                             float *__restrict__ Tout, uint32_t *__restrict__ last_out) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);  // wave-uniform
    const int tile = blockIdx.x;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int pi0 = tx * kTile + 2 * (lane & 7);
    const int pj = ty * kTile + wave * 8 + (lane >> 3);
    const bool in0 = pi0 < W && pj < H, in1 = pi0 + 1 < W && pj < H;
    const float py = (float)pj + 0.5f;

    const uint2 rg = ranges[tile];
    const uint32_t start = rg.x, end = rg.y > rg.x ? rg.y : rg.x;  // an empty tile may hold start > end
    Pixel p0{in0 ? (float)pi0 + 0.5f : kFar, 1.0f, 0.0f, 0.0f, 0.0f, 0u, 0u, !in0};
    Pixel p1{in1 ? (float)pi0 + 1.5f : kFar, 1.0f, 0.0f, 0.0f, 0.0f, 0u, 0u, !in1};
    bool wave_done = __ballot(!(p0.done && p1.done)) == 0;
    const float amax = op.alpha_max + 0.0f;
    const float tstop = op.T_stop;

    if (!wave_done && start < end) {
        // bounds-checked buffer loads with a wave-uniform offset
        const __amdgpu_buffer_rsrc_t vrs =
            __builtin_amdgcn_make_buffer_rsrc(const_cast<uint32_t *>(values), (short)0, (int)(nvalues * 4u), 0x00020000);
        const __amdgpu_buffer_rsrc_t grs = __builtin_amdgcn_make_buffer_rsrc(
            const_cast<GaussState *>(gs), (short)0, (int)(ngs * (uint32_t)sizeof(GaussState)), 0x00020000);
        auto index = [&](uint32_t i) -> uint32_t {  // entry i's Gaussian (past the list: entry start's)
            return (uint32_t)__builtin_amdgcn_raw_buffer_load_b32(vrs, (i < end ? i : start) * 4u, 0, 0);
        };
        auto state = [&](uint32_t g) -> GaussState {
            GaussState st;
            const uint32_t o = g * (uint32_t)sizeof(GaussState);
            const auto v0 = __builtin_amdgcn_raw_buffer_load_b128(grs, o, 0, 0);
            const auto v1 = __builtin_amdgcn_raw_buffer_load_b128(grs, o + 16u, 0, 0);
            const auto v2 = __builtin_amdgcn_raw_buffer_load_b128(grs, o + 32u, 0, 0);
            st.f0 = make_float4(__uint_as_float(v0[0]), __uint_as_float(v0[1]), __uint_as_float(v0[2]),
                                __uint_as_float(v0[3]));
            st.f1 = make_float4(__uint_as_float(v1[0]), __uint_as_float(v1[1]), __uint_as_float(v1[2]),
                                __uint_as_float(v1[3]));
            st.f2 = make_float4(__uint_as_float(v2[0]), __uint_as_float(v2[1]), __uint_as_float(v2[2]),
                                __uint_as_float(v2[3]));
            return st;
        };
        // one entry for both pixels of the lane; true once every pixel of the
        // wavefront has stopped
        auto blend_one = [&](const GaussState &gsx, uint32_t pos) {
            float4 f0, f1;
            float2 f2;
            stage_gauss(gsx, f0, f1, f2);
            const RowTerms rt = row_terms(f0, f1, py);
            const float e0 = exponent_at(f0, rt, p0.x);
            const float e1 = exponent_at(f0, rt, p1.x);
            Step s0 = step(p0, e0, f1.y, amax, tstop);
            Step s1 = step(p1, e1, f1.y, amax, tstop);
            if (__ballot(s0.stop || s1.stop) != 0) {
                if (s0.stop) stop_before<false>(p0, s0, pos);
                if (s1.stop) stop_before<false>(p1, s1, pos);
                wave_done = __ballot(!(p0.done && p1.done)) == 0;
            }
            apply<kLast>(p0, s0, f1, f2, pos);
            apply<kLast>(p1, s1, f1, f2, pos);
            return wave_done;
        };
        // two entries per trip, so that the prefetched values alternate
        // between two register sets instead of being copied
        uint32_t i = start;
        uint32_t inext = index(i + 1);
        GaussState sa = state(index(i)), sb;
        for (;;) {
            sb = state(inext);                // entry i + 1
            const uint32_t inn = index(i + 2);
            if (blend_one(sa, i - start) || ++i >= end) break;
            sa = state(inn);                  // entry i + 1
            const uint32_t in3 = index(i + 2);
            if (blend_one(sb, i - start) || ++i >= end) break;
            inext = in3;
        }
    }

    const size_t hw = (size_t)W * H;
    const size_t q = (size_t)pj * W + pi0;
    if (in0) {
        rgb[q] = p0.c0 + p0.T * op.bg[0];
        rgb[hw + q] = p0.c1 + p0.T * op.bg[1];
        rgb[2 * hw + q] = p0.c2 + p0.T * op.bg[2];
        if (Tout) Tout[q] = p0.T;
        if (kLast && last_out) last_out[q] = p0.last;
    }
    if (in1) {
        rgb[q + 1] = p1.c0 + p1.T * op.bg[0];
        rgb[hw + q + 1] = p1.c1 + p1.T * op.bg[1];
        rgb[2 * hw + q + 1] = p1.c2 + p1.T * op.bg[2];
        if (Tout) Tout[q + 1] = p1.T;
        if (kLast && last_out) last_out[q + 1] = p1.last;
    }
}

}  // namespace

void launch_blend(const GaussState *gs, const uint32_t *values, const uint2 *ranges, int W, int H,
                  const DevOptions &op, float *rgb, float *T, uint32_t *last, unsigned long long *work,
                  int variant, uint32_t nvalues, uint32_t ngs, hipStream_t s) {
    const int tiles_x = (W + kTile - 1) / kTile, tiles_y = (H + kTile - 1) / kTile;
    const dim3 grid((unsigned)(tiles_x * tiles_y)), block(kThreads);
    if (variant == 1 && !work && nvalues > 0 && ngs > 0) {
        if (last)
            hipLaunchKernelGGL((k_blend_prefetch<true>), grid, block, 0, s, gs, values, ranges, W, H, tiles_x, nvalues,
                               ngs, op, rgb, T, last);
        else
            hipLaunchKernelGGL((k_blend_prefetch<false>), grid, block, 0, s, gs, values, ranges, W, H, tiles_x,
                               nvalues, ngs, op, rgb, T, last);
        return;
    }
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
