// Measured peak rates of the device, the denominators beside the published
// ones for the rooflines: binary32 FMA issue (non-packed), v_exp_f32 issue,
// and device-to-device copy bandwidth.  Each rate comes from a kernel that
// does nothing but that operation over enough wavefronts to fill every SIMD.
#include "fgs_internal.hpp"

namespace fgs {
namespace {

constexpr int kChains = 8;  // independent dependency chains per lane

// kIters x kChains FMAs per lane on registers; m and c come from the host so
// nothing folds, and the result is stored only if it equals a value it never
// takes, so nothing is dead.
__global__ __launch_bounds__(kBlock) void k_peak_fma(float m, float c, int iters, float *sink) {
    float a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = (float)(threadIdx.x + j);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = __builtin_fmaf(a[j], m, c);
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    if (s == -1.2345e-30f) sink[0] = s;
}

// kIters x kChains v_exp_f32 per lane.
__global__ __launch_bounds__(kBlock) void k_peak_exp(float x0, int iters, float *sink) {
    float a[kChains];
#pragma unroll
    for (int j = 0; j < kChains; ++j) a[j] = x0 - (float)(threadIdx.x + j);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int j = 0; j < kChains; ++j) a[j] = __builtin_amdgcn_exp2f(a[j]);
    }
    float s = 0.0f;
#pragma unroll
    for (int j = 0; j < kChains; ++j) s += a[j];
    if (s == -1.2345e-30f) sink[0] = s;
}

// Grid-stride copy of n 16-byte elements.
__global__ __launch_bounds__(kBlock) void k_peak_copy(const uint4 *__restrict__ src, uint4 *__restrict__ dst,
                                                      size_t n) {
    for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (size_t)gridDim.x * kBlock)
        dst[i] = src[i];
}

}  // namespace

void launch_peak_fma(int blocks, int iters, float *sink, hipStream_t s) {
    hipLaunchKernelGGL(k_peak_fma, dim3(blocks), dim3(kBlock), 0, s, 0.999999f, 1e-7f, iters, sink);
}

void launch_peak_exp(int blocks, int iters, float *sink, hipStream_t s) {
    hipLaunchKernelGGL(k_peak_exp, dim3(blocks), dim3(kBlock), 0, s, -3.0f, iters, sink);
}

void launch_peak_copy(const void *src, void *dst, size_t bytes, hipStream_t s) {
    const size_t n = bytes / sizeof(uint4);
    hipLaunchKernelGGL(k_peak_copy, dim3(8192), dim3(kBlock), 0, s, static_cast<const uint4 *>(src),
                       static_cast<uint4 *>(dst), n);
}

}  // namespace fgs
