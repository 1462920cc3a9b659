// Kernel-launcher stand-ins for the host-only sanitizer build of the runtime
// (runtime.cpp, pipeline.cpp, server.cpp compiled for the host with
// AddressSanitizer and UBSan, without the .hip kernel files).  The sanitizer
// driver exercises argument validation, error paths and the admission
// arena, none of which reaches a kernel launch; reaching one means a path
// launched work without a device, which the driver reports as a failure.
// The signatures are those of fgs_internal.hpp, so any drift fails to link.
#include <cstdio>
#include <cstdlib>

#include "fgs_internal.hpp"

namespace {
[[noreturn]] void reached(const char *what) {
    std::fprintf(stderr, "kernel launcher %s reached in the host-only build\n", what);
    std::abort();
}
}  // namespace

namespace fgs {

void launch_fill_u32(uint32_t *, uint32_t, size_t, hipStream_t) { reached("fill_u32"); }
hipError_t noalloc_scratch(int, unsigned char **) { reached("noalloc_scratch"); }
void launch_peak_fma(int, int, float *, hipStream_t) { reached("peak_fma"); }
void launch_peak_exp(int, int, float *, hipStream_t) { reached("peak_exp"); }
void launch_peak_copy(const void *, void *, size_t, hipStream_t) { reached("peak_copy"); }
unsigned preprocess_grid(int64_t) { reached("preprocess_grid"); }
unsigned emit_grid(uint32_t) { reached("emit_grid"); }
void launch_preprocess(const DevScene &, const DevPrepared *, const DevCamera &, const DevCam64 &, const DevOptions &, int, int,
                       GaussState *, float4 *, uint4 *, uint32_t *, uint8_t *, uint4 *, uint32_t *, uint32_t *,
                       uint32_t *, uint32_t *, uint2 *, uint32_t, FrameCounters *, uint32_t *, bool, hipStream_t) {
    reached("preprocess");
}
void launch_cull(const DevScene &, const DevPrepared &, const DevCamera &, const DevOptions &, int, int, uint32_t *,
                 uint32_t *, FrameCounters *, hipStream_t) {
    reached("cull");
}
void launch_preprocess_multi(const DevScene &, const DevPrepared &, const MultiOut &, const DevOptions &, uint32_t *,
                             uint32_t *, uint32_t *, hipStream_t) {
    reached("preprocess_multi");
}
void launch_prepare(const DevScene &, const DevOptions &, const uint32_t *, float4 *, float4 *, float *, float2 *,
                    uint32_t *, int, hipStream_t) {
    reached("prepare");
}
void launch_spatial_keys(const DevScene &, uint32_t *, uint32_t *, hipStream_t) { reached("spatial_keys"); }
void launch_block_bounds(const float4 *, const float2 *, int64_t, float4 *, hipStream_t) { reached("block_bounds"); }
void launch_depth_ties(const uint32_t *, uint32_t *, const uint32_t *, uint32_t, const uint32_t *, uint32_t *,
                       FrameCounters *, uint32_t *, hipStream_t) {
    reached("depth_ties");
}
void launch_big_count(int, int, int, const GaussState *, const float4 *, const uint4 *, const uint2 *, uint32_t,
                      uint32_t *, uint32_t *, FrameCounters *, hipStream_t) {
    reached("big_count");
}
void launch_super_emit(int, int, const uint32_t *, uint32_t, const uint32_t *, const uint32_t *, const uint4 *,
                       uint32_t, const uint2 *, uint2 *, const uint32_t *, uint32_t, const FrameCounters *, uint16_t *,
                       uint32_t *, uint64_t *, uint32_t, uint2 *, uint32_t, uint32_t *, hipStream_t) {
    reached("super_emit");
}
void launch_tile_lists(int, int, const uint2 *, const uint32_t *, const uint64_t *, uint32_t, uint32_t *, uint2 *,
                       uint32_t *, uint32_t, hipStream_t) {
    reached("tile_lists");
}
void launch_radix_pass(const void *, const uint32_t *, void *, uint32_t *, uint32_t, const uint32_t *, int, int, bool,
                       bool, uint32_t *, uint32_t *, uint32_t *, hipStream_t, uint2 *, uint32_t, int, const uint64_t *,
                       uint64_t *, bool) {
    reached("radix_pass");
}
void launch_count_scan(const uint32_t *, const uint8_t *, const uint4 *, uint32_t, const uint32_t *, uint32_t *,
                       uint32_t *, uint32_t *, uint32_t *, hipStream_t) {
    reached("count_scan");
}
void launch_single_range(uint2 *, uint32_t, const uint32_t *, hipStream_t) { reached("single_range"); }
void launch_blend(const GaussState *, const uint32_t *, const uint2 *, int, int, const DevOptions &, float *, float *,
                  uint32_t *, unsigned long long *, int, uint32_t, uint32_t, hipStream_t) {
    reached("blend");
}
void launch_blend_backward(const GaussState *, const uint32_t *, const uint2 *, const float *, const uint32_t *,
                           const float *, int, int, const DevOptions &, float *, int64_t, hipStream_t) {
    reached("blend_backward");
}
void launch_preprocess_backward(const DevScene &, const DevCamera &, const DevOptions &, int, int, const GaussState *,
                                const float *, int64_t, float *, float *, float *, float *, float *, int64_t,
                                hipStream_t) {
    reached("preprocess_backward");
}

}  // namespace fgs
