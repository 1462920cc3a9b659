// Tile-range extraction from the sorted tile ids (each tile's workload is its
// run of the sorted list, Sec. 2.2) and a fill kernel used to clear counters.
#include "fgs_internal.hpp"

namespace fgs {
namespace {

__global__ void k_fill_u32(uint32_t *p, uint32_t value, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// ranges[t] = [first, last + 1) of tile t in the sorted keys (empty: [0, 0)).
// n_dev, if given, holds the actual key count (at most n).
__global__ void k_tile_ranges(const uint32_t *__restrict__ keys, uint32_t n, const uint32_t *__restrict__ n_dev,
                              uint2 *__restrict__ ranges, uint32_t ntiles) {
    if (n_dev) n = min(n, *n_dev);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t t = keys[i];
        if (t >= ntiles) continue;
        if (i == 0 || keys[i - 1] != t) ranges[t].x = i;
        if (i + 1 == n || keys[i + 1] != t) ranges[t].y = i + 1;
    }
}

}  // namespace

void launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t s) {
    if (n == 0) return;
    size_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(kBlock), 0, s, p, value, n);
}

void launch_tile_ranges(const uint32_t *tile_keys, uint32_t n, const uint32_t *n_dev, uint2 *ranges,
                        uint32_t ntiles, hipStream_t s) {
    launch_fill_u32(reinterpret_cast<uint32_t *>(ranges), 0u, (size_t)ntiles * 2, s);
    if (n == 0) return;
    uint32_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_tile_ranges, dim3(blocks), dim3(kBlock), 0, s, tile_keys, n, n_dev, ranges, ntiles);
}

}  // namespace fgs
