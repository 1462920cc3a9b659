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
__global__ void k_tile_ranges(const uint32_t *__restrict__ keys, uint32_t n, uint2 *__restrict__ ranges,
                              uint32_t ntiles) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t t = keys[i];
    if (t >= ntiles) return;
    if (i == 0 || keys[i - 1] != t) ranges[t].x = i;
    if (i + 1 == n || keys[i + 1] != t) ranges[t].y = i + 1;
}

}  // namespace

void launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t s) {
    if (n == 0) return;
    size_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(kBlock), 0, s, p, value, n);
}

void launch_tile_ranges(const uint32_t *tile_keys, uint32_t n, uint2 *ranges, uint32_t ntiles, hipStream_t s) {
    launch_fill_u32(reinterpret_cast<uint32_t *>(ranges), 0u, (size_t)ntiles * 2, s);
    if (n == 0) return;
    hipLaunchKernelGGL(k_tile_ranges, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, tile_keys, n, ranges,
                       ntiles);
}

}  // namespace fgs
