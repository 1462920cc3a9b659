// Tile ranges (each tile's workload is its run of the sorted list, Sec. 2.2):
// their initial empty state, which the last tile-sort pass narrows, the range
// of a one-tile image, and a fill kernel used to clear counters.
#include "fgs_internal.hpp"

namespace fgs {
namespace {

__global__ void k_fill_u32(uint32_t *p, uint32_t value, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// The one range of a one-tile image: every pair (*n_dev of them, at most n).
__global__ void k_single_range(uint2 *__restrict__ ranges, uint32_t n, const uint32_t *__restrict__ n_dev) {
    if (threadIdx.x == 0) ranges[0] = make_uint2(0u, min(n, *n_dev));
}

__global__ void k_init_ranges(uint2 *__restrict__ ranges, uint32_t ntiles) {
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < ntiles; t += gridDim.x * blockDim.x)
        ranges[t] = make_uint2(0xffffffffu, 0u);
}

}  // namespace

void launch_init_ranges(uint2 *ranges, uint32_t ntiles, hipStream_t s) {
    if (ntiles == 0) return;
    uint32_t blocks = (ntiles + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_init_ranges, dim3(blocks), dim3(kBlock), 0, s, ranges, ntiles);
}

void launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t s) {
    if (n == 0) return;
    size_t blocks = (n + kBlock - 1) / kBlock;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)blocks), dim3(kBlock), 0, s, p, value, n);
}

void launch_single_range(uint2 *ranges, uint32_t n, const uint32_t *n_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_single_range, dim3(1), dim3(64), 0, s, ranges, n, n_dev);
}

}  // namespace fgs
