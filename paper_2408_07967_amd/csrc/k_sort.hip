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
// n_dev, if given, holds the actual key count (at most n).  Each thread
// takes four consecutive keys with one 16-byte load (keys is 16-byte
// aligned) and compares them with their neighbours.
__global__ void k_tile_ranges(const uint32_t *__restrict__ keys, uint32_t n, const uint32_t *__restrict__ n_dev,
                              uint2 *__restrict__ ranges, uint32_t ntiles) {
    if (n_dev) n = min(n, *n_dev);
    const uint32_t nq = (n + 3) / 4;
    for (uint32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) {
        const uint32_t i0 = 4 * q;
        uint32_t k[6];
        if (i0 + 4 <= n) {
            const uint4 v = reinterpret_cast<const uint4 *>(keys)[q];
            k[1] = v.x;
            k[2] = v.y;
            k[3] = v.z;
            k[4] = v.w;
        } else {
            for (int j = 0; j < 4; ++j) k[1 + j] = i0 + j < n ? keys[i0 + j] : 0xffffffffu;
        }
        k[0] = i0 > 0 ? keys[i0 - 1] : 0xffffffffu;
        k[5] = i0 + 4 < n ? keys[i0 + 4] : 0xffffffffu;
#pragma unroll
        for (int j = 1; j <= 4; ++j) {
            const uint32_t i = i0 + (uint32_t)(j - 1);
            const uint32_t t = k[j];
            if (i >= n || t >= ntiles) continue;
            if (i == 0 || k[j - 1] != t) ranges[t].x = i;
            if (i + 1 == n || k[j + 1] != t) ranges[t].y = i + 1;
        }
    }
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

void launch_tile_ranges(const uint32_t *tile_keys, uint32_t n, const uint32_t *n_dev, uint2 *ranges,
                        uint32_t ntiles, hipStream_t s) {
    launch_fill_u32(reinterpret_cast<uint32_t *>(ranges), 0u, (size_t)ntiles * 2, s);
    if (n == 0) return;
    uint32_t blocks = ((n + 3) / 4 + kBlock - 1) / kBlock;
    if (blocks > 8192) blocks = 8192;
    hipLaunchKernelGGL(k_tile_ranges, dim3(blocks), dim3(kBlock), 0, s, tile_keys, n, n_dev, ranges, ntiles);
}

}  // namespace fgs
