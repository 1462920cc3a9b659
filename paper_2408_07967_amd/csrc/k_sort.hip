// The tile range of a one-tile image (each tile's workload is its run of the
// sorted list, Sec. 2.2) and a fill kernel used to clear counters.
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

}  // namespace

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
