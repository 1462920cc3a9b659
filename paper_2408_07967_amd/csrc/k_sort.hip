// Per-tile lists from the super-tile entries sorted by super-tile (the
// sort stage of Sec. 2.2: pairs ordered by tile, then depth, each tile's
// workload is its run of the list), the range of a one-run list, and a fill
// kernel used to clear counters.
//
// After the stable sort by super-tile, super-tile s holds its entries in
// depth order, each with the 64-bit mask of the Gaussian's hit tiles in s.
// The sorted pair list is the concatenation over tiles t (in id order) of
// the Gaussians hitting t in depth order, so a pair (entry i of s, tile bit
// j) goes to start(t) + #{entries of s before i with bit j set}, with start
// the exclusive scan of the tiles' pair counts.  A super-tile's entries are
// cut into chunks of kListChunk, one wavefront each, so that a dense
// super-tile spreads over many CUs:
//   k_list_chunks  one workgroup: chunk bases of the super-tiles (a scan of
//                  their chunk counts) and the super-tile of every chunk;
//   k_list_count   per chunk: the 64 tiles' hit counts (lane j: bit j), by
//                  transposing each 64 x 64 bit block of masks across lanes;
//   k_list_scan    one workgroup per super-tile: exclusive scan of its
//                  chunks' counts per tile; its tile totals, and its sum
//                  added to its row of super-tiles;
//   k_tile_starts  one workgroup per row of super-tiles (a contiguous band
//                  of tile ids): the earlier rows' sums, then an exclusive
//                  scan of the band's tile totals in tile id order ->
//                  ranges[t] = [start, start + count);
//   k_list_write   per chunk again, tile by tile over its four 64-entry
//                  blocks (one entry per lane): the lanes whose mask has the
//                  tile's bit write their Gaussian at the tile's running
//                  position plus their rank among those lanes (a ballot),
//                  one contiguous store per block.
// Chunks are dealt to the XCDs in eight contiguous ranges, so that a
// super-tile's consecutive chunks, which write the same tiles' lists, share
// an L2.
#include <algorithm>

#include "fgs_internal.hpp"

namespace fgs {
namespace {

constexpr int kWave = 64;

__global__ void k_fill_u32(uint32_t *p, uint32_t value, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = value;
}

// The one range of a one-run list: every element (*n_dev of them, at most n).
__global__ void k_single_range(uint2 *__restrict__ ranges, uint32_t n, const uint32_t *__restrict__ n_dev) {
    if (threadIdx.x == 0) ranges[0] = make_uint2(0u, min(n, *n_dev));
}

// Entries [b, e) of super-tile s (start > end: none; clamped to ecap).
__device__ __forceinline__ uint2 super_entries(const uint2 *sranges, uint32_t s, uint32_t ecap) {
    const uint2 r = sranges[s];
    uint32_t b = r.x, e = r.y;
    if (b > e) b = e = 0;
    e = e < ecap ? e : ecap;
    b = b < e ? b : e;
    return make_uint2(b, e);
}

// Tile of bit j (lane) of super-tile s, or -1 past the image's edge.
__device__ __forceinline__ int64_t lane_tile(uint32_t s, uint32_t stx, int tiles_x, int tiles_y, int lane) {
    const int tx = (int)(s % stx) * kSuper + (lane & (kSuper - 1));
    const int ty = (int)(s / stx) * kSuper + (lane >> kSuperShift);
    return (tx < tiles_x && ty < tiles_y) ? (int64_t)ty * tiles_x + tx : -1;
}

// Transpose of the 64 x 64 bit matrix whose row i is lane i's word: lane j
// gets column j (bit i = bit j of row i).  Six butterfly stages swap the
// off-diagonal s x s blocks of every 2s x 2s block (s = 32 ... 1).
__device__ __forceinline__ uint64_t transpose64(uint64_t x, int lane) {
    const uint64_t kM[6] = {0x00000000ffffffffull, 0x0000ffff0000ffffull, 0x00ff00ff00ff00ffull,
                            0x0f0f0f0f0f0f0f0full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int sh = 32 >> k;
        const uint64_t m = kM[k];
        const uint32_t ylo = (uint32_t)__shfl_xor((int)(uint32_t)x, sh, kWave);
        const uint32_t yhi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), sh, kWave);
        const uint64_t y = (uint64_t)ylo | ((uint64_t)yhi << 32);
        x = (lane & sh) ? ((x & ~m) | ((y >> sh) & m)) : ((x & m) | ((y & m) << sh));
    }
    return x;
}

// The chunks of [0, n) that this wavefront takes: n is cut into eight
// contiguous ranges, one per XCD (workgroups are placed on the eight XCDs in
// turn, and the grid is a multiple of eight workgroups), and the XCD's
// wavefronts take its range's chunks in turn.
struct ChunkWalk {
    uint32_t next, end, stride;
};
__device__ __forceinline__ ChunkWalk chunk_walk(uint32_t n, uint32_t wave_in_block, uint32_t waves_per_block) {
    const uint32_t nb = gridDim.x, x = blockIdx.x % 8u, k = blockIdx.x / 8u;
    const uint32_t nx = (nb - x + 7u) / 8u;  // workgroups on this XCD
    const uint32_t lo = (uint32_t)(((uint64_t)n * x) / 8u), hi = (uint32_t)(((uint64_t)n * (x + 1u)) / 8u);
    ChunkWalk w;
    w.next = lo + k * waves_per_block + wave_in_block;
    w.end = hi;
    w.stride = nx * waves_per_block;
    return w;
}

constexpr int kListBlock = 256;  // chunk kernels: four wavefronts, one chunk each at a time
constexpr int kScanBlock = 1024;

// cbase[s] = first chunk of super-tile s (cbase[nsuper] = the total), and
// csuper[q] = the super-tile of chunk q.
__global__ __launch_bounds__(kScanBlock) void k_list_chunks(const uint2 *__restrict__ sranges, uint32_t nsuper,
                                                            uint32_t ecap, uint32_t *__restrict__ cbase,
                                                            uint32_t *__restrict__ csuper,
                                                            uint32_t *__restrict__ rowsum) {
    __shared__ uint32_t s_w[kScanBlock / kWave];
    const uint32_t tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    const uint32_t run = (nsuper + kScanBlock - 1) / kScanBlock;
    const uint32_t s0 = tid * run < nsuper ? tid * run : nsuper;
    const uint32_t s1 = s0 + run < nsuper ? s0 + run : nsuper;
    uint32_t own = 0;
    for (uint32_t s = s0; s < s1; ++s) {
        const uint2 r = super_entries(sranges, s, ecap);
        own += (r.y - r.x + kListChunk - 1) / kListChunk;
    }
    uint32_t x = own;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, d, kWave);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) s_w[wave] = x;
    __syncthreads();
    uint32_t base = x - own, total = 0;
    for (int q = 0; q < kScanBlock / kWave; ++q) {
        base += q < wave ? s_w[q] : 0u;
        total += s_w[q];
    }
    for (uint32_t s = s0; s < s1; ++s) {
        const uint2 r = super_entries(sranges, s, ecap);
        const uint32_t n = (r.y - r.x + kListChunk - 1) / kListChunk;
        cbase[s] = base;
        rowsum[s] = 0;  // (the rows of super-tiles are at most nsuper)
        for (uint32_t c = 0; c < n; ++c) csuper[base + c] = s;
        base += n;
    }
    if (tid == 0) cbase[nsuper] = total;
}

__global__ __launch_bounds__(kListBlock) void k_list_count(const uint2 *__restrict__ sranges, uint32_t ecap,
                                                           const uint32_t *__restrict__ cbase, uint32_t nsuper,
                                                           const uint32_t *__restrict__ csuper,
                                                           const uint64_t *__restrict__ smask,
                                                           uint32_t *__restrict__ cnt) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const uint32_t n = cbase[nsuper];
    for (ChunkWalk cw = chunk_walk(n, wv, kListBlock / kWave); cw.next < cw.end; cw.next += cw.stride) {
        const uint32_t q = cw.next;
        const uint32_t s = csuper[q];
        const uint2 r = super_entries(sranges, s, ecap);
        const uint32_t b = r.x + (q - cbase[s]) * kListChunk;
        const uint32_t e = b + kListChunk < r.y ? b + kListChunk : r.y;
        uint64_t m[kListChunk / kWave];
#pragma unroll
        for (int k = 0; k < (int)(kListChunk / kWave); ++k) {
            const uint32_t i = b + (uint32_t)(k * kWave + lane);
            m[k] = i < e ? smask[i] : 0ull;
        }
        uint32_t c = 0;
#pragma unroll
        for (int k = 0; k < (int)(kListChunk / kWave); ++k) c += (uint32_t)__popcll(transpose64(m[k], lane));
        cnt[(size_t)q * kWave + lane] = c;
    }
}

// One workgroup per super-tile: its chunks' counts become exclusive
// prefixes per tile (in place), and its tile totals go to ranges[t].x.
__global__ __launch_bounds__(kScanBlock) void k_list_scan(const uint32_t *__restrict__ cbase, uint32_t stx,
                                                          int tiles_x, int tiles_y, uint32_t *__restrict__ cnt,
                                                          uint2 *__restrict__ ranges, uint32_t *__restrict__ rowsum) {
    constexpr int kWaves = kScanBlock / kWave;
    __shared__ uint32_t s_sum[kWaves][kWave];
    const uint32_t s = blockIdx.x;
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t w = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const uint32_t c0 = cbase[s], n = cbase[s + 1] - c0;
    const uint32_t per = (n + kWaves - 1) / kWaves;
    const uint32_t r0 = c0 + (w * per < n ? w * per : n), r1 = c0 + ((w + 1) * per < n ? (w + 1) * per : n);
    uint32_t sum = 0;
    for (uint32_t q = r0; q < r1; ++q) sum += cnt[(size_t)q * kWave + lane];
    s_sum[w][lane] = sum;
    __syncthreads();
    uint32_t run = 0, tot = 0;
#pragma unroll
    for (uint32_t k = 0; k < (uint32_t)kWaves; ++k) {
        const uint32_t v = s_sum[k][lane];
        run += k < w ? v : 0u;
        tot += v;
    }
    for (uint32_t q = r0; q < r1; ++q) {
        const uint32_t v = cnt[(size_t)q * kWave + lane];
        cnt[(size_t)q * kWave + lane] = run;
        run += v;
    }
    if (w == 0) {
        const int64_t t = lane_tile(s, stx, tiles_x, tiles_y, lane);
        if (t >= 0) ranges[t] = make_uint2(tot, 0u);
        uint32_t st = tot;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) st += (uint32_t)__shfl_xor((int)st, d, kWave);
        if (lane == 0 && st) atomicAdd(&rowsum[s / stx], st);
    }
}

// Workgroup b: the tiles of super-tile row b (tile rows kSuper b ...
// kSuper b + kSuper - 1, a contiguous range of tile ids).  Its first start is
// the sum of the earlier rows; its tiles are scanned kScanBlock at a time.
__global__ __launch_bounds__(kScanBlock) void k_tile_starts(uint2 *__restrict__ ranges, int tiles_x, uint32_t ntiles,
                                                            const uint32_t *__restrict__ rowsum, uint32_t ncap) {
    __shared__ uint32_t s_w[kScanBlock / kWave];
    __shared__ uint32_t s_base;
    const uint32_t tid = threadIdx.x, b = blockIdx.x;
    const int lane = tid & (kWave - 1), wave = tid / kWave;
    if (wave == 0) {
        uint32_t x = 0;
        for (uint32_t q = (uint32_t)lane; q < b; q += kWave) x += rowsum[q];
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) x += (uint32_t)__shfl_xor((int)x, d, kWave);
        if (lane == 0) s_base = x;
    }
    __syncthreads();
    uint32_t start = s_base;
    const uint32_t band = (uint32_t)kSuper * (uint32_t)tiles_x;
    const uint32_t t_lo = b * band, t_hi = t_lo + band < ntiles ? t_lo + band : ntiles;
    for (uint32_t r0 = t_lo; r0 < t_hi; r0 += kScanBlock) {
        const uint32_t t = r0 + tid;
        const uint32_t c = t < t_hi ? ranges[t].x : 0u;
        uint32_t x = c;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint32_t y = (uint32_t)__shfl_up((int)x, d, kWave);
            if (lane >= d) x += y;
        }
        if (lane == kWave - 1) s_w[wave] = x;
        __syncthreads();
        uint32_t before = 0, all = 0;
#pragma unroll
        for (int q = 0; q < kScanBlock / kWave; ++q) {
            const uint32_t v = s_w[q];
            before += q < wave ? v : 0u;
            all += v;
        }
        __syncthreads();
        const uint32_t a0 = start + before + x - c;
        if (t < t_hi) {
            const uint32_t a = a0 < ncap ? a0 : ncap;
            const uint32_t e = a0 + c < ncap ? a0 + c : ncap;
            ranges[t] = make_uint2(a, e);
        }
        start += all;
    }
}

// kBuf: values are stored through a buffer resource of ncap words, whose
// range check drops a store past the end (byte offsets: ncap < 2^29).
template <bool kBuf>
__global__ __launch_bounds__(kListBlock) void k_list_write(const uint2 *__restrict__ sranges, uint32_t ecap,
                                                           const uint32_t *__restrict__ cbase, uint32_t nsuper,
                                                           const uint32_t *__restrict__ csuper, uint32_t stx,
                                                           int tiles_x, int tiles_y,
                                                           const uint32_t *__restrict__ gidx,
                                                           const uint64_t *__restrict__ smask,
                                                           const uint32_t *__restrict__ pre,
                                                           const uint2 *__restrict__ ranges,
                                                           uint32_t *__restrict__ values, uint32_t ncap) {
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t wv = (uint32_t)__builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
    const uint32_t n = cbase[nsuper];
    const __amdgpu_buffer_rsrc_t vrs =
        __builtin_amdgcn_make_buffer_rsrc(values, (short)0, kBuf ? (int)(ncap * 4u) : 0, 0x00020000);
    for (ChunkWalk cw = chunk_walk(n, wv, kListBlock / kWave); cw.next < cw.end; cw.next += cw.stride) {
        const uint32_t q = cw.next;
        const uint32_t s = csuper[q];
        const uint2 r = super_entries(sranges, s, ecap);
        const uint32_t b = r.x + (q - cbase[s]) * kListChunk;
        const uint32_t e = b + kListChunk < r.y ? b + kListChunk : r.y;
        uint64_t m[kListChunk / kWave];
        uint32_t g[kListChunk / kWave];
#pragma unroll
        for (int k = 0; k < (int)(kListChunk / kWave); ++k) {
            const uint32_t i = b + (uint32_t)(k * kWave + lane);
            m[k] = i < e ? smask[i] : 0ull;
            g[k] = i < e ? gidx[i] : 0u;
        }
        // lane j: the first output position of tile j (bit j) of this super-tile
        const int64_t t = lane_tile(s, stx, tiles_x, tiles_y, lane);
        const uint32_t first = t >= 0 ? ranges[t].x + pre[(size_t)q * kWave + lane] : 0u;
        // tile by tile: the chunk's four 64-entry blocks in order, the
        // running position kept as a wavefront-uniform value
#pragma unroll
        for (int j = 0; j < kWave; ++j) {
            uint32_t base = (uint32_t)__builtin_amdgcn_readlane((int)first, j);
#pragma unroll
            for (int k = 0; k < (int)(kListChunk / kWave); ++k) {
                const uint32_t w = j < 32 ? (uint32_t)m[k] : (uint32_t)(m[k] >> 32);
                const bool hit = ((w >> (j & 31)) & 1u) != 0u;
                const uint64_t bal = __ballot(hit);
                if (bal) {  // uniform
                    const uint32_t pos =
                        base + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
                    if (hit) {
                        if constexpr (kBuf)
                            __builtin_amdgcn_raw_buffer_store_b32(g[k], vrs, pos * 4u, 0, 0);
                        else if (pos < ncap)  // never leave the values
                            values[pos] = g[k];
                    }
                    base += (uint32_t)__popcll(bal);
                }
            }
        }
    }
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

void launch_tile_lists(int W, int H, const uint2 *sranges, const uint32_t *gidx, const uint64_t *smask,
                       uint32_t ecap, uint32_t *scratch, uint2 *ranges, uint32_t *values, uint32_t ncap,
                       hipStream_t s) {
    const int tiles_x = (W + kTile - 1) / kTile, tiles_y = (H + kTile - 1) / kTile;
    const uint32_t stx = (uint32_t)((tiles_x + kSuper - 1) >> kSuperShift);
    const uint32_t sty = (uint32_t)((tiles_y + kSuper - 1) >> kSuperShift);
    const uint32_t nsuper = stx * sty, ntiles = (uint32_t)tiles_x * (uint32_t)tiles_y;
    if (nsuper == 0) return;
    // scratch: chunk bases, chunk super-tiles, per-chunk counts (see list_scratch_words)
    const size_t g = list_chunks_max(ecap, nsuper);
    uint32_t *cbase = scratch;
    uint32_t *rowsum = cbase + nsuper + 1;
    uint32_t *csuper = cbase + (2 * nsuper + 1 + 63) / 64 * 64;
    uint32_t *cnt = csuper + (g + 63) / 64 * 64;
    // chunk grids: four chunks per workgroup, at most a few resident rounds,
    // a multiple of eight workgroups (every XCD's range has workgroups)
    const unsigned chunk_blocks = (unsigned)((std::min<size_t>((g + 3) / 4, 8192) + 7) / 8 * 8);
    hipLaunchKernelGGL(k_list_chunks, dim3(1), dim3(kScanBlock), 0, s, sranges, nsuper, ecap, cbase, csuper, rowsum);
    hipLaunchKernelGGL(k_list_count, dim3(chunk_blocks), dim3(kListBlock), 0, s, sranges, ecap, cbase, nsuper, csuper,
                       smask, cnt);
    hipLaunchKernelGGL(k_list_scan, dim3(nsuper), dim3(kScanBlock), 0, s, cbase, stx, tiles_x, tiles_y, cnt, ranges,
                       rowsum);
    hipLaunchKernelGGL(k_tile_starts, dim3(sty), dim3(kScanBlock), 0, s, ranges, tiles_x, ntiles, rowsum, ncap);
    if (ncap < (1u << 29))
        hipLaunchKernelGGL(k_list_write<true>, dim3(chunk_blocks), dim3(kListBlock), 0, s, sranges, ecap, cbase, nsuper,
                           csuper, stx, tiles_x, tiles_y, gidx, smask, cnt, ranges, values, ncap);
    else
        hipLaunchKernelGGL(k_list_write<false>, dim3(chunk_blocks), dim3(kListBlock), 0, s, sranges, ecap, cbase,
                           nsuper, csuper, stx, tiles_x, tiles_y, gidx, smask, cnt, ranges, values, ncap);
}

}  // namespace fgs
