// Stable LSD radix sort pass and exclusive scan without any wait between
// workgroups (the sort stage of Sec. 2.2; the scan of Alg. 2's offsets).
//
// A pass over n keys uses a fixed grid of kSortBlocks workgroups; workgroup b
// owns a contiguous range of 4096-key tiles (the range is derived on the
// device from n, so n may be a device-side count):
//   upsweep    - digit histogram of each workgroup's range   -> hist[b][d],
//                and added (device-scope atomics) into the row
//                of its group of kSortGroup workgroups       -> gsum[w][d]
//   downsweep  - each workgroup derives the global offset of its first key
//                of every digit (digit totals, earlier groups, earlier
//                workgroups of its own group), then walks its tiles in order:
//                stable ballot ranking per wave64, LDS staging in digit
//                order, coalesced scatter, running per-digit offsets.
// Keys are read twice (upsweep and downsweep); in exchange no workgroup ever
// waits for another one, which on gfx950 is cheaper than a decoupled
// look-back across eight XCDs.  (Handing the histograms over inside the
// upsweep, by a release fence and an arrival counter, was measured slower:
// a device-scope release on gfx950 writes back the XCD's L2.)
#include "fgs_internal.hpp"

namespace fgs {
namespace {

constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;

__device__ __forceinline__ uint32_t count_of(uint32_t n_host, const uint32_t *n_dev) {
    if (!n_dev) return n_host;
    const uint32_t nd = *n_dev;
    return nd < n_host ? nd : n_host;
}

// key range [lo, hi) of workgroup b: whole tiles of `granule` keys (4096 for
// the sort passes) split evenly
__device__ __forceinline__ void block_range(uint32_t n, uint32_t b, uint32_t nb, uint32_t *lo, uint32_t *hi,
                                            uint32_t granule = kSortTile) {
    const uint32_t tiles = (n + granule - 1) / granule;
    const uint32_t t0 = (uint32_t)(((uint64_t)tiles * b) / nb);
    const uint32_t t1 = (uint32_t)(((uint64_t)tiles * (b + 1)) / nb);
    *lo = t0 * granule;
    const uint32_t h = t1 * granule;
    *hi = h < n ? h : n;
    if (*lo > *hi) *lo = *hi;
}

// Exclusive scan of one value per thread over a 256-thread workgroup.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_tmp, uint32_t *total) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, d, kWave);
        if (lane >= d) x += y;
    }
    if (lane == kWave - 1) s_tmp[wave] = x;
    __syncthreads();
    uint32_t wpre = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const uint32_t t = s_tmp[w];
        wpre += (w < wave) ? t : 0u;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return wpre + x - v;
}

// kDB: digit bits the pass may take (8, or 9 for a one-pass sort of up to
// 512 keys); each thread owns kDigitsPerThread consecutive digits.
template <int kDB>
constexpr int digits_per_thread() {
    return (1 << kDB) / kBlock;
}

template <bool kFilter, class KeyT, int kDB = kRadixBits>
__global__ __launch_bounds__(kBlock) void k_radix_upsweep(const KeyT *__restrict__ keys, uint32_t n_host,
                                                          const uint32_t *n_dev, int shift, int bits,
                                                          uint32_t *__restrict__ hist, uint32_t *gsum) {
    constexpr int kR = 1 << kDB, kP = digits_per_thread<kDB>();
    static_assert(kP >= 1 && kR <= kRadixMax, "digit width");
    __shared__ uint32_t s_h[kWaves][kR];
    const int tid = threadIdx.x, wave = tid / kWave;
    for (int i = tid; i < kWaves * kR; i += kBlock) (&s_h[0][0])[i] = 0;
    __syncthreads();
    const uint32_t n = count_of(n_host, n_dev);
    uint32_t lo, hi;
    block_range(n, blockIdx.x, gridDim.x, &lo, &hi);
    const uint32_t dmask = (1u << bits) - 1u;
    // Each thread counts kSortItems consecutive keys of a tile (the histogram
    // ignores their order), read with 16-byte loads where the tile is whole:
    // all loads in flight before any use.
    constexpr int kPerVec = 16 / (int)sizeof(KeyT);
    static_assert(kSortItems % kPerVec == 0, "whole 16-byte groups per thread");
    for (uint32_t c0 = lo; c0 < hi; c0 += kSortTile) {
        const uint32_t b = c0 + (uint32_t)tid * kSortItems;
        uint32_t k[kSortItems];
        if (b + kSortItems <= hi) {
            uint4 q[kSortItems / kPerVec];
#pragma unroll
            for (int j = 0; j < kSortItems / kPerVec; ++j) q[j] = reinterpret_cast<const uint4 *>(keys + b)[j];
#pragma unroll
            for (int j = 0; j < kSortItems / kPerVec; ++j) {
                const uint32_t w[4] = {q[j].x, q[j].y, q[j].z, q[j].w};
#pragma unroll
                for (int e = 0; e < kPerVec; ++e)
                    k[j * kPerVec + e] = sizeof(KeyT) == 2 ? (w[e / 2] >> (16 * (e % 2))) & 0xffffu : w[e];
            }
        } else {
#pragma unroll
            for (int i = 0; i < kSortItems; ++i) k[i] = b + i < hi ? (uint32_t)keys[b + i] : kInvalidKey;
        }
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            if (b + i < hi && (!kFilter || k[i] != kInvalidKey)) atomicAdd(&s_h[wave][(k[i] >> shift) & dmask], 1u);
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kP; ++q) {
        const int d = tid * kP + q;
        const uint32_t h = s_h[0][d] + s_h[1][d] + s_h[2][d] + s_h[3][d];
        hist[(size_t)blockIdx.x * kR + d] = h;
        if (h) atomicAdd(&gsum[(size_t)(blockIdx.x / kSortGroup) * kR + d], h);
    }
}

static_assert(kSortBlocks % kSortGroup == 0, "whole groups of workgroups");

// (LDS holds four workgroups per CU, so registers are capped at what four
// waves per SIMD allow; a 9-bit pass, whose digit bookkeeping needs more,
// at what three allow.)
// kPayload: the values are the input positions while ranking (as with
// kIdentityVals), and each element's payload (vals_in, mask_in at that
// position, inside the workgroup's tile) is read when it is stored.
template <bool kIdentityVals, bool kFilter, bool kWriteKeys, class KeyT, bool kPayload = false, int kDB = kRadixBits>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(kDB > kRadixBits ? 3 : 4))) void k_radix_downsweep(const KeyT *__restrict__ keys_in,
                                                            const uint32_t *__restrict__ vals_in,
                                                            KeyT *__restrict__ keys_out,
                                                            uint32_t *__restrict__ vals_out, uint32_t n_host,
                                                            const uint32_t *n_dev, int shift, int bits,
                                                            const uint32_t *__restrict__ hist,
                                                            const uint32_t *__restrict__ gsum,
                                                            uint32_t *__restrict__ gsum_next,
                                                            uint32_t *__restrict__ run_end, uint32_t nruns,
                                                            const uint64_t *__restrict__ mask_in,
                                                            uint64_t *__restrict__ mask_out,
                                                            uint32_t *__restrict__ digit_run) {
    static_assert(!kPayload || kIdentityVals, "a payload is ranked by position");
    constexpr int kR = 1 << kDB, kP = digits_per_thread<kDB>();
    static_assert(kP >= 1 && kR <= kRadixMax, "digit width");
    // (per-wave and per-tile digit counts are at most kSortTile: 16 bits)
    __shared__ KeyT s_keys[kSortTile];
    __shared__ uint32_t s_vals[kSortTile];
    __shared__ uint16_t s_wave[kWaves][kR];
    __shared__ uint32_t s_off[kR];
    __shared__ uint16_t s_excl[kR + 1];
    __shared__ uint32_t s_gbase[kR];  // output position of tile element j of digit d: s_gbase[d] + j
    __shared__ uint32_t s_tmp[kWaves];
    __shared__ uint32_t s_nv;

    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    // the next pass's group sums start at zero
    if (gsum_next)
        for (uint32_t i = blockIdx.x * kBlock + tid; i < (uint32_t)kGsumWords; i += gridDim.x * kBlock) gsum_next[i] = 0;
    const uint32_t n = count_of(n_host, n_dev);
    const uint32_t b = blockIdx.x, nb = gridDim.x;
    uint32_t lo, hi;
    block_range(n, b, nb, &lo, &hi);

    // global offset of this workgroup's first key of each of the thread's
    // digits: every group sum and every earlier histogram row of the group is
    // loaded at once per digit (a fixed, unrolled trip count keeps all the
    // loads in flight together)
    {
        constexpr uint32_t kGroups = kSortGroups;
        const uint32_t mygroup = b / kSortGroup;
        uint32_t dtot[kP], dbefore[kP], own = 0;
#pragma unroll
        for (int q = 0; q < kP; ++q) dtot[q] = dbefore[q] = 0;
        // the group sums of the thread's digits, then the earlier rows of its
        // group (each phase's loads issued together)
        {
            uint32_t gv[kGroups][kP];
#pragma unroll
            for (uint32_t w = 0; w < kGroups; ++w)
#pragma unroll
                for (int q = 0; q < kP; ++q) gv[w][q] = gsum[(size_t)w * kR + tid * kP + q];
#pragma unroll
            for (uint32_t w = 0; w < kGroups; ++w)
#pragma unroll
                for (int q = 0; q < kP; ++q) {
                    dtot[q] += gv[w][q];
                    dbefore[q] += (w < mygroup) ? gv[w][q] : 0u;
                }
        }
        {
            uint32_t hv[kSortGroup][kP];
#pragma unroll
            for (uint32_t r = 0; r < (uint32_t)kSortGroup; ++r) {
                const uint32_t row = mygroup * kSortGroup + r;
#pragma unroll
                for (int q = 0; q < kP; ++q) hv[r][q] = row < b ? hist[(size_t)row * kR + tid * kP + q] : 0u;
            }
#pragma unroll
            for (uint32_t r = 0; r < (uint32_t)kSortGroup; ++r)
#pragma unroll
                for (int q = 0; q < kP; ++q) dbefore[q] += hv[r][q];
        }
#pragma unroll
        for (int q = 0; q < kP; ++q) own += dtot[q];
        uint32_t all = 0;
        uint32_t dbase = block_exclusive_scan(own, s_tmp, &all);
#pragma unroll
        for (int q = 0; q < kP; ++q) {
            const uint32_t d = (uint32_t)(tid * kP + q);
            s_off[d] = dbase + dbefore[q];
            // a pass by the whole key: digit d's run is [its offset, + its total)
            if (digit_run && b == 0 && d < nruns) {
                digit_run[2 * (size_t)d] = dbase;
                digit_run[2 * (size_t)d + 1] = dbase + dtot[q];
            }
            dbase += dtot[q];
        }
    }
    if (lo >= hi) return;  // uniform: no tile for this workgroup

    const uint32_t dmask = (1u << bits) - 1u;
    // A tile's loads are all issued before any use, and the next tile's are
    // issued as soon as the current one sits in LDS, so that they are in
    // flight while the current tile is written out.
    // (identity values are the input positions, computed where they are
    // staged rather than held in registers)
    uint32_t key[kSortItems], val[kIdentityVals ? 1 : kSortItems], rank[kSortItems];
    auto load_tile = [&](uint32_t t) {
        const uint32_t base = t + (uint32_t)wave * (kSortItems * kWave);
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            const uint32_t idx = base + (uint32_t)(i * kWave + lane);
            const bool in = idx < hi;
            key[i] = in ? (uint32_t)keys_in[idx] : kInvalidKey;
            if constexpr (!kIdentityVals) val[i] = in ? vals_in[idx] : 0u;
        }
    };
    load_tile(lo);
    for (uint32_t t0 = lo; t0 < hi; t0 += kSortTile) {
        for (int i = tid; i < kWaves * kR; i += kBlock) (&s_wave[0][0])[i] = 0;
        __syncthreads();
        const uint32_t base = t0 + (uint32_t)wave * (kSortItems * kWave);
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            const uint32_t idx = base + (uint32_t)(i * kWave + lane);
            const bool in = idx < hi;
            const uint32_t k = key[i];
            const bool ok = in && (!kFilter || k != kInvalidKey);
            const uint32_t d = (k >> shift) & dmask;
            // lanes of this step with the same digit (stable rank = lower
            // lanes): a lane differs from this one where some digit bit
            // disagrees, i.e. where ballot(bit) xor (own bit, widened) is
            // set.  All kDB bits are matched (a narrower digit has zero high
            // bits in every lane).  Per bit: one bitfield extract, one
            // compare and one three-input logic op per half mask
            // (bitop3 table 0xf6 = src0 | (src1 ^ src2)).
            uint32_t diff_lo = 0, diff_hi = 0;
#pragma unroll
            for (int bb = 0; bb < kDB; ++bb) {
                // bit bb of d widened to 0 or ~0 by one signed bitfield extract
                // (written out: the compiler otherwise splits it into two shifts)
                uint32_t t;
                asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(t) : "v"(d), "i"(bb));
                const uint64_t m = __ballot(t != 0u);
                diff_lo = __builtin_amdgcn_bitop3_b32(diff_lo, (uint32_t)m, t, 0xf6);
                diff_hi = __builtin_amdgcn_bitop3_b32(diff_hi, (uint32_t)(m >> 32), t, 0xf6);
            }
            const uint64_t okm = __ballot(ok);
            const uint32_t peers_lo = (uint32_t)okm & ~diff_lo, peers_hi = (uint32_t)(okm >> 32) & ~diff_hi;
            // set bits of peers below this lane
            const uint32_t before = __builtin_amdgcn_mbcnt_hi(peers_hi, __builtin_amdgcn_mbcnt_lo(peers_lo, 0u));
            const uint32_t cnt = (uint32_t)__popc(peers_lo) + (uint32_t)__popc(peers_hi);
            uint32_t prev = 0;
            if (ok) prev = s_wave[wave][d];
            if (ok && before == 0) s_wave[wave][d] = prev + cnt;
            rank[i] = ok ? prev + before : 0xffffffffu;
        }
        __syncthreads();
        // thread tid owns digits tid kP ... tid kP + kP - 1: per-wave counts
        // -> exclusive over waves
        uint32_t dsum[kP], own = 0;
#pragma unroll
        for (int q = 0; q < kP; ++q) {
            const int d = tid * kP + q;
            const uint32_t c0 = s_wave[0][d], c1 = s_wave[1][d], c2 = s_wave[2][d], c3 = s_wave[3][d];
            s_wave[0][d] = 0;
            s_wave[1][d] = c0;
            s_wave[2][d] = c0 + c1;
            s_wave[3][d] = c0 + c1 + c2;
            dsum[q] = c0 + c1 + c2 + c3;
            own += dsum[q];
        }
        uint32_t nvalid = 0;
        uint32_t excl = block_exclusive_scan(own, s_tmp, &nvalid);
#pragma unroll
        for (int q = 0; q < kP; ++q) {
            const int d = tid * kP + q;
            s_excl[d] = (uint16_t)excl;
            s_gbase[d] = s_off[d] - excl;
            excl += dsum[q];
        }
        if (tid == 0) {
            s_nv = nvalid;
            s_excl[kR] = (uint16_t)nvalid;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kSortItems; ++i) {
            if (rank[i] != 0xffffffffu) {
                const uint32_t d = (key[i] >> shift) & dmask;
                const uint32_t lp = s_excl[d] + s_wave[wave][d] + rank[i];
                s_keys[lp] = (KeyT)key[i];
                if constexpr (kIdentityVals)
                    s_vals[lp] = t0 + (uint32_t)wave * (kSortItems * kWave) + (uint32_t)(i * kWave + lane);
                else
                    s_vals[lp] = val[i];
            }
        }
        if (t0 + kSortTile < hi) load_tile(t0 + kSortTile);
        __syncthreads();
        const uint32_t nv = s_nv;
        for (uint32_t j = tid; j < nv; j += kBlock) {
            const uint32_t k = s_keys[j];
            const uint32_t d = (k >> shift) & dmask;
            const uint32_t gpos = s_gbase[d] + j;
            if (gpos < n) {  // never leave the output (n bounds the scattered count)
                if (kWriteKeys) keys_out[gpos] = (KeyT)k;
                if constexpr (kPayload) {
                    const uint32_t src = s_vals[j];  // < hi: an element of this tile
                    vals_out[gpos] = vals_in[src];
                    mask_out[gpos] = mask_in[src];
                } else {
                    vals_out[gpos] = s_vals[j];
                }
                // last pass of a sort by the whole key: the keys of one
                // digit run of this tile are in key order, so the first and
                // last element of each key's stretch may start and end its run
                if (run_end && k < nruns) {
                    if (j == 0 || s_keys[j - 1] != k) atomicMin(&run_end[2 * (size_t)k], gpos);
                    if (j + 1 == nv || s_keys[j + 1] != k) atomicMax(&run_end[2 * (size_t)k + 1], gpos + 1);
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kP; ++q) s_off[tid * kP + q] += dsum[q];
    }
}

// ---- exclusive scan of per-Gaussian tile counts in depth order -------------

// Workgroup ranges of the scan are whole 1024-entry tiles: the few million
// visible Gaussians keep every one of the kSortBlocks workgroups busy.
constexpr uint32_t kScanGranule = 1024;

// cs[r] = count of order[r] (from the one-byte copy, or the super-tile span
// of a chunked rectangle's record); sums[b] = sum over the workgroup's range
__global__ __launch_bounds__(kBlock) void k_scan_upsweep(const uint32_t *__restrict__ order,
                                                         const uint8_t *__restrict__ count8,
                                                         const uint4 *__restrict__ erec, uint32_t n_host,
                                                         const uint32_t *n_dev, uint32_t *__restrict__ cs,
                                                         uint32_t *__restrict__ sums) {
    __shared__ uint32_t s_tmp[kWaves];
    const uint32_t n = count_of(n_host, n_dev);
    uint32_t lo, hi;
    block_range(n, blockIdx.x, gridDim.x, &lo, &hi, kScanGranule);
    uint32_t s = 0;
    for (uint32_t c0 = lo; c0 < hi; c0 += 8 * kBlock) {
        uint32_t g[8], c[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t i = c0 + (uint32_t)(k * kBlock) + threadIdx.x;
            g[k] = i < hi ? order[i] : 0u;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t i = c0 + (uint32_t)(k * kBlock) + threadIdx.x;
            c[k] = i < hi ? count8[g[k]] : 0u;
        }
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (c[k] == kCount8Big) {  // a chunked rectangle (rare)
                const uint4 r = erec[g[k]];
                c[k] = super_span((int)(r.x & 0xffffu), (int)(r.x >> 16), (int)(r.y & 0xffffu), (int)(r.y >> 16));
            }
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint32_t i = c0 + (uint32_t)(k * kBlock) + threadIdx.x;
            if (i < hi) cs[i] = c[k];
            s += c[k];
        }
    }
    uint32_t tot = 0;
    (void)block_exclusive_scan(s, s_tmp, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// offsets[r] = exclusive prefix of cs; offsets[n] and *total = total.  Each
// workgroup sums the kSortBlocks workgroup sums itself (4 KB from L2) for its
// base and the total.
__global__ __launch_bounds__(kBlock) void k_scan_downsweep(const uint32_t *__restrict__ cs, uint32_t n_host,
                                                           const uint32_t *n_dev, const uint32_t *__restrict__ sums,
                                                           uint32_t *__restrict__ offsets, uint32_t *total) {
    __shared__ uint32_t s_tmp[kWaves];
    const uint32_t n = count_of(n_host, n_dev);
    uint32_t lo, hi;
    block_range(n, blockIdx.x, gridDim.x, &lo, &hi, kScanGranule);
    uint32_t run = 0;
    {
        constexpr int kPer = kSortBlocks / kBlock;
        static_assert(kSortBlocks % kBlock == 0, "whole rows of workgroup sums per thread");
        uint32_t pre = 0, all = 0;
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const uint32_t j = (uint32_t)(i * kBlock) + threadIdx.x;
            const uint32_t v = j < gridDim.x ? sums[j] : 0u;
            pre += j < blockIdx.x ? v : 0u;
            all += v;
        }
        uint32_t tot_pre = 0, tot_all = 0;
        (void)block_exclusive_scan(pre, s_tmp, &tot_pre);
        (void)block_exclusive_scan(all, s_tmp, &tot_all);
        run = tot_pre;
        if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total = tot_all;
    }
    // one 4096-entry tile per step: every thread scans its own 16
    // consecutive entries (four 16-byte loads and stores where the tile is
    // whole), then the threads' totals are scanned across the workgroup
    constexpr int kRun = kSortTile / kBlock;
    static_assert(kRun % 4 == 0, "whole 16-byte groups per thread");
    for (uint32_t c0 = lo; c0 < hi; c0 += kSortTile) {
        const uint32_t b = c0 + threadIdx.x * (uint32_t)kRun;
        uint32_t v[kRun];
        const bool whole = b + kRun <= hi;
        if (whole) {
#pragma unroll
            for (int q = 0; q < kRun / 4; ++q) {
                const uint4 x = *reinterpret_cast<const uint4 *>(cs + b + 4 * q);
                v[4 * q] = x.x;
                v[4 * q + 1] = x.y;
                v[4 * q + 2] = x.z;
                v[4 * q + 3] = x.w;
            }
        } else {
#pragma unroll
            for (int k = 0; k < kRun; ++k) v[k] = b + k < hi ? cs[b + k] : 0u;
        }
        uint32_t own = 0;
#pragma unroll
        for (int k = 0; k < kRun; ++k) {
            const uint32_t x = v[k];
            v[k] = own;  // exclusive within the thread's run
            own += x;
        }
        uint32_t tot = 0;
        const uint32_t ex = run + block_exclusive_scan(own, s_tmp, &tot);
        if (whole) {
#pragma unroll
            for (int q = 0; q < kRun / 4; ++q)
                *reinterpret_cast<uint4 *>(offsets + b + 4 * q) =
                    make_uint4(ex + v[4 * q], ex + v[4 * q + 1], ex + v[4 * q + 2], ex + v[4 * q + 3]);
        } else {
#pragma unroll
            for (int k = 0; k < kRun; ++k)
                if (b + k < hi) offsets[b + k] = ex + v[k];
        }
        run += tot;
    }
    if (hi == n && lo < hi && threadIdx.x == 0) offsets[n] = run;
}

// ---- depth ties of a prepared scene's frame -------------------------------
// The depth sort is stable over list positions, whose order follows the
// precompute's spatial order; the method orders equal depths by Gaussian
// index.  Each wavefront owns kTieOwn consecutive sorted positions and also
// reads the kTieLook after them.  A run of equal keys that begins among its
// own positions and ends within that span is re-ordered in place: every
// member reads its list position's Gaussian index, counts the members with
// a smaller index (through LDS) and stores its list position at that rank.
// The wavefront whose positions hold a run's start is the only one that
// touches the run.  A run that reaches the end of the span (at least
// kTieLook + 1 long) is listed for k_depth_long_ties.  Keys and list
// positions are read once, coalesced; only tied positions gather.
constexpr int kTieOwn = 256, kTieLook = 32, kTieSpan = kTieOwn + kTieLook;
static_assert(kTieLook <= kWave && kTieOwn % kWave == 0, "span of whole wavefront loads");
static_assert(kTieLook <= kShortTieRun, "runs listed as long are longer than kShortTieRun");
__global__ __launch_bounds__(kBlock) void k_depth_ties(const uint32_t *__restrict__ keys, uint32_t *vals,
                                                       const uint32_t *__restrict__ gmap, uint32_t n_host,
                                                       const uint32_t *n_dev, uint32_t *__restrict__ long_list,
                                                       FrameCounters *fc) {
    constexpr int kSub = (kTieSpan + kWave - 1) / kWave;
    __shared__ uint32_t s_key[kWaves][kTieSpan], s_idx[kWaves][kTieSpan];
    const uint32_t n = count_of(n_host, n_dev);
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const uint32_t base = (blockIdx.x * kWaves + (uint32_t)wv) * (uint32_t)kTieOwn;
    if (base >= n) return;  // uniform over the wavefront
    uint32_t *const sk = s_key[wv], *const si = s_idx[wv];
    // sorted keys are valid depth bits, never kInvalidKey
    uint32_t k[kSub], v[kSub];
#pragma unroll
    for (int w = 0; w < kSub; ++w) {
        const int q = w * kWave + lane;
        const bool in = q < kTieSpan && base + (uint32_t)q < n;
        k[w] = in ? keys[base + q] : kInvalidKey;
        v[w] = in ? vals[base + q] : 0u;
        if (q < kTieSpan) sk[q] = k[w];
    }
    const uint32_t kbefore = base > 0 ? keys[base - 1] : kInvalidKey;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    int S[kSub], E[kSub];
    bool here[kSub];
#pragma unroll
    for (int w = 0; w < kSub; ++w) {
        const int q = w * kWave + lane;
        here[w] = false;
        S[w] = E[w] = q;
        if (q >= kTieSpan || k[w] == kInvalidKey) continue;
        const uint32_t kq = k[w];
        const bool prev_eq = q > 0 ? sk[q - 1] == kq : kbefore == kq;
        const bool next_eq = q + 1 < kTieSpan ? sk[q + 1] == kq : true;  // unknown past the span
        if (!prev_eq && !next_eq) continue;
        int s0 = q;
        while (s0 > 0 && sk[s0 - 1] == kq) --s0;
        if (s0 == 0 && kbefore == kq) continue;  // begun before these positions
        if (s0 >= kTieOwn) continue;              // the next wavefront's run
        int e0 = q + 1;
        while (e0 < kTieSpan && sk[e0] == kq) ++e0;
        if (e0 == kTieSpan) {
            // reaches the end of the span: a long run, ordered elsewhere
            if (q == s0) long_list[atomicAdd(&fc->nlong, 1u)] = base + (uint32_t)s0;
            continue;
        }
        S[w] = s0;
        E[w] = e0;
        here[w] = true;
        si[q] = gmap[v[w]];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int w = 0; w < kSub; ++w) {
        if (!here[w]) continue;
        const int q = w * kWave + lane;
        const uint32_t o = si[q];
        uint32_t rank = 0;
        for (int j = S[w]; j < E[w]; ++j) rank += si[j] < o ? 1u : 0u;
        vals[base + (uint32_t)S[w] + rank] = v[w];
    }
}

// Position of the first of the n ascending Gaussian indices gmap[v[.]] that
// is not below key.
__device__ __forceinline__ uint32_t tie_lower_bound(const uint32_t *v, uint32_t n, const uint32_t *gmap,
                                                    uint32_t key) {
    uint32_t lo = 0, hi = n;
    while (lo < hi) {
        const uint32_t m = (lo + hi) >> 1;
        if (gmap[v[m]] < key)
            lo = m + 1;
        else
            hi = m;
    }
    return lo;
}

// One workgroup per listed run of more than kShortTieRun equal keys: its
// length, then a sort of its list positions by Gaussian index (distinct
// keys): chunks of kTieChunk by a bitonic sort in LDS, then merge passes in
// which every element finds its place in the merged pair of sorted pieces by
// a binary search in the other piece.  The values ping-pong between vals and
// tmp_v (the run's own region of each), so runs never touch each other's data.
constexpr uint32_t kTieChunk = 1024;
__global__ __launch_bounds__(kBlock) void k_depth_long_ties(const uint32_t *__restrict__ keys, uint32_t *vals,
                                                            const uint32_t *__restrict__ gmap, uint32_t n_host,
                                                            const uint32_t *n_dev,
                                                            const uint32_t *__restrict__ long_list,
                                                            const FrameCounters *fc, uint32_t *tmp_v) {
    __shared__ uint32_t s_k[kTieChunk], s_v[kTieChunk];
    __shared__ uint32_t s_len;
    const uint32_t n = count_of(n_host, n_dev);
    const uint32_t nl = fc->nlong;
    const uint32_t tid = threadIdx.x;
    for (uint32_t r = blockIdx.x; r < nl; r += gridDim.x) {
        const uint32_t s0 = long_list[r];
        const uint32_t k = keys[s0];
        if (tid == 0) s_len = n - s0;
        __syncthreads();
        // run length: the first later position with another key
        for (uint32_t base = s0; base < n; base += kBlock) {
            const uint32_t p = base + tid;
            if (p < n && keys[p] != k) atomicMin(&s_len, p - s0);
            __syncthreads();
            const bool found = s_len < base + kBlock - s0;
            __syncthreads();
            if (found) break;
        }
        const uint32_t L = s_len;
        uint32_t *run = vals + s0, *tmp = tmp_v + s0;
        // sorted chunks, written to tmp
        for (uint32_t c0 = 0; c0 < L; c0 += kTieChunk) {
            for (uint32_t j = tid; j < kTieChunk; j += kBlock) {
                const uint32_t p = c0 + j;
                const uint32_t v = p < L ? run[p] : 0u;
                s_v[j] = v;
                s_k[j] = p < L ? gmap[v] : 0xffffffffu;
            }
            __syncthreads();
            for (uint32_t size = 2; size <= kTieChunk; size <<= 1) {
                for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                    for (uint32_t j = tid; j < kTieChunk; j += kBlock) {
                        const uint32_t q = j ^ stride;
                        if (q > j) {
                            const bool up = (j & size) == 0;
                            const uint32_t kj = s_k[j], kq = s_k[q];
                            if ((kj > kq) == up) {
                                s_k[j] = kq;
                                s_k[q] = kj;
                                const uint32_t t = s_v[j];
                                s_v[j] = s_v[q];
                                s_v[q] = t;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            for (uint32_t j = tid; j < kTieChunk; j += kBlock)
                if (c0 + j < L) tmp[c0 + j] = s_v[j];
            __syncthreads();
        }
        // merge passes: pieces of w sorted values, pairs merged into the
        // other buffer
        const uint32_t *src = tmp;
        uint32_t *dst = run;
        for (uint32_t w = kTieChunk; w < L; w <<= 1) {
            for (uint32_t p = tid; p < L; p += kBlock) {
                const uint32_t p0 = p / (2 * w) * (2 * w);
                const uint32_t mid = p0 + w < L ? p0 + w : L, end = p0 + 2 * w < L ? p0 + 2 * w : L;
                const uint32_t v = src[p], key = gmap[v];
                const uint32_t pos = p < mid ? (p - p0) + tie_lower_bound(src + mid, end - mid, gmap, key)
                                             : (p - mid) + tie_lower_bound(src + p0, mid - p0, gmap, key);
                dst[p0 + pos] = v;
            }
            __syncthreads();
            const uint32_t *t = src;
            src = dst;
            dst = const_cast<uint32_t *>(t);
        }
        if (src != run)
            for (uint32_t p = tid; p < L; p += kBlock) run[p] = src[p];
        __syncthreads();
    }
}

}  // namespace

void launch_radix_pass(const void *keys_in, const uint32_t *vals_in, void *keys_out, uint32_t *vals_out,
                       uint32_t n_host, const uint32_t *n_dev, int shift, int bits, bool filter, bool write_keys,
                       uint32_t *hist, uint32_t *gsum, uint32_t *gsum_next, hipStream_t s, uint2 *run_ends,
                       uint32_t nruns, int key_bytes, const uint64_t *mask_in, uint64_t *mask_out, bool whole_key) {
    if (n_host == 0) return;
    const unsigned nb = kSortBlocks;
    const bool k16 = key_bytes == 2;
    const uint32_t *k32i = static_cast<const uint32_t *>(keys_in);
    const uint16_t *k16i = static_cast<const uint16_t *>(keys_in);
    const bool wide = bits > kRadixBits;  // a 9-bit digit: 16-bit keys with a payload only
    if (k16 && wide)
        hipLaunchKernelGGL((k_radix_upsweep<false, uint16_t, kRadixBitsMax>), dim3(nb), dim3(kBlock), 0, s, k16i,
                           n_host, n_dev, shift, bits, hist, gsum);
    else if (k16)
        hipLaunchKernelGGL((k_radix_upsweep<false, uint16_t>), dim3(nb), dim3(kBlock), 0, s, k16i, n_host, n_dev,
                           shift, bits, hist, gsum);
    else if (filter)
        hipLaunchKernelGGL((k_radix_upsweep<true, uint32_t>), dim3(nb), dim3(kBlock), 0, s, k32i, n_host, n_dev,
                           shift, bits, hist, gsum);
    else
        hipLaunchKernelGGL((k_radix_upsweep<false, uint32_t>), dim3(nb), dim3(kBlock), 0, s, k32i, n_host, n_dev,
                           shift, bits, hist, gsum);
    const bool ident = vals_in == nullptr;
    uint32_t *ends = reinterpret_cast<uint32_t *>(run_ends);
#define FGS_DS(I, F, K, T)                                                                                          \
    hipLaunchKernelGGL((k_radix_downsweep<I, F, K, T>), dim3(nb), dim3(kBlock), 0, s, static_cast<const T *>(keys_in), \
                       vals_in, static_cast<T *>(keys_out), vals_out, n_host, n_dev, shift, bits, hist, gsum,         \
                       gsum_next, ends, nruns, nullptr, nullptr, nullptr)
#define FGS_DSP(K, DB)                                                                                              \
    hipLaunchKernelGGL((k_radix_downsweep<true, false, K, uint16_t, true, DB>), dim3(nb), dim3(kBlock), 0, s,     \
                       static_cast<const uint16_t *>(keys_in), vals_in, static_cast<uint16_t *>(keys_out), vals_out,   \
                       n_host, n_dev, shift, bits, hist, gsum, gsum_next, whole_key ? nullptr : ends, nruns, mask_in,  \
                       mask_out, whole_key ? ends : nullptr)
    // 16-bit keys with a payload: the super-tile passes (one 9-bit pass
    // sorts up to 512 super-tiles)
    if (k16 && mask_in && wide && write_keys) FGS_DSP(true, kRadixBitsMax);
    else if (k16 && mask_in && wide) FGS_DSP(false, kRadixBitsMax);
    else if (k16 && mask_in && write_keys) FGS_DSP(true, kRadixBits);
    else if (k16 && mask_in) FGS_DSP(false, kRadixBits);
    // 16-bit keys: unfiltered, explicit values
    else if (k16 && write_keys) FGS_DS(false, false, true, uint16_t);
    else if (k16) FGS_DS(false, false, false, uint16_t);
    else if (ident && filter && write_keys) FGS_DS(true, true, true, uint32_t);
    else if (!ident && !filter && write_keys) FGS_DS(false, false, true, uint32_t);
    else if (!ident && !filter && !write_keys) FGS_DS(false, false, false, uint32_t);
    else if (ident && !filter && write_keys) FGS_DS(true, false, true, uint32_t);
    else FGS_DS(false, true, true, uint32_t);
#undef FGS_DS
#undef FGS_DSP
}

void launch_count_scan(const uint32_t *order, const uint8_t *count8, const uint4 *erec, uint32_t n_host,
                       const uint32_t *n_dev, uint32_t *cs, uint32_t *sums, uint32_t *offsets, uint32_t *total,
                       hipStream_t s) {
    if (n_host == 0) return;
    hipLaunchKernelGGL(k_scan_upsweep, dim3(kSortBlocks), dim3(kBlock), 0, s, order, count8, erec, n_host, n_dev, cs,
                       sums);
    hipLaunchKernelGGL(k_scan_downsweep, dim3(kSortBlocks), dim3(kBlock), 0, s, cs, n_host, n_dev, sums, offsets,
                       total);
}

void launch_depth_ties(const uint32_t *keys, uint32_t *vals, const uint32_t *gmap, uint32_t n_host,
                       const uint32_t *n_dev, uint32_t *long_list, FrameCounters *fc, uint32_t *tmp_v, hipStream_t s) {
    if (n_host == 0) return;
    const uint32_t per_block = (uint32_t)kWaves * kTieOwn;
    const uint32_t blocks = (n_host + per_block - 1) / per_block;
    hipLaunchKernelGGL(k_depth_ties, dim3(blocks), dim3(kBlock), 0, s, keys, vals, gmap, n_host, n_dev, long_list,
                       fc);
    hipLaunchKernelGGL(k_depth_long_ties, dim3(64), dim3(kBlock), 0, s, keys, vals, gmap, n_host, n_dev, long_list,
                       static_cast<const FrameCounters *>(fc), tmp_v);
}

}  // namespace fgs
