// Radix sort of (key, value) pairs by one onesweep pass per 8-bit digit, the
// device-wide scan of per-Gaussian tile counts, and tile-range extraction
// (the sort stage of Sec. 2.2; Alg. 2 offsets).
//
// Onesweep pass (one workgroup per 4096 keys, wave64):
//   1. a dynamic workgroup id from an atomic counter (forward progress of
//      the look-back: every predecessor already runs);
//   2. each wave ranks its 1024 keys, 64 at a time, by digit with ballots
//      (stable: lane order within a step, step order within the wave);
//   3. the workgroup's digit counts are published and the exclusive prefix
//      over predecessor workgroups is found by decoupled look-back;
//   4. keys are staged in LDS in digit order and written out coalesced.
// Status words carry an epoch so that no clearing is needed between passes;
// every wait is bounded and reports through FrameCounters::error.
#include "fgs_internal.hpp"

namespace fgs {
namespace {

constexpr int kWave = 64;
constexpr int kWaves = kBlock / kWave;
constexpr uint32_t kSpinLimit = 1u << 22;

__device__ __forceinline__ uint64_t status_word(uint32_t epoch, uint32_t flag, uint32_t value) {
    return ((uint64_t)((epoch << 2) | flag) << 32) | value;
}

__device__ __forceinline__ uint64_t load_status(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_status(uint64_t *p, uint64_t w) {
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Exclusive scan of one value per thread over a 256-thread workgroup.
// Returns the exclusive prefix; *total receives the sum.  Uses s_tmp[kWaves].
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *s_tmp, uint32_t *total) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, kWave);
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

template <bool kIdentityVals, bool kFilter, bool kWriteKeys>
__global__ __launch_bounds__(kBlock) void k_onesweep(const uint32_t *__restrict__ keys_in,
                                                     const uint32_t *__restrict__ vals_in,
                                                     uint32_t *__restrict__ keys_out, uint32_t *__restrict__ vals_out,
                                                     uint32_t n_host, const uint32_t *n_dev, int shift, int bits,
                                                     int pass, FrameCounters *fc, uint64_t *status, uint32_t epoch) {
    __shared__ uint32_t s_keys[kSortTile];
    __shared__ uint32_t s_vals[kSortTile];
    __shared__ uint32_t s_wave[kWaves][kRadix];
    __shared__ uint32_t s_block_excl[kRadix];
    __shared__ uint32_t s_gbase[kRadix];
    __shared__ uint32_t s_tmp[kWaves];
    __shared__ uint32_t s_bid, s_nvalid, s_err;

    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    if (tid == 0) {
        s_bid = atomicAdd(&fc->block_ctr[pass], 1u);
        s_err = 0u;
    }
    for (int i = tid; i < kWaves * kRadix; i += kBlock) (&s_wave[0][0])[i] = 0;
    __syncthreads();
    const uint32_t bid = s_bid;
    uint32_t n = n_host;
    if (n_dev) {
        const uint32_t nd = *n_dev;
        n = nd < n_host ? nd : n_host;
    }
    const uint32_t nblocks = (n + kSortTile - 1) / kSortTile;
    if (bid >= nblocks) return;  // uniform across the workgroup

    const uint32_t dmask = (1u << bits) - 1u;
    const uint32_t base = bid * kSortTile + (uint32_t)wave * (kSortItems * kWave);
    const uint64_t lt = (1ull << lane) - 1ull;
    uint32_t key[kSortItems], val[kSortItems], rank[kSortItems];

#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const uint32_t idx = base + (uint32_t)(i * kWave + lane);
        const bool in = idx < n;
        const uint32_t k = in ? keys_in[idx] : kInvalidKey;
        const bool ok = in && (!kFilter || k != kInvalidKey);
        key[i] = k;
        val[i] = kIdentityVals ? idx : (in ? vals_in[idx] : 0u);
        const uint32_t d = (k >> shift) & dmask;
        uint64_t peers = __ballot(ok);
        for (int b = 0; b < bits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        const uint32_t before = (uint32_t)__popcll(peers & lt);
        const uint32_t cnt = (uint32_t)__popcll(peers);
        uint32_t prev = 0;
        if (ok) prev = s_wave[wave][d];
        if (ok && before == 0) s_wave[wave][d] = prev + cnt;
        rank[i] = ok ? prev + before : 0xffffffffu;
    }
    __syncthreads();

    // thread t owns digit t: counts per wave -> exclusive over waves
    uint32_t dsum = 0;
    {
        const uint32_t c0 = s_wave[0][tid], c1 = s_wave[1][tid], c2 = s_wave[2][tid], c3 = s_wave[3][tid];
        s_wave[0][tid] = 0;
        s_wave[1][tid] = c0;
        s_wave[2][tid] = c0 + c1;
        s_wave[3][tid] = c0 + c1 + c2;
        dsum = c0 + c1 + c2 + c3;
    }
    uint32_t nvalid = 0;
    const uint32_t bexcl = block_exclusive_scan(dsum, s_tmp, &nvalid);
    s_block_excl[tid] = bexcl;
    // global digit bases from the pass histogram
    uint32_t htot = 0;
    const uint32_t hexcl = block_exclusive_scan(fc->hist[pass][tid], s_tmp, &htot);

    // decoupled look-back over predecessor workgroups for digit tid
    uint64_t *st = status + (uint64_t)bid * kRadix + tid;
    uint32_t prefix = 0;
    if (bid == 0) {
        store_status(st, status_word(epoch, kFlagInclusive, dsum));
    } else {
        store_status(st, status_word(epoch, kFlagAggregate, dsum));
        int64_t j = (int64_t)bid - 1;
        uint32_t spins = 0;
        while (true) {
            const uint64_t w = load_status(status + (uint64_t)j * kRadix + tid);
            const uint32_t tag = (uint32_t)(w >> 32);
            const uint32_t flag = tag & 3u;
            if ((tag >> 2) != (epoch & 0x3fffffffu) || flag == 0u) {
                if (++spins > kSpinLimit) {
                    atomicOr(&fc->error, 1u);
                    s_err = 1u;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            prefix += (uint32_t)w;
            if (flag == kFlagInclusive) break;
            --j;
        }
        store_status(st, status_word(epoch, kFlagInclusive, prefix + dsum));
    }
    s_gbase[tid] = hexcl + prefix;
    if (tid == 0) s_nvalid = nvalid;
    __syncthreads();

    // stage in LDS in digit order
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        if (rank[i] != 0xffffffffu) {
            const uint32_t d = (key[i] >> shift) & dmask;
            const uint32_t lp = s_block_excl[d] + s_wave[wave][d] + rank[i];
            s_keys[lp] = key[i];
            s_vals[lp] = val[i];
        }
    }
    __syncthreads();
    if (s_err) return;  // a bounded wait gave up: write nothing
    const uint32_t nv = s_nvalid;
    for (uint32_t j = tid; j < nv; j += kBlock) {
        const uint32_t k = s_keys[j];
        const uint32_t d = (k >> shift) & dmask;
        const uint32_t gpos = s_gbase[d] + (j - s_block_excl[d]);
        if (gpos >= n) continue;  // never leave the output (n bounds the scattered count)
        if (kWriteKeys) keys_out[gpos] = k;
        vals_out[gpos] = s_vals[j];
    }
}

// Gather per-Gaussian tile counts in depth order and exclusive-scan them
// (single pass with decoupled look-back); offsets[n] and fc->pairs get the total.
__global__ __launch_bounds__(kBlock) void k_count_scan(const uint32_t *__restrict__ order,
                                                       const uint32_t *__restrict__ count, uint32_t n_host,
                                                       uint32_t *__restrict__ offsets, FrameCounters *fc,
                                                       uint64_t *status, uint32_t epoch) {
    __shared__ uint32_t s_tmp[kWaves];
    __shared__ uint32_t s_bid, s_prefix, s_err;
    const int tid = threadIdx.x, lane = tid & (kWave - 1);
    if (tid == 0) {
        s_bid = atomicAdd(&fc->block_ctr[kMaxPasses], 1u);
        s_err = 0u;
    }
    __syncthreads();
    const uint32_t bid = s_bid;
    const uint32_t vis = fc->visible;
    const uint32_t n = vis < n_host ? vis : n_host;
    const uint32_t nblocks = (n + kSortTile - 1) / kSortTile;
    if (bid >= nblocks) return;
    const uint32_t base = bid * kSortTile + (uint32_t)tid * kSortItems;
    uint32_t c[kSortItems];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const uint32_t idx = base + (uint32_t)i;
        c[i] = idx < n ? count[order[idx]] : 0u;
        sum += c[i];
    }
    uint32_t agg = 0;
    const uint32_t texcl = block_exclusive_scan(sum, s_tmp, &agg);
    if (tid < kWave) {
        uint32_t prefix = 0;
        if (bid == 0) {
            if (lane == 0) store_status(status + bid, status_word(epoch, kFlagInclusive, agg));
        } else {
            if (lane == 0) store_status(status + bid, status_word(epoch, kFlagAggregate, agg));
            int64_t j = (int64_t)bid - 1;
            uint32_t spins = 0;
            while (true) {
                const int64_t idx = j - lane;
                uint64_t w;
                if (idx >= 0)
                    w = load_status(status + idx);
                else
                    w = status_word(epoch, kFlagInclusive, 0u);
                const uint32_t tag = (uint32_t)(w >> 32);
                const bool ready = (tag >> 2) == (epoch & 0x3fffffffu) && (tag & 3u) != 0u;
                const uint64_t incl = __ballot(ready && (tag & 3u) == kFlagInclusive);
                const uint64_t notready = __ballot(!ready);
                const int first = incl ? (__ffsll((unsigned long long)incl) - 1) : kWave;
                const uint64_t need = first >= kWave - 1 ? ~0ull : ((2ull << first) - 1ull);
                if (notready & need) {
                    if (++spins > kSpinLimit) {
                        if (lane == 0) {
                            atomicOr(&fc->error, 1u);
                            s_err = 1u;
                        }
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                uint32_t v = lane <= first ? (uint32_t)w : 0u;
#pragma unroll
                for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d, kWave);
                prefix += v;
                if (first < kWave) break;
                j -= kWave;
            }
            if (lane == 0) store_status(status + bid, status_word(epoch, kFlagInclusive, prefix + agg));
        }
        if (lane == 0) s_prefix = prefix;
    }
    __syncthreads();
    if (s_err) return;
    uint32_t run = s_prefix + texcl;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const uint32_t idx = base + (uint32_t)i;
        if (idx < n) offsets[idx] = run;
        run += c[i];
        if (idx + 1 == n) {
            offsets[n] = run;
            fc->pairs = run;
        }
    }
}

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

void launch_onesweep(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_out, uint32_t *vals_out,
                     uint32_t n_host, const uint32_t *n_dev, int shift, int bits, int pass, bool filter,
                     bool write_keys, FrameCounters *fc, uint64_t *status, uint32_t epoch, hipStream_t s) {
    if (n_host == 0) return;
    const unsigned grid = (n_host + kSortTile - 1) / kSortTile;
    const bool ident = vals_in == nullptr;
#define FGS_OS(I, F, K)                                                                                    \
    hipLaunchKernelGGL((k_onesweep<I, F, K>), dim3(grid), dim3(kBlock), 0, s, keys_in, vals_in, keys_out, \
                       vals_out, n_host, n_dev, shift, bits, pass, fc, status, epoch)
    if (ident && filter && write_keys) FGS_OS(true, true, true);
    else if (!ident && !filter && write_keys) FGS_OS(false, false, true);
    else if (!ident && !filter && !write_keys) FGS_OS(false, false, false);
    else if (ident && !filter && write_keys) FGS_OS(true, false, true);
    else FGS_OS(false, true, true);
#undef FGS_OS
}

void launch_count_scan(const uint32_t *order, const uint32_t *count, uint32_t n_host, uint32_t *offsets,
                       FrameCounters *fc, uint64_t *status, uint32_t epoch, hipStream_t s) {
    if (n_host == 0) return;
    const unsigned grid = (n_host + kSortTile - 1) / kSortTile;
    hipLaunchKernelGGL(k_count_scan, dim3(grid), dim3(kBlock), 0, s, order, count, n_host, offsets, fc, status,
                       epoch);
}

void launch_tile_ranges(const uint32_t *tile_keys, uint32_t n, uint2 *ranges, uint32_t ntiles, hipStream_t s) {
    launch_fill_u32(reinterpret_cast<uint32_t *>(ranges), 0u, (size_t)ntiles * 2, s);
    if (n == 0) return;
    hipLaunchKernelGGL(k_tile_ranges, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, tile_keys, n, ranges, ntiles);
}

}  // namespace fgs
