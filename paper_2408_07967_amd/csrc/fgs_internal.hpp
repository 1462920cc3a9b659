// Internal declarations shared by the runtime and the kernel translation
// units of the gfx950 rasterizer.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace fgs {

constexpr int kTile = 16;          // tile edge in pixels (16 x 16 tiles)
constexpr int kBlock = 256;        // threads per workgroup for 1D kernels
constexpr int kSortItems = 16;     // keys per thread in a sort pass
constexpr int kSortTile = kBlock * kSortItems;  // keys per sort workgroup
constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr uint32_t kInvalidKey = 0xffffffffu;
constexpr int kMaxPasses = 8;      // 4 depth passes + up to 3 tile passes (+1 spare)

// Camera and options passed by value: they land in the kernel-argument
// segment and are read through scalar registers (the paper's constant-memory
// placement of frame constants, Sec. 5.3.1).
struct DevCamera {
    float R[9], t[3], eye[3];
    float fx, fy, cx, cy, near_z;
};

struct DevOptions {
    float alpha_min, T_stop, alpha_max, dilation, jac_clip;
    float bg[3];
    int cap_3sigma, binning;
};

struct DevScene {
    const float *means, *log_scales, *quats, *logits, *sh;
    int64_t P, stride;
    int D;
};

// Per-Gaussian state for the blend, 48 bytes = 3 x float4.
//   f0 = (u, v, A, B)   f1 = (C, k2, log2 o, r)   f2 = (g, b, depth, o)
struct alignas(16) GaussState {
    float4 f0, f1, f2;
};

// Frame-scoped device counters and histograms, cleared at the start of a frame.
struct FrameCounters {
    uint32_t visible;                    // Gaussians that passed preprocessing
    uint32_t pairs;                      // total pairs (written by the scan)
    uint32_t error;                      // non-zero: a bounded wait gave up
    uint32_t nchunks;                    // entries appended to the large-Gaussian chunk list
    uint32_t block_ctr[kMaxPasses + 2];  // dynamic workgroup ids per pass / scan
    uint32_t hist[kMaxPasses][kRadix];   // digit histograms per pass
    unsigned long long work;             // blend evaluations (instrumented runs)
};

// Lookback status word: high 32 bits = (epoch << 2) | flag, low 32 = value.
constexpr uint32_t kFlagAggregate = 1u;
constexpr uint32_t kFlagInclusive = 2u;

// ---- launchers (implemented in the .hip files) ----------------------------

void launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t s);

// Rectangles of more than kBigTiles tiles are tested and emitted in chunks of
// kChunkTiles tiles by workgroups spread over the whole GPU.
constexpr int kBigTiles = 64;
constexpr int kChunkTiles = kBlock;
constexpr uint32_t kNoChunk = 0xffffffffu;
constexpr int kPersistentBlocks = 2048;
constexpr int kBigList = 512;                    // pending chunk reservations per workgroup
constexpr int kTileHistBins = 3 * kRadix;        // histogram row of the (up to 3) tile passes
constexpr int kDepthHistBins = 4 * kRadix;       // histogram row of the 4 depth passes
// FrameCounters::error bits
constexpr uint32_t kErrLookback = 1u;            // a bounded look-back wait gave up
constexpr uint32_t kErrChunkOverflow = 2u;       // chunk list too small: render again

// Per-workgroup histogram rows: preprocess writes grid rows of kDepthHistBins,
// emission writes rows of kTileHistBins; k_hist_reduce sums them into
// FrameCounters::hist.
void launch_hist_reduce(const uint32_t *rows, uint32_t nrows, int nbins, uint32_t *out, hipStream_t s);
unsigned preprocess_grid(int64_t P);
unsigned emit_grid(uint32_t visible);

// Preprocess: per-Gaussian state, tile rectangle, exact tile count, hit mask,
// depth key (kInvalidKey for culled Gaussians), depth-digit histograms and
// the visible count.  Large rectangles append chunk entries (g, first chunk)
// to `chunks` (capacity chunk_cap; on overflow the Gaussian is counted in
// its own wavefront instead) and get count 0, mask = (0, first chunk).
void launch_preprocess(const DevScene &sc, const DevCamera &cam, const DevOptions &op, int W, int H,
                       GaussState *gs, uint4 *rect, uint32_t *count, uint2 *mask, uint32_t *dkey, uint2 *chunks,
                       uint32_t chunk_cap, uint32_t *block_hist, FrameCounters *fc, hipStream_t s);

// Exact tile counts of the chunked Gaussians: per-chunk hits and atomic
// per-Gaussian sums.
void launch_big_count(int W, int H, int binning, const GaussState *gs, const uint4 *rect, const uint2 *chunks,
                      uint32_t chunk_cap, uint32_t *chunk_hits, uint32_t *count, const FrameCounters *fc,
                      hipStream_t s);

// Emit (tile, gaussian) pairs for Gaussians in depth order.  Chunked
// Gaussians only record their output base in mask[g].x.
void launch_emit(const DevScene &sc, int W, int H, int binning, const uint32_t *order, uint32_t visible,
                 const uint32_t *offsets, const GaussState *gs, const uint4 *rect, const uint32_t *count,
                 uint2 *mask, uint32_t *tile_keys, uint32_t *values, uint32_t cap, uint32_t *block_hist,
                 int npasses, const int *shifts, const int *bits, hipStream_t s);

// Emit the pairs of the chunked Gaussians (after launch_emit); histogram rows
// go after the emit kernel's rows (row0 = emit_grid(visible)).
void launch_big_emit(int W, int H, int binning, const GaussState *gs, const uint4 *rect, const uint2 *mask,
                     const uint2 *chunks, uint32_t chunk_cap, const uint32_t *chunk_hits, uint32_t *tile_keys,
                     uint32_t *values, uint32_t cap, const FrameCounters *fc, uint32_t *block_hist, uint32_t row0,
                     int npasses, const int *shifts, const int *bits, hipStream_t s);

// One onesweep pass: stable scatter of (key, value) by digit
// (key >> shift) & ((1 << bits) - 1).
//   n_host  upper bound on the number of keys (sizes the grid)
//   n_dev   if non-null, the actual count is read here on the device
//   vals_in null: values are the input positions (identity)
//   filter  drop keys equal to kInvalidKey
void launch_onesweep(const uint32_t *keys_in, const uint32_t *vals_in, uint32_t *keys_out, uint32_t *vals_out,
                     uint32_t n_host, const uint32_t *n_dev, int shift, int bits, int pass, bool filter,
                     bool write_keys, FrameCounters *fc, uint64_t *status, uint32_t epoch, hipStream_t s);

// Gather counts in depth order and exclusive-scan them into offsets;
// writes the total into fc->pairs.
void launch_count_scan(const uint32_t *order, const uint32_t *count, uint32_t n_host, uint32_t *offsets,
                       FrameCounters *fc, uint64_t *status, uint32_t epoch, hipStream_t s);

void launch_tile_ranges(const uint32_t *tile_keys, uint32_t n, uint2 *ranges, uint32_t ntiles, hipStream_t s);

// work: if non-null, the blend adds the number of list entries every pixel
// examines (a separate, slower kernel instantiation)
void launch_blend(const GaussState *gs, const uint32_t *values, const uint2 *ranges, int W, int H,
                  const DevOptions &op, float *rgb, float *T, uint32_t *last, unsigned long long *work,
                  hipStream_t s);

}  // namespace fgs
