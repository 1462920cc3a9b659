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
constexpr int kRadixBitsMax = 9;  // a single pass may take a 9-bit digit
constexpr int kRadixMax = 1 << kRadixBitsMax;
constexpr uint32_t kInvalidKey = 0xffffffffu;

// Camera and options passed by value: they land in the kernel-argument
// segment and are read through scalar registers (the paper's constant-memory
// placement of frame constants, Sec. 5.3.1).
struct DevCamera {
    float R[9], t[3], eye[3];
    float fx, fy, cx, cy, near_z;
};

// The camera in binary64 for the blend's conic (see GaussState): rotation,
// translation and focal lengths promoted from the binary32 camera, and the
// Jacobian clamp limits jac_clip (W / 2) / fx, jac_clip (H / 2) / fy.
// Computed on the host, so that the kernels read them as uniform arguments.
struct DevCam64 {
    double R[9], t[3];
    double fx, fy, limx, limy;
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

// View-independent precompute of a resident scene (see launch_prepare).
struct DevPrepared {
    const float4 *pos_o;  // (x, y, z, opacity); opacity 0: never visible
    const float4 *cov;    // 2 per Gaussian: (s0, s1, s2, k^2), (w, x, y, z): scales exp(log-scale)
                          // and the unit quaternion, both binary32 as the canonical evaluation rounds them
    const float *sh;      // Gaussian-major SH, sh_stride floats per Gaussian
    const float2 *bnd;    // (trace of the 3D covariance, k^2): bounds the screen extent
    const uint32_t *orig; // Gaussian (index in the caller's scene) of each precompute slot: the slots
                          // follow a spatial order of the means (see launch_prepare)
    int sh_stride;
    // per batch of kBlock consecutive slots, over its members that can be
    // visible (opacity > 0, finite mean): (min x, min y, min z, max opacity),
    // (max x, max y, max z, max trace), (max k^2, 0, 0, 0); a NaN trace or k^2
    // is taken as +inf (see launch_block_bounds)
    const float4 *blk;
};

// Per-Gaussian state of the blend, 48 bytes = 3 x float4.
//   f0 = (u, v, Ab, Bb)   f1 = (Cb, k2, log2 o, r)   f2 = (g, b, depth, o)
// (Ab, Bb, Cb) is the conic evaluated in binary64 from the binary32 scales
// and unit quaternion and rounded once: the blend and its adjoint evaluate
// pixels with it.  The canonical binary32 conic (A, B, C), which decides the
// Gaussian-tile pairs (exact tile test) bit for bit, travels in a separate
// float4 array (A, B, C, 0): the preprocess tests the small rectangles
// itself, so only the large ones' tests (and the frame introspection) read
// it.  For long thin footprints the binary32 inverse of the dilated 2D
// covariance loses most of its bits to cancellation in the determinant; the
// binary64 one keeps the narrow axis.
struct alignas(16) GaussState {
    float4 f0, f1, f2;
};

// Frame-scoped device counters, cleared at the start of a frame.
struct FrameCounters {
    uint32_t visible;  // Gaussians that passed preprocessing
    uint32_t pairs;    // total (Gaussian, tile) pairs: the preprocess adds the small rectangles' hits, the
                       // large-rectangle tests theirs
    uint32_t error;    // error bits (kErrChunkOverflow)
    uint32_t nchunks;  // entries requested in the large-Gaussian chunk list
    uint32_t ncand;    // candidates of a prepared scene's cull (dense depth keys)
    uint32_t nlong;    // runs of more than kShortTieRun equal depths (prepared scene)
    uint32_t entries;  // (Gaussian, super-tile) entries (written by the count scan)
    uint32_t cull_read;  // batches of kBlock slots a prepared scene's cull read (the others its
                         // batch bounds skipped; written by the preprocess)
};

// Super-tiles: blocks of kSuper x kSuper tiles (the last row and column may be
// cut by the image).  Key emission writes one entry per (Gaussian, super-tile
// its tile rectangle overlaps): the super-tile's id and the 64-bit mask of
// the Gaussian's tiles in it (bit lx + kSuper ly, after the exact test; an
// overlapped super-tile none of whose tiles is hit keeps a zero mask).  The
// entries are sorted by super-tile, and each super-tile's depth-ordered
// entries are expanded into its 64 tiles' lists (see launch_tile_lists).
constexpr int kSuperShift = 3;
constexpr int kSuper = 1 << kSuperShift;
constexpr int kMaxSupers = 65536;  // super-tile ids travel as uint16
// The four per-pair arrays of capacity capN are one block: the last holds
// the sorted values, the first three (12 capN bytes) the entries of both
// sort buffers (kEntryBytes each: mask, Gaussian index, super-tile id) and
// the tile-list scratch (list_scratch_words).
constexpr size_t kEntryBytes = 2 * (sizeof(uint64_t) + sizeof(uint32_t) + sizeof(uint16_t));
// The tile lists are built from chunks of kListChunk consecutive entries of
// one super-tile (a super-tile's last chunk may be shorter), one wavefront
// each; at most list_chunks_max of them.
constexpr uint32_t kListChunk = 256;
__host__ __device__ inline size_t list_chunks_max(size_t ecap, size_t nsuper) {
    return (ecap + kListChunk - 1) / kListChunk + nsuper;
}
// Tile-list scratch (words): chunk base of each super-tile (nsuper + 1) and
// pair count of each row of super-tiles (at most nsuper), the super-tile of
// each chunk, 64 per-tile counts of each chunk; each part padded to 64 words.
__host__ __device__ inline size_t list_scratch_words(size_t ecap, size_t nsuper) {
    const size_t g = list_chunks_max(ecap, nsuper);
    return (2 * nsuper + 1 + 63) / 64 * 64 + (g + 63) / 64 * 64 + g * 64;
}

// ---- launchers (implemented in the .hip files) ----------------------------

// Device address of the fixed scratch of fgs_render_noalloc
// (FGS_NOALLOC_SCRATCH_BYTES) on `device`, which must be the current device.
hipError_t noalloc_scratch(int device, unsigned char **base);

void launch_fill_u32(uint32_t *p, uint32_t value, size_t n, hipStream_t s);

// Peak-rate kernels (fgs_measure_peaks): `blocks` workgroups of kBlock lanes,
// each lane running `iters` x 8 independent binary32 FMAs / v_exp_f32; a
// 16-byte-element device copy of `bytes`.
constexpr int kPeakChains = 8;
void launch_peak_fma(int blocks, int iters, float *sink, hipStream_t s);
void launch_peak_exp(int blocks, int iters, float *sink, hipStream_t s);
void launch_peak_copy(const void *src, void *dst, size_t bytes, hipStream_t s);

// Rectangles of more than kBigTiles tiles are tested in chunks of
// kChunkTiles tiles (row-major over the rectangle) by wavefronts spread over
// the whole GPU.
constexpr int kBigTiles = 64;
constexpr int kChunkTiles = kBlock;
constexpr uint32_t kNoChunk = 0xffffffffu;
constexpr size_t kChunkCapAlign = 64;  // chunk-list capacities are multiples of this
constexpr int kPersistentBlocks = 2048;
constexpr int kBigList = 512;                    // pending chunk reservations per workgroup
// FrameCounters::error bits
constexpr uint32_t kErrChunkOverflow = 2u;       // chunk list too small: render again

// Radix sort / scan passes use a fixed grid of kSortBlocks workgroups,
// grouped by kSortGroup for the offset computation.
constexpr int kSortBlocks = 1024;
constexpr int kSortGroup = 32;
constexpr int kSortGroups = (kSortBlocks + kSortGroup - 1) / kSortGroup;
// Group sums of one pass: kSortGroups x (up to kRadixMax) counters.  Every
// pass of a frame has its own (4 depth passes, up to 4 tile passes), cleared
// by the kernel that runs before the pass.
constexpr int kGsumWords = kSortGroups * kRadixMax;
constexpr int kGsumSlots = 8;

unsigned preprocess_grid(int64_t P);
unsigned emit_grid(uint32_t visible);

// Preprocess: per-Gaussian state, tile rectangle, exact tile count, emission
// record, depth key (kInvalidKey for culled Gaussians) and the visible count.
// What later kernels need is always written: state, emission record, one-byte
// count, depth key, Gaussian map, and for rectangles of more than kBigTiles
// tiles the canonical conic and count 0.  With `full` (a frame kept for
// introspection or the backward) the rectangle, the count and the canonical
// conic of every valid Gaussian are written too, and a prepared scene's
// culled candidates get zero state, rectangle and conic.
// The emission record is (tx0 | tx1 << 16, ty0 | ty1 << 16, hit mask low,
// hit mask high).  Large rectangles append one chunk entry (g, first chunk)
// per kChunkTiles tiles to `chunks` (capacity chunk_cap; on overflow the
// error bit kErrChunkOverflow is set and the host renders the frame again
// with a larger list) and get count 0 and record (rectangle, 0, first
// chunk).  The small rectangles' hits are added to fc->pairs.
// pp: NULL (raw parameters) or the scene's precompute.  With a precompute a
// cull pass of kCullBlocks workgroups (which also clears *fc) first lists, for each workgroup's
// contiguous range, the Gaussians that may be visible (in index order, at the
// start of the range in cand, capacity sc.P; their number in
// seg_count[workgroup]), and the preprocess runs over those lists only, taken
// as one list of fc->ncand positions: every per-Gaussian output (gs, rect,
// count, erec, dkey, chunk entries) of position i goes to index i, and the
// Gaussian of position i to gmap[i].  Without a precompute the outputs are
// indexed by Gaussian and gmap is unused.
// seg_count holds 2 kCullBlocks words: the candidate counts, then the
// batches each cull workgroup read.
constexpr int kCullBlocks = 2048;
// count8: the number of super-tiles the rectangle overlaps, i.e. its
// entries (kCount8Big for a chunked rectangle, whose entries the scan takes
// from its record): the scan gathers this 1-byte array, which the L2 caches
// hold whole.
constexpr uint8_t kCount8Big = 255;
// gsum_clear: kGsumWords counters cleared (the first depth pass's group sums).
// With a precompute, launch_cull runs first (the preprocess reads its lists).
void launch_cull(const DevScene &sc, const DevPrepared &pp, const DevCamera &cam, const DevOptions &op, int W, int H,
                 uint32_t *cand, uint32_t *seg_count, FrameCounters *fc, hipStream_t s);
void launch_preprocess(const DevScene &sc, const DevPrepared *pp, const DevCamera &cam, const DevCam64 &cam64,
                       const DevOptions &op, int W, int H, GaussState *gs, float4 *conic, uint4 *rect, uint32_t *count,
                       uint8_t *count8, uint4 *erec, uint32_t *dkey, uint32_t *cand, uint32_t *seg_count,
                       uint32_t *gmap, uint2 *chunks, uint32_t chunk_cap, FrameCounters *fc, uint32_t *gsum_clear,
                       bool full, hipStream_t s);

// Multi-camera batch over one prepared scene (Sec. 5.3.1 applied to several
// viewpoints at once): one cull keeps the union of the cameras' candidates,
// and one preprocess pass over that list reads each Gaussian's precompute
// once from HBM and evaluates it for every camera in turn.  Camera c's
// outputs are those launch_preprocess would write for it alone over the
// union list (a candidate culled for camera c gets key kInvalidKey and count
// 0), so every later stage runs per camera unchanged.
constexpr int kMaxCams = 8;  // FGS_MAX_BATCH_CAMERAS
struct CamOut {
    DevCamera cam;
    DevCam64 cam64;
    int W, H;  // this camera's image
    GaussState *gs;
    float4 *conic;
    uint4 *rect;
    uint32_t *count;
    uint8_t *count8;
    uint4 *erec;
    uint32_t *dkey;
    uint32_t *gmap;        // this camera's copy of the list's Gaussian indices
    uint2 *chunks;
    FrameCounters *fc;     // this camera's counters (cleared by the cull)
    uint32_t *gsum_clear;  // this camera's first depth pass group sums
    uint32_t chunk_cap;
};
struct MultiOut {
    CamOut c[kMaxCams];
    int n;  // cameras in the batch, 1..kMaxCams
};
// Each camera has its own image size.  cand, seg_count: as for
// launch_preprocess (one union list); each camera gets the list's Gaussian
// indices in its own CamOut::gmap (gmap is unused).
void launch_preprocess_multi(const DevScene &sc, const DevPrepared &pp, const MultiOut &mo, const DevOptions &op,
                             uint32_t *cand, uint32_t *seg_count, uint32_t *gmap, hipStream_t s);

// View-independent precompute (opacity, 3D covariance, k^2, log2 opacity,
// Gaussian-major SH) for options op (alpha_min and cap_3sigma), stored in
// slot order: slot i holds Gaussian perm[i] (orig[i] = perm[i]).
void launch_prepare(const DevScene &sc, const DevOptions &op, const uint32_t *perm, float4 *pos_o, float4 *cov,
                    float *sh, float2 *bnd, uint32_t *orig, int sh_stride, hipStream_t s);
// Batch bounds of a prepared scene (DevPrepared::blk, 3 float4 per batch of
// kBlock slots), from the precompute's positions, opacities and extent
// bounds.  The cull skips a batch whose bounds show that it would drop every
// member (Sec. 5.3.1: the view-independent part precomputed once): behind
// the near plane, below the opacity threshold, or off the image.
void launch_block_bounds(const float4 *pos_o, const float2 *bnd, int64_t P, float4 *blk, hipStream_t s);
// Spatial order of a scene's Gaussians: bounds[0..5] = (min x, y, z, max x,
// y, z) of the finite means (bounds: 6 words, initialised by the launcher),
// then keys[g] = 30-bit Morton code of the mean quantised to 1024 cells per
// axis of that box (0xffffffff for a non-finite mean).  Sorting (key, g) by
// key gives the precompute's slot order: a cull's candidates then lie in
// few contiguous runs of slots.
void launch_spatial_keys(const DevScene &sc, uint32_t *bounds, uint32_t *keys, hipStream_t s);

// Depth ties of a prepared scene's frame: the depth sort orders equal depths
// by list position, which follows the precompute's spatial order; the
// method's order (depth, then Gaussian index) needs every run of equal keys
// re-ordered by gmap (the list position's Gaussian index).  keys: the sorted
// depth keys, vals: the sorted list positions (n = *n_dev, bounded by
// n_host).  A run of at most kShortTieRun is sorted by the thread that
// starts it; longer runs (rare: that many Gaussians at one binary32 depth)
// are listed in long_list (fc->nlong of them, which the frame's cull
// cleared) and sorted by one workgroup each, with the run's region of tmp_v
// ([n_host]) as scratch.
constexpr int kShortTieRun = 32;
void launch_depth_ties(const uint32_t *keys, uint32_t *vals, const uint32_t *gmap, uint32_t n_host,
                       const uint32_t *n_dev, uint32_t *long_list, FrameCounters *fc, uint32_t *tmp_v, hipStream_t s);

// Exact tile tests of the chunked Gaussians: chunk c of a Gaussian holds
// tiles [c kChunkTiles, (c + 1) kChunkTiles) of its rectangle in row-major
// order.  Writes each chunk's hit mask (kChunkTiles / 32 words, bit i = tile
// c kChunkTiles + i), adds the hits to count[g] and to fc->pairs.
void launch_big_count(int W, int H, int binning, const GaussState *gs, const float4 *conic, const uint4 *erec,
                      const uint2 *chunks, uint32_t chunk_cap, uint32_t *chunk_mask, uint32_t *count,
                      FrameCounters *fc, hipStream_t s);

// Number of super-tiles a tile rectangle [tx0, tx1] x [ty0, ty1] overlaps:
// the rectangle's entries.
__host__ __device__ inline uint32_t super_span(int tx0, int tx1, int ty0, int ty1) {
    return (uint32_t)(((tx1 >> kSuperShift) - (tx0 >> kSuperShift) + 1) *
                      ((ty1 >> kSuperShift) - (ty0 >> kSuperShift) + 1));
}

// Key emission at super-tile granularity: for the visible Gaussians in depth
// order (order, `visible` or the bound-checked *visible_dev), the entries of
// Gaussian order[r] go to [offsets[r], offsets[r] + its count) in row-major
// order of the overlapped super-tiles: key = super-tile id (sy * stx + sx),
// gidx = the Gaussian's output slot, mask = its hit tiles in the super-tile.
// Small rectangles take the hit mask of their emission record.  A chunked
// Gaussian leaves (output slot, offset) at big[first chunk], and a second
// kernel gathers its super-tiles' bits from the chunk masks of
// launch_big_count (chunks, big: capacity chunk_cap; ng bounds the output
// slots).  Entries at or beyond ecap are dropped (the host sees the count
// and renders again).  Also sets the super-tile ranges empty, (0xffffffff,
// 0) for s < nsuper, and clears the first sort pass's group sums
// (gsum_clear, kGsumWords words).
void launch_super_emit(int W, int H, const uint32_t *order, uint32_t visible, const uint32_t *visible_dev,
                       const uint32_t *offsets, const uint4 *erec, uint32_t ng, const uint2 *chunks, uint2 *big,
                       const uint32_t *chunk_mask, uint32_t chunk_cap, const FrameCounters *fc, uint16_t *skey,
                       uint32_t *gidx, uint64_t *smask, uint32_t ecap, uint2 *sranges, uint32_t nsuper,
                       uint32_t *gsum_clear, hipStream_t s);

// Per-tile lists from the entries sorted by super-tile (stable, so each
// super-tile's entries are in depth order): sranges[s] = [start, end) of
// super-tile s in the sorted arrays (start > end: none; at most ecap).  Every
// pair (entry, set mask bit) is written to values at its tile's start plus
// the number of earlier entries of the super-tile that hit the same tile,
// which is the order of the method's stable sort by (tile, depth).  ranges[t]
// = [start, end) of tile t for every tile of the W x H image (an empty tile
// gets start == end), clamped to ncap; writes beyond ncap are dropped.
// scratch: list_scratch_words(ecap, super-tiles) words.
void launch_tile_lists(int W, int H, const uint2 *sranges, const uint32_t *gidx, const uint64_t *smask,
                       uint32_t ecap, uint32_t *scratch, uint2 *ranges, uint32_t *values, uint32_t ncap,
                       hipStream_t s);

// One stable LSD radix pass of (key, value) pairs by the digit
// (key >> shift) & ((1 << bits) - 1), bits <= kRadixBitsMax (9 only for
// 16-bit keys with a payload).
//   n_host  upper bound on the number of keys; n_dev: if non-null, the
//           actual count is read there on the device
//   vals_in null: values are the input positions
//   filter  drop keys equal to kInvalidKey
//   hist    scratch [kSortBlocks][kRadixMax]
//   gsum    [kSortGroups][kRadixMax], zero on entry: the upsweep adds each
//           workgroup's histogram into its group's row (so no separate group
//           kernel runs); gsum_next, if non-null, is cleared by the downsweep
//           for the next pass
//   run_ends if non-null (the last pass of a sort by the whole key, keys <
//           nruns): run_ends[k] = [start, end) of key k's run in the output,
//           by atomic min / max on entries that the caller set empty (the
//           emission does for the super-tiles); a key with no element keeps
//           start > end
//   key_bytes 4 (uint32 keys) or 2 (uint16 keys: unfiltered passes with
//           explicit values, or with a payload)
//   mask_in if non-null (16-bit keys only): the payload (vals_in[i],
//           mask_in[i]) travels with key i to (vals_out, mask_out); it is
//           read at its destination's store, from the workgroup's tile
//   whole_key (with a payload and run_ends): the digit is the whole key
//           (shift 0, keys < 2^bits), so each key's run is its digit's
//           range, written by the first workgroup from the digit offsets
//           (every key < nruns gets it, an absent key start == end)
void launch_radix_pass(const void *keys_in, const uint32_t *vals_in, void *keys_out, uint32_t *vals_out,
                       uint32_t n_host, const uint32_t *n_dev, int shift, int bits, bool filter, bool write_keys,
                       uint32_t *hist, uint32_t *gsum, uint32_t *gsum_next, hipStream_t s,
                       uint2 *run_ends = nullptr, uint32_t nruns = 0, int key_bytes = 4,
                       const uint64_t *mask_in = nullptr, uint64_t *mask_out = nullptr, bool whole_key = false);

// offsets[r] = sum of count[order[r']] for r' < r over the n visible
// Gaussians (n_dev, bounded by n_host); offsets[n] and *total get the total.
// The count (super-tile entries) is read from count8, and computed from the
// emission record's rectangle where count8 holds kCount8Big.  cs: scratch
// [n_host]; sums: scratch [kSortBlocks].
void launch_count_scan(const uint32_t *order, const uint8_t *count8, const uint4 *erec, uint32_t n_host,
                       const uint32_t *n_dev, uint32_t *cs, uint32_t *sums, uint32_t *offsets, uint32_t *total,
                       hipStream_t s);

// A one-tile image: ranges[0] = [0, min(*n_dev, n)).
void launch_single_range(uint2 *ranges, uint32_t n, const uint32_t *n_dev, hipStream_t s);

// work: if non-null, work[0] += the number of list entries every pixel
// examines, work[1] += the (wavefront, entry) steps the blend executes (a
// separate, slower kernel instantiation)
// variant: 0 the LDS-batched blend; 1 the prefetch-pipeline blend (same
// image bit for bit; not with work).  nvalues, ngs: entries held by the
// values and gs buffers (the bounds of the variant's buffer loads).
void launch_blend(const GaussState *gs, const uint32_t *values, const uint2 *ranges, int W, int H,
                  const DevOptions &op, float *rgb, float *T, uint32_t *last, unsigned long long *work,
                  int variant, uint32_t nvalues, uint32_t ngs, hipStream_t s);

// Adjoint of the blend: accumulates per-Gaussian sums (9 planes of stride
// acc_stride, cleared by the caller) from dL/dRGB, replaying each pixel's
// tile list back to front from its final transmittance and last contributor.
void launch_blend_backward(const GaussState *gs, const uint32_t *values, const uint2 *ranges, const float *Tfin,
                           const uint32_t *last, const float *dL, int W, int H, const DevOptions &op, float *acc,
                           int64_t acc_stride, hipStream_t s);

// Adjoint of the preprocessing: raw-parameter gradients (planar, stride
// grad_stride, overwritten) from the blend adjoint's sums.
void launch_preprocess_backward(const DevScene &sc, const DevCamera &cam, const DevOptions &op, int W, int H,
                                const GaussState *gs, const float *acc, int64_t acc_stride, float *g_means,
                                float *g_log_scales, float *g_quats, float *g_logits, float *g_sh,
                                int64_t grad_stride, hipStream_t s);

}  // namespace fgs
