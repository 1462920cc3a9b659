// Host-side frame pipeline shared by the plain renderer (runtime.cpp) and the
// render server (server.cpp): device buffers of one frame, argument checks,
// and the two halves of a frame's kernel sequence.  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <string>

#include "fgs.h"
#include "fgs_internal.hpp"

namespace fgs {

// One frame's device buffers, sized for a capacity and reused across frames
// (Sec. 5.3.1: no per-frame allocation once warmed up).
struct FrameBuffers {
    size_t capP = 0, capN = 0, capTiles = 0, capPix = 0;
    // per Gaussian
    GaussState *gs = nullptr;
    float4 *conic = nullptr;  // canonical binary32 conic (A, B, C, 0): large rectangles always, all with `full`
    uint4 *rect = nullptr;    // written with `full` only (introspection)
    uint32_t *count = nullptr;
    uint8_t *count8 = nullptr;  // tile count of a small rectangle, kCount8Big for a chunked one (the scan's gather)
    uint4 *erec = nullptr;  // emission record: rectangle (16-bit) and hit mask
    uint32_t *dkey = nullptr, *dk_b = nullptr, *dv_a = nullptr, *dv_b = nullptr;
    uint32_t *offsets = nullptr;
    uint32_t *seg_count = nullptr;  // a prepared scene's cull: kCullBlocks candidate counts, then batches read
    uint32_t *gmap = nullptr;       // prepared scene: Gaussian of each candidate list position
    // per pair: four arrays of capN words, consecutive parts of one block
    // that starts at tk_a (the entries and the values, see entry_capacity)
    uint32_t *tk_a = nullptr, *tk_b = nullptr, *tv_a = nullptr, *tv_b = nullptr;
    bool pairs_owned = true;  // false: the pair arrays live in a caller's arena
    // per tile / pixel (sranges: per super-tile, sized like ranges)
    uint2 *ranges = nullptr, *sranges = nullptr;
    float *T = nullptr;
    uint32_t *last = nullptr;

    size_t gauss_bytes() const {
        return capP * (sizeof(GaussState) + sizeof(float4) + sizeof(uint4) + sizeof(uint32_t) + sizeof(uint4) +
                       5 * sizeof(uint32_t) +
                       sizeof(uint8_t)) +
               (capP + 1) * sizeof(uint32_t) + 2 * kCullBlocks * sizeof(uint32_t);
    }
    size_t bytes() const {
        return gauss_bytes() + (pairs_owned ? capN * 4 * sizeof(uint32_t) : 0) + capTiles * 2 * sizeof(uint2) +
               capPix * (sizeof(float) + sizeof(uint32_t));
    }
};

// Radix-sort and scan scratch of one in-flight frame.
struct SortScratch {
    uint32_t *rhist = nullptr, *gsum = nullptr, *sums = nullptr;  // gsum: kGsumSlots slots of kGsumWords
    uint32_t *slot(int i) const { return gsum + (size_t)i * kGsumWords; }
    static size_t bytes() {
        return ((size_t)kSortBlocks * kRadixMax + (size_t)kGsumSlots * kGsumWords + kSortBlocks) * sizeof(uint32_t);
    }
};

// List of Gaussians whose rectangles exceed kBigTiles tiles, in chunks of
// kChunkTiles tiles.
struct ChunkList {
    uint2 *chunks = nullptr;
    uint32_t *mask = nullptr;  // kChunkTiles-bit hit mask per chunk
    uint2 *big = nullptr;      // at a Gaussian's first chunk: its output slot and entry offset
    size_t cap = 0;
    size_t bytes() const { return cap * (2 * sizeof(uint2) + (kChunkTiles / 32) * sizeof(uint32_t)); }
};

// Super-tiles of a W x H image.
inline uint32_t super_tiles_x(int W) { return (uint32_t)((((W + kTile - 1) / kTile) + kSuper - 1) >> kSuperShift); }
inline uint32_t super_count(int W, int H) { return super_tiles_x(W) * super_tiles_x(H); }

// Passes of the entries' sort by super-tile id: one for up to
// kRadixBitsMax bits, else kRadixBits per pass.
inline int super_sort_passes(int W, int H) {
    int b = 0;
    while ((1ull << b) < (uint64_t)super_count(W, H)) ++b;
    return b == 0 ? 0 : (b <= kRadixBitsMax ? 1 : (b + kRadixBits - 1) / kRadixBits);
}

// Bytes of the first three per-pair arrays that ecap entries and their
// tile-list scratch take for nsuper super-tiles.
inline size_t entry_bytes(size_t ecap, size_t nsuper) {
    return ecap * kEntryBytes + list_scratch_words(ecap, nsuper) * sizeof(uint32_t);
}

// Entries that the first three per-pair arrays (12 capN bytes) hold beside
// their tile-list scratch for a W x H image (a multiple of 64; 0 if the
// scratch alone does not fit).
inline size_t entry_capacity(size_t capN, int W, int H) {
    const size_t ns = super_count(W, H), room = 12 * capN;
    const size_t fixed = entry_bytes(0, ns);
    if (room < fixed) return 0;
    // per entry kEntryBytes plus a chunk's 65 scratch words per kListChunk
    size_t e = (room - fixed) * kListChunk / (kEntryBytes * kListChunk + 65 * sizeof(uint32_t)) / 64 * 64;
    while (e > 0 && entry_bytes(e, ns) > room) e -= 64;
    return e;
}

// Capacity (in pairs) of the per-pair arrays that a frame with `pairs`
// pairs and `entries` super-tile entries needs: the values in the last
// array, the entries and the tile-list scratch in the other three.
inline size_t pair_capacity_needed(size_t pairs, size_t entries, int W, int H) {
    const size_t e = (entries + 63) / 64 * 64;
    const size_t rest = (entry_bytes(e, super_count(W, H)) + 11) / 12;
    size_t need = pairs > rest ? pairs : rest;
    while (entry_capacity(need, W, H) < e) need += 64;  // rounding of entry_capacity
    return need;
}

hipError_t ensure_gauss(FrameBuffers &b, size_t P);
hipError_t ensure_pairs(FrameBuffers &b, size_t N);
hipError_t ensure_tiles(FrameBuffers &b, size_t tiles);
hipError_t ensure_pixels(FrameBuffers &b, size_t pix);
hipError_t ensure_sort_scratch(SortScratch &s);
hipError_t ensure_chunks(ChunkList &c, size_t need);
void free_frame_buffers(FrameBuffers &b);
void free_sort_scratch(SortScratch &s);
void free_chunks(ChunkList &c);

// Text that fgs_last_error(NULL) returns on this thread (calls without a
// context).
void set_error_without_context(const char *msg);

// Argument checks shared by every entry point; writes a message to err.
fgs_status check_args(const fgs_scene *sc, const fgs_camera *cam, int32_t W, int32_t H, const fgs_options *opt,
                      std::string &err);

DevOptions to_dev(const fgs_options &o);
DevCamera to_dev(const fgs_camera &c);
DevCam64 to_dev64(const fgs_camera &c, const fgs_options &o, int W, int H);
DevCam64 to_dev64(const DevCamera &c, const DevOptions &o, int W, int H);
DevScene to_dev(const fgs_scene &s);

// Optional per-stage HIP events: 0..7 around the stages (0 before the
// preprocess, 1 before the depth sort, 2 before the scan, 3 before the
// emission, 4 before the super-tile sort, 5 before the tile lists, 6 before
// the blend, 7 after it), and kMarkCulled between a prepared scene's cull and
// the preprocess (recorded right after 0 for raw parameters).
constexpr int kMarkCulled = 8;
constexpr int kStageMarks = 9;
struct StageMarks {
    hipEvent_t *ev = nullptr;
    void mark(int i, hipStream_t s) const {
        if (ev) (void)hipEventRecord(ev[i], s);
    }
};

// A second stream and two events that let independent work of one frame run
// beside the main stream (fork: side waits for main; join: main waits for
// side).  All three are owned by the caller; side == nullptr runs everything
// on the main stream.
struct SideStream {
    hipStream_t side = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    hipError_t create();  // non-blocking stream, default priority
    void destroy();
};

// Stages 1 and 2a: preprocess with the exact tile count, depth order of the
// visible Gaussians, scan of the tile counts in depth order.  The exact tests
// of the large rectangles run on the side stream while the depth order is
// sorted on s; the scan waits for both.  Ends with an asynchronous copy of
// the frame counters to host_fc (pinned; NULL: no copy): on s when
// counters_ready is NULL; otherwise on the side stream, followed there by
// counters_ready, so that s goes straight on to the second half.
// pp: NULL (raw parameters) or the scene's view-independent precompute.
// full: also write what only a kept frame's introspection reads (see
// launch_preprocess).
void enqueue_front(const DevScene &sc, const DevPrepared *pp, const DevCamera &cam, const DevOptions &op, int W,
                   int H, FrameBuffers &fb, ChunkList &ch, SortScratch &ss, FrameCounters *fc,
                   FrameCounters *host_fc, hipStream_t s, const SideStream &side, const StageMarks &mk,
                   hipEvent_t counters_ready = nullptr, bool full = false);
// The part of enqueue_front after the preprocess (for a preprocess run
// elsewhere, as in a multi-camera batch).  dense: the outputs are over a
// candidate list of fc->ncand positions (a prepared scene); P32 bounds it.
void enqueue_front_rest(bool dense, uint32_t P32, const DevOptions &op, int W, int H, FrameBuffers &fb, ChunkList &ch,
                        SortScratch &ss, FrameCounters *fc, FrameCounters *host_fc, hipStream_t s,
                        const SideStream &side, const StageMarks &mk, hipEvent_t counters_ready = nullptr);

// Device buffers of a scene's view-independent precompute.
struct PreparedBuffers {
    float4 *pos_o = nullptr;
    float4 *cov = nullptr;
    float *sh = nullptr;
    float2 *bnd = nullptr;
    uint32_t *orig = nullptr;  // Gaussian of each slot (the slots follow a spatial order)
    float4 *blk = nullptr;     // batch bounds, 3 per kBlock slots (see DevPrepared)
    int sh_stride = 0;
    int64_t P = 0;
    size_t batches() const { return (size_t)((P + kBlock - 1) / kBlock); }
    size_t bytes() const {
        return (size_t)P * (3 * sizeof(float4) + sizeof(float2) + sizeof(uint32_t) + (size_t)sh_stride * sizeof(float)) +
               3 * batches() * sizeof(float4);
    }
    DevPrepared dev() const { return DevPrepared{pos_o, cov, sh, bnd, orig, sh_stride, blk}; }
};

// Allocate and fill the precompute of sc for options op on stream s, in a
// spatial slot order (Morton order of the means); waits for the stream.
hipError_t build_prepared(const fgs_scene &sc, const fgs_options &op, PreparedBuffers &pb, hipStream_t s);
void free_prepared(PreparedBuffers &pb);

// Stages 2b to 4: key emission (super-tile entries), their stable sort by
// super-tile, the per-tile lists and ranges, and blending.  Every count is
// read on the device from fc, and every grid is sized by a capacity, so the
// sequence holds no host dependency and can be captured in a graph.  P
// bounds the visible count; fb.capN bounds the pair count (and, through
// entry_capacity, the entries).  The sorted values end in tv_b (returns
// false: not in tv_a).  blend_variant: see launch_blend.
bool enqueue_back(int W, int H, const DevOptions &op, uint32_t P, FrameBuffers &fb, ChunkList &ch, SortScratch &ss,
                  FrameCounters *fc, float *rgb, float *T, uint32_t *last, unsigned long long *work, hipStream_t s,
                  const StageMarks &mk, int blend_variant = 0);

}  // namespace fgs
