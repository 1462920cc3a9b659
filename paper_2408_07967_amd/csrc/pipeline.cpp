// Host-side frame pipeline: buffer management, argument checks and the
// kernel sequence of one frame (preprocess -> depth order -> count scan ->
// super-tile entries -> their sort by super-tile -> per-tile lists and
// ranges -> blend).
#include "pipeline.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace fgs {

namespace {

template <class T>
hipError_t grow(T *&p, size_t n_need) {
    if (p) {
        // the old buffer may still be read by queued work
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return e;
        (void)hipFree(p);
    }
    p = nullptr;
    return hipMalloc((void **)&p, (n_need ? n_need : 1) * sizeof(T));
}

#define FGS_GROW(p, n)                       \
    do {                                     \
        hipError_t e_ = grow((p), (n));      \
        if (e_ != hipSuccess) return e_;     \
    } while (0)

void free_p(void *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

bool finite_all(const float *p, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

int ceil_log2(uint64_t x) {
    int b = 0;
    while ((1ull << b) < x) ++b;
    return b;
}

// Split `bits` key bits into passes: one pass of up to kRadixBitsMax bits,
// else passes of at most kRadixBits each.
int plan_tile_passes(int bits, int *shift, int *width) {
    if (bits <= 0) return 0;
    if (bits <= kRadixBitsMax) {
        shift[0] = 0;
        width[0] = bits;
        return 1;
    }
    const int np = (bits + kRadixBits - 1) / kRadixBits;
    int s = 0;
    for (int p = 0; p < np; ++p) {
        const int w = (bits - s + (np - p) - 1) / (np - p);
        shift[p] = s;
        width[p] = w;
        s += w;
    }
    return np;
}

}  // namespace

hipError_t ensure_gauss(FrameBuffers &b, size_t P) {
    if (P <= b.capP && b.gs) return hipSuccess;
    const size_t cap = P + P / 8 + 1024;
    FGS_GROW(b.gs, cap);
    FGS_GROW(b.conic, cap);
    FGS_GROW(b.rect, cap);
    FGS_GROW(b.count, cap);
    FGS_GROW(b.count8, cap);
    FGS_GROW(b.erec, cap);
    FGS_GROW(b.dkey, cap);
    FGS_GROW(b.dk_b, cap);
    FGS_GROW(b.dv_a, cap);
    FGS_GROW(b.dv_b, cap);
    FGS_GROW(b.offsets, cap + 1);
    FGS_GROW(b.seg_count, 2 * kCullBlocks);
    FGS_GROW(b.gmap, cap);
    b.capP = cap;
    return hipSuccess;
}

hipError_t ensure_pairs(FrameBuffers &b, size_t N) {
    if (N <= b.capN && b.tk_a) return hipSuccess;
    const size_t cap = (N + N / 4 + 4096 + 63) / 64 * 64;
    // one block for the four arrays
    FGS_GROW(b.tk_a, 4 * cap);
    b.tk_b = b.tk_a + cap;
    b.tv_a = b.tk_a + 2 * cap;
    b.tv_b = b.tk_a + 3 * cap;
    b.capN = cap;
    b.pairs_owned = true;
    return hipSuccess;
}

hipError_t ensure_tiles(FrameBuffers &b, size_t tiles) {
    if (tiles <= b.capTiles && b.ranges) return hipSuccess;
    FGS_GROW(b.ranges, tiles);
    FGS_GROW(b.sranges, tiles);
    b.capTiles = tiles;
    return hipSuccess;
}

hipError_t ensure_pixels(FrameBuffers &b, size_t pix) {
    if (pix <= b.capPix && b.T) return hipSuccess;
    FGS_GROW(b.T, pix);
    FGS_GROW(b.last, pix);
    b.capPix = pix;
    return hipSuccess;
}

hipError_t ensure_sort_scratch(SortScratch &s) {
    if (s.rhist) return hipSuccess;
    FGS_GROW(s.rhist, (size_t)kSortBlocks * kRadixMax);
    FGS_GROW(s.gsum, (size_t)kGsumSlots * kGsumWords);
    FGS_GROW(s.sums, (size_t)kSortBlocks);
    return hipSuccess;
}

hipError_t ensure_chunks(ChunkList &c, size_t need) {
    need = (std::max<size_t>(need, 65536) + kChunkCapAlign - 1) / kChunkCapAlign * kChunkCapAlign;
    if (need <= c.cap && c.chunks) return hipSuccess;
    FGS_GROW(c.chunks, need);
    FGS_GROW(c.mask, need * (kChunkTiles / 32));
    FGS_GROW(c.big, need);
    c.cap = need;
    return hipSuccess;
}

void free_frame_buffers(FrameBuffers &b) {
    void **ps[] = {(void **)&b.gs, (void **)&b.conic, (void **)&b.rect, (void **)&b.count, (void **)&b.count8, (void **)&b.erec, (void **)&b.dkey,
                   (void **)&b.dk_b, (void **)&b.dv_a, (void **)&b.dv_b, (void **)&b.offsets, (void **)&b.seg_count, (void **)&b.gmap,
                   (void **)&b.ranges, (void **)&b.sranges,
                   (void **)&b.T, (void **)&b.last};
    for (void **p : ps) free_p(*p);
    if (b.pairs_owned) {
        free_p(*(void **)&b.tk_a);  // the block of all four
    }
    b = FrameBuffers{};
}

void free_sort_scratch(SortScratch &s) {
    free_p(*(void **)&s.rhist);
    free_p(*(void **)&s.gsum);
    free_p(*(void **)&s.sums);
}

void free_chunks(ChunkList &c) {
    free_p(*(void **)&c.chunks);
    free_p(*(void **)&c.mask);
    free_p(*(void **)&c.big);
    c.cap = 0;
}

fgs_status check_args(const fgs_scene *sc, const fgs_camera *cam, int32_t W, int32_t H, const fgs_options *opt,
                      std::string &err) {
    auto bad = [&](const char *m) {
        err = m;
        return FGS_ERR_INVALID_ARGUMENT;
    };
    if (!sc) return bad("scene is NULL");
    if (!cam) return bad("camera is NULL");
    if (sc->num_gaussians < 0 || sc->num_gaussians > 0x7fffffffLL) return bad("num_gaussians out of range [0, 2^31)");
    if (sc->plane_stride < sc->num_gaussians) return bad("plane_stride < num_gaussians");
    if (sc->sh_degree < 0 || sc->sh_degree > 3) return bad("sh_degree outside 0..3");
    if (sc->reserved != 0) return bad("scene.reserved must be 0");
    if (sc->num_gaussians > 0 && (!sc->means || !sc->log_scales || !sc->quats || !sc->opacity_logits || !sc->sh))
        return bad("a scene attribute pointer is NULL");
    if (W < 1 || W > 16384 || H < 1 || H > 16384) return bad("image size outside 1..16384");
    if (!finite_all(cam->R, 9) || !finite_all(cam->t, 3) || !finite_all(cam->eye, 3) || !std::isfinite(cam->fx) ||
        !std::isfinite(cam->fy) || !std::isfinite(cam->cx) || !std::isfinite(cam->cy) || !std::isfinite(cam->near_z))
        return bad("camera has a non-finite value");
    if (!(cam->fx > 0.0f) || !(cam->fy > 0.0f)) return bad("focal length <= 0");
    if (!(cam->near_z > 0.0f)) return bad("near_z <= 0");
    if (opt) {
        if (!(opt->alpha_min > 0.0f && opt->alpha_min < 1.0f)) return bad("alpha_min outside (0, 1)");
        if (!(opt->T_stop >= 0.0f && opt->T_stop < 1.0f)) return bad("T_stop outside [0, 1)");
        if (!(opt->alpha_max > 0.0f && opt->alpha_max < 1.0f)) return bad("alpha_max outside (0, 1)");
        if (!(opt->dilation >= 0.0f) || !std::isfinite(opt->dilation)) return bad("dilation must be finite and >= 0");
        if (!(opt->jac_clip > 0.0f) || !std::isfinite(opt->jac_clip)) return bad("jac_clip must be finite and > 0");
        if (!finite_all(opt->bg, 3)) return bad("background is not finite");
        if (opt->binning < 0 || opt->binning > 2) return bad("binning not in {0, 1, 2}");
    }
    return FGS_OK;
}

DevOptions to_dev(const fgs_options &o) {
    DevOptions d{};
    d.alpha_min = o.alpha_min;
    d.T_stop = o.T_stop;
    d.alpha_max = o.alpha_max;
    d.dilation = o.dilation;
    d.jac_clip = o.jac_clip;
    for (int i = 0; i < 3; ++i) d.bg[i] = o.bg[i];
    d.cap_3sigma = o.cap_3sigma;
    d.binning = o.binning;
    return d;
}

DevCamera to_dev(const fgs_camera &c) {
    DevCamera d{};
    memcpy(d.R, c.R, sizeof d.R);
    memcpy(d.t, c.t, sizeof d.t);
    memcpy(d.eye, c.eye, sizeof d.eye);
    d.fx = c.fx;
    d.fy = c.fy;
    d.cx = c.cx;
    d.cy = c.cy;
    d.near_z = c.near_z;
    return d;
}

DevCam64 to_dev64(const DevCamera &c, const DevOptions &o, int W, int H) {
    DevCam64 d{};
    for (int i = 0; i < 9; ++i) d.R[i] = c.R[i];
    for (int i = 0; i < 3; ++i) d.t[i] = c.t[i];
    d.fx = c.fx;
    d.fy = c.fy;
    d.limx = (double)o.jac_clip * ((0.5 * (double)W) / d.fx);
    d.limy = (double)o.jac_clip * ((0.5 * (double)H) / d.fy);
    return d;
}

DevCam64 to_dev64(const fgs_camera &c, const fgs_options &o, int W, int H) {
    return to_dev64(to_dev(c), to_dev(o), W, H);
}

DevScene to_dev(const fgs_scene &s) {
    DevScene d{};
    d.means = s.means;
    d.log_scales = s.log_scales;
    d.quats = s.quats;
    d.logits = s.opacity_logits;
    d.sh = s.sh;
    d.P = s.num_gaussians;
    d.stride = s.plane_stride;
    d.D = s.sh_degree;
    return d;
}

hipError_t build_prepared(const fgs_scene &sc, const fgs_options &op, PreparedBuffers &pb, hipStream_t s) {
    free_prepared(pb);
    const int64_t P = sc.num_gaussians;
    const int ncoef = 3 * (sc.sh_degree + 1) * (sc.sh_degree + 1);
    pb.P = P;
    pb.sh_stride = (ncoef + 3) / 4 * 4;
    const size_t n = (size_t)(P > 0 ? P : 1);
    hipError_t e;
    if ((e = hipMalloc((void **)&pb.pos_o, n * sizeof(float4))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&pb.cov, 2 * n * sizeof(float4))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&pb.sh, n * (size_t)pb.sh_stride * sizeof(float))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&pb.bnd, n * sizeof(float2))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&pb.orig, n * sizeof(uint32_t))) != hipSuccess) return e;
    if ((e = hipMalloc((void **)&pb.blk, 3 * (pb.batches() > 0 ? pb.batches() : 1) * sizeof(float4))) != hipSuccess)
        return e;
    // Slot order: the Gaussians sorted by the Morton code of their means
    // (stable, so equal codes keep index order), so that the candidates of a
    // frame's cull, which see one region of the scene, occupy few contiguous
    // runs of slots and their precompute is read line by line.
    const DevScene dsc = to_dev(sc);
    uint32_t *tmp = nullptr;  // keys a, keys b, values a, values b (n each), bounds (8)
    SortScratch ss;
    if ((e = hipMalloc((void **)&tmp, (4 * n + 8) * sizeof(uint32_t))) != hipSuccess) return e;
    if ((e = ensure_sort_scratch(ss)) != hipSuccess) {
        (void)hipFree(tmp);
        return e;
    }
    uint32_t *ka = tmp, *kb = tmp + n, *va = tmp + 2 * n, *vb = tmp + 3 * n, *bounds = tmp + 4 * n;
    const uint32_t P32 = (uint32_t)(P > 0 ? P : 0);
    launch_spatial_keys(dsc, bounds, ka, s);
    launch_fill_u32(ss.slot(0), 0u, (size_t)kGsumWords, s);
    launch_radix_pass(ka, nullptr, kb, vb, P32, nullptr, 0, 8, false, true, ss.rhist, ss.slot(0), ss.slot(1), s);
    launch_radix_pass(kb, vb, ka, va, P32, nullptr, 8, 8, false, true, ss.rhist, ss.slot(1), ss.slot(2), s);
    launch_radix_pass(ka, va, kb, vb, P32, nullptr, 16, 8, false, true, ss.rhist, ss.slot(2), ss.slot(3), s);
    launch_radix_pass(kb, vb, nullptr, va, P32, nullptr, 24, 8, false, false, ss.rhist, ss.slot(3), nullptr, s);
    launch_prepare(dsc, to_dev(op), va, pb.pos_o, pb.cov, pb.sh, pb.bnd, pb.orig, pb.sh_stride, s);
    launch_block_bounds(pb.pos_o, pb.bnd, P, pb.blk, s);
    e = hipGetLastError();
    // the temporary buffers are read by the work just enqueued
    const hipError_t e2 = hipStreamSynchronize(s);
    (void)hipFree(tmp);
    free_sort_scratch(ss);
    return e != hipSuccess ? e : e2;
}

void free_prepared(PreparedBuffers &pb) {
    free_p(*(void **)&pb.orig);
    free_p(*(void **)&pb.pos_o);
    free_p(*(void **)&pb.cov);
    free_p(*(void **)&pb.sh);
    free_p(*(void **)&pb.bnd);
    free_p(*(void **)&pb.blk);
    pb = PreparedBuffers{};
}

hipError_t SideStream::create() {
    hipError_t e = hipStreamCreateWithFlags(&side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&join, hipEventDisableTiming);
    return e;
}

void SideStream::destroy() {
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    if (side) (void)hipStreamDestroy(side);
    *this = SideStream{};
}

void enqueue_front(const DevScene &sc, const DevPrepared *pp, const DevCamera &cam, const DevOptions &op, int W,
                   int H, FrameBuffers &fb, ChunkList &ch, SortScratch &ss, FrameCounters *fc,
                   FrameCounters *host_fc, hipStream_t s, const SideStream &side, const StageMarks &mk,
                   hipEvent_t counters_ready, bool full) {
    const uint32_t chunk_cap = (uint32_t)std::min<size_t>(ch.cap, 0xffffffffu);
    // ---- stage 1: preprocess + exact tile count -------------------------------
    // (a prepared scene's cull clears the counters itself)
    if (!pp || sc.P <= 0) launch_fill_u32(reinterpret_cast<uint32_t *>(fc), 0u, sizeof(FrameCounters) / 4, s);
    mk.mark(0, s);
    // the candidate list of a prepared scene lives in dv_b until the depth sort
    // (a prepared scene's outputs are dense over the candidate list, with the
    // Gaussian of each list position in fb.gmap)
    // group-sum slots: depth passes 0-3, tile passes 4-7; each slot is cleared
    // by the kernel before its pass (the preprocess, the emission, or the
    // previous pass's downsweep)
    if (pp) launch_cull(sc, *pp, cam, op, W, H, fb.dv_b, fb.seg_count, fc, s);
    mk.mark(kMarkCulled, s);
    launch_preprocess(sc, pp, cam, to_dev64(cam, op, W, H), op, W, H, fb.gs, fb.conic, fb.rect, fb.count, fb.count8,
                      fb.erec, fb.dkey, fb.dv_b, fb.seg_count, fb.gmap, ch.chunks, chunk_cap, fc, ss.slot(0), full, s);
    enqueue_front_rest(pp != nullptr, (uint32_t)sc.P, op, W, H, fb, ch, ss, fc, host_fc, s, side, mk, counters_ready);
}

void enqueue_front_rest(bool dense, uint32_t P32, const DevOptions &op, int W, int H, FrameBuffers &fb, ChunkList &ch,
                        SortScratch &ss, FrameCounters *fc, FrameCounters *host_fc, hipStream_t s,
                        const SideStream &side, const StageMarks &mk, hipEvent_t counters_ready) {
    const uint32_t chunk_cap = (uint32_t)std::min<size_t>(ch.cap, 0xffffffffu);
    // the large rectangles' exact tests touch neither the depth keys nor the
    // sort scratch: they run beside the depth sort
    hipStream_t sb = s;
    if (side.side && hipEventRecord(side.fork, s) == hipSuccess &&
        hipStreamWaitEvent(side.side, side.fork, 0) == hipSuccess)
        sb = side.side;
    launch_big_count(W, H, op.binning, fb.gs, fb.conic, fb.erec, ch.chunks, chunk_cap, ch.mask, fb.count, fc, sb);
    const bool joined = sb == s || hipEventRecord(side.join, sb) == hipSuccess;
    if (!joined) (void)hipStreamSynchronize(sb);  // cannot order the streams by an event: wait here instead
    // ---- depth order of the visible Gaussians: 4 LSD passes over the depth
    // digits, hoisted before key duplication (the low half of the (tile |
    // depth) key is the same for every pair of a Gaussian) --------------------
    mk.mark(1, s);
    // (values: the output slots, i.e. list positions of a prepared scene's
    // candidates or Gaussian indices)
    launch_radix_pass(fb.dkey, nullptr, fb.dk_b, fb.dv_b, P32, dense ? &fc->ncand : nullptr, 0, 8, true, true, ss.rhist,
                      ss.slot(0), ss.slot(1), s);
    launch_radix_pass(fb.dk_b, fb.dv_b, fb.dkey, fb.dv_a, P32, &fc->visible, 8, 8, false, true, ss.rhist, ss.slot(1),
                      ss.slot(2), s);
    launch_radix_pass(fb.dkey, fb.dv_a, fb.dk_b, fb.dv_b, P32, &fc->visible, 16, 8, false, true, ss.rhist, ss.slot(2),
                      ss.slot(3), s);
    // (a prepared scene's frame keeps the sorted keys: its ties need them)
    launch_radix_pass(fb.dk_b, fb.dv_b, fb.dkey, fb.dv_a, P32, &fc->visible, 24, 8, false, dense, ss.rhist,
                      ss.slot(3), nullptr, s);
    // A prepared scene's list positions follow the precompute's spatial
    // order, so the stable sort left equal depths in that order: re-order each
    // run of equal depths by Gaussian index (the long-run list borrows the
    // offsets, which the scan writes next; dv_b is free after the last pass)
    if (dense) launch_depth_ties(fb.dkey, fb.dv_a, fb.gmap, P32, &fc->visible, fb.offsets, fc, fb.dv_b, s);
    mk.mark(2, s);
    // ---- stage 2a: scan of the super-tile entry counts in depth order --------------
    // (a large rectangle's entries follow from its rectangle: the scan does
    // not wait for its tests)
    launch_count_scan(fb.dv_a, fb.count8, fb.erec, P32, &fc->visible, fb.dk_b, ss.sums, fb.offsets, &fc->entries, s);
    // the pair count and the emission read what the large-rectangle tests wrote
    if (sb != s && joined && hipStreamWaitEvent(s, side.join, 0) != hipSuccess) (void)hipStreamSynchronize(sb);
    mk.mark(3, s);
    // the second half reads the counters on the device; only the host waits
    // for their copy, which therefore runs beside it when it can
    hipStream_t sc2 = s;
    if (counters_ready && side.side && hipEventRecord(side.fork, s) == hipSuccess &&
        hipStreamWaitEvent(side.side, side.fork, 0) == hipSuccess)
        sc2 = side.side;
    if (host_fc) (void)hipMemcpyAsync(host_fc, fc, sizeof(FrameCounters), hipMemcpyDeviceToHost, sc2);
    if (counters_ready) (void)hipEventRecord(counters_ready, sc2);
}

bool enqueue_back(int W, int H, const DevOptions &op, uint32_t P, FrameBuffers &fb, ChunkList &ch, SortScratch &ss,
                  FrameCounters *fc, float *rgb, float *T, uint32_t *last, unsigned long long *work, hipStream_t s,
                  const StageMarks &mk, int blend_variant) {
    const uint32_t nsuper = super_count(W, H);
    const uint32_t chunk_cap = (uint32_t)std::min<size_t>(ch.cap, 0xffffffffu);
    const uint32_t pair_cap = (uint32_t)std::min<size_t>(fb.capN, 0xffffffffu);
    // The values go to tv_b; the entries of both sort buffers and the
    // tile-list scratch fill the 12 capN bytes before it (tk_a, tk_b, tv_a:
    // one block), each array 128-byte aligned (ecap is a multiple of 64).
    const size_t ecap_z = std::min<size_t>(entry_capacity(fb.capN, W, H), 0xffffffc0u);
    const uint32_t ecap = (uint32_t)ecap_z;
    uint8_t *blk = reinterpret_cast<uint8_t *>(fb.tk_a);
    uint64_t *mask_a = reinterpret_cast<uint64_t *>(blk), *mask_b = mask_a + ecap;
    uint32_t *gidx_a = reinterpret_cast<uint32_t *>(mask_b + ecap), *gidx_b = gidx_a + ecap;
    uint16_t *skey_a = reinterpret_cast<uint16_t *>(gidx_b + ecap), *skey_b = skey_a + ecap;
    uint32_t *lscratch = reinterpret_cast<uint32_t *>(skey_b + ecap);
    const bool fits = ecap_z > 0;
    // ---- stage 2b: key emission ----------------------------------------------------
    int shifts[4] = {0, 0, 0, 0}, widths[4] = {0, 0, 0, 0};
    const int npass = plan_tile_passes(ceil_log2(nsuper), shifts, widths);
    // the emission also sets every super-tile's range empty when a sort pass
    // records the ranges (one super-tile: no pass, its range holds every entry)
    static_assert(kGsumSlots >= 4 + 2, "four depth and up to two super-tile passes (ids < 65536)");
    launch_super_emit(W, H, fb.dv_a, P, &fc->visible, fb.offsets, fb.erec, (uint32_t)std::min<size_t>(fb.capP, 0xffffffffu),
                      ch.chunks, ch.big, ch.mask, chunk_cap, fc, skey_a, gidx_a, mask_a, ecap,
                      npass > 0 ? fb.sranges : nullptr, nsuper, npass > 0 ? ss.slot(4) : nullptr, s);
    mk.mark(4, s);
    // ---- stage 3: stable LSD sort of the entries by super-tile ----------------------
    uint16_t *ki = skey_a, *ko = skey_b;
    uint32_t *vi = gidx_a, *vo = gidx_b;
    uint64_t *mi = mask_a, *mo = mask_b;
    // The last pass records where each super-tile's run starts and ends
    // instead of writing the sorted keys (an empty super-tile keeps start > end).
    for (int p = 0; p < npass; ++p) {
        const bool last_pass = p + 1 == npass;
        launch_radix_pass(ki, vi, ko, vo, ecap, &fc->entries, shifts[p], widths[p], false, !last_pass, ss.rhist,
                          ss.slot(4 + p), last_pass ? nullptr : ss.slot(5 + p), s, last_pass ? fb.sranges : nullptr,
                          nsuper, 2, mi, mo, npass == 1);
        std::swap(ki, ko);
        std::swap(vi, vo);
        std::swap(mi, mo);
    }
    if (npass == 0) launch_single_range(fb.sranges, ecap, &fc->entries, s);
    mk.mark(5, s);
    // ---- per-tile lists and ranges (the sorted pairs) -----------------------------
    if (fits)
        launch_tile_lists(W, H, fb.sranges, vi, mi, ecap, lscratch, fb.ranges, fb.tv_b, pair_cap, s);
    else  // too small for the list scratch: empty ranges (the host renders the frame again)
        launch_fill_u32(reinterpret_cast<uint32_t *>(fb.ranges), 0u,
                        (size_t)2 * (size_t)((W + kTile - 1) / kTile) * (size_t)((H + kTile - 1) / kTile), s);
    mk.mark(6, s);
    // ---- stage 4: blend -------------------------------------------------------------
    // (the variant's buffer loads take 32-bit byte offsets)
    const bool fits32 = fb.capN <= 0x7fffffffu / 4u && fb.capP <= 0x7fffffffu / sizeof(GaussState);
    launch_blend(fb.gs, fb.tv_b, fb.ranges, W, H, op, rgb, T, last, work, fits32 ? blend_variant : 0,
                 (uint32_t)fb.capN, (uint32_t)fb.capP, s);
    mk.mark(7, s);
    return false;
}

}  // namespace fgs
