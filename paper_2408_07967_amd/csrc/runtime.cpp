// Host runtime behind the C ABI of include/fgs.h: argument validation,
// context and scratch-arena management, the plain per-request renderer, the
// backward, frame introspection and instrumentation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fgs.h"
#include "fgs_internal.hpp"
#include "pipeline.hpp"

using namespace fgs;

namespace {
thread_local std::string g_null_ctx_error;
}  // namespace


void fgs::set_error_without_context(const char *msg) { g_null_ctx_error = msg; }

struct fgs_frame {
    FrameBuffers fb;
    int W = 0, H = 0;
    int64_t P = 0;
    uint32_t visible = 0, pairs = 0;
    bool tiles_in_a = true;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;  // recorded on `stream` after the forward's last kernel
    fgs_camera cam{};
    fgs_options opt{};
    fgs_stats stats{};
    // rendered from a prepared scene: per-Gaussian buffers are indexed by
    // candidate list position (ncand of them; fb.gmap gives the Gaussian)
    bool dense = false;
    uint32_t ncand = 0;
};

struct fgs_prepared {
    fgs_scene scene{};
    fgs_options opt{};
    PreparedBuffers pb;
};

struct fgs_context {
    int device = 0;
    std::string err;
    FrameBuffers fb;
    std::vector<FrameBuffers> pool;
    std::vector<fgs_frame *> frames;
    FrameCounters *fc_dev = nullptr;
    FrameCounters *fc_host = nullptr;
    hipEvent_t front_done = nullptr;  // the front half's counters are on the host
    SideStream side;                  // independent work of a frame runs beside the frame's stream
    SortScratch ss;
    ChunkList ch;
    // instrumentation
    int instr = 0;
    int blend_variant = 0;  // FGS_BLEND_*
    hipEvent_t ev[2][kStageMarks] = {};
    int ev_pending = -1;  // event set of the last instrumented frame not yet folded in
    int ev_next = 0;
    fgs_timings acc{};
    unsigned long long *work_dev = nullptr;
    // backward: per-Gaussian sums of the blend adjoint, 9 planes of gacc_stride
    float *gacc = nullptr;
    size_t gacc_stride = 0;
    std::vector<fgs_prepared *> prepared;
    // multi-camera batches: the buffers of each camera of a batch
    struct BatchCam {
        FrameBuffers fb;
        ChunkList ch;
        SortScratch ss;
    };
    std::vector<BatchCam> batch;
    FrameCounters *bfc_dev = nullptr, *bfc_host = nullptr;  // kMaxCams each
    unsigned char *noalloc_base = nullptr;  // this device's fixed scratch (fgs_render_noalloc)
};

namespace {

fgs_status fail(fgs_context *ctx, fgs_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (ctx)
        ctx->err = buf;
    else
        g_null_ctx_error = buf;
    return s;
}

fgs_status hip_fail(fgs_context *ctx, hipError_t e, const char *what) {
    return fail(ctx, e == hipErrorOutOfMemory ? FGS_ERR_OUT_OF_MEMORY : FGS_ERR_DEVICE, "%s: %s", what,
                hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                     \
    do {                                                       \
        hipError_t e_ = (expr);                                \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

fgs_status validate(fgs_context *ctx, const fgs_scene *sc, const fgs_camera *cam, int32_t W, int32_t H,
                    const fgs_options *opt) {
    std::string m;
    const fgs_status s = check_args(sc, cam, W, H, opt, m);
    if (s != FGS_OK) return fail(ctx, s, "%s", m.c_str());
    return FGS_OK;
}

// Per-Gaussian records as fgs_frame_download documents them (16 floats): the
// device keeps the blend's state (GaussState, 12 floats) and the canonical
// conic (4 floats) in two arrays; the host field lists the canonical conic
// first.  Builds n host records from n device entries of each array.
constexpr size_t kHostGaussFloats = 16;
void gauss_to_host(const float *gs, const float *conic, size_t n, float *dst) {
    static_assert(sizeof(GaussState) == 12 * sizeof(float), "12 floats of blend state");
    // host column j takes column from[j] of (state | conic)
    static const int from[16] = {0, 1, 12, 13, 14, 5, 6, 7, 8, 9, 10, 11, 2, 3, 4, 15};
    for (size_t i = 0; i < n; ++i, dst += kHostGaussFloats) {
        float t[16];
        memcpy(t, gs + 12 * i, 12 * sizeof(float));
        memcpy(t + 12, conic + 4 * i, 4 * sizeof(float));
        for (int j = 0; j < 16; ++j) dst[j] = t[from[j]];
    }
}

// Add the stage times of a completed instrumented frame to the sums.
void fold_events(fgs_context *ctx) {
    if (ctx->ev_pending < 0) return;
    hipEvent_t *e = ctx->ev[ctx->ev_pending];
    float ms[7] = {0, 0, 0, 0, 0, 0, 0}, cull = 0.0f;
    for (int i = 0; i < 7; ++i)
        if (hipEventElapsedTime(&ms[i], e[i == 0 ? kMarkCulled : i], e[i + 1]) != hipSuccess) ms[i] = 0.0f;
    if (hipEventElapsedTime(&cull, e[0], e[kMarkCulled]) != hipSuccess) cull = 0.0f;
    ctx->acc.frames += 1;
    ctx->acc.ms_cull += cull;
    ctx->acc.ms_preprocess += ms[0];
    ctx->acc.ms_depth_sort += ms[1];
    ctx->acc.ms_scan += ms[2];
    ctx->acc.ms_emit += ms[3];
    ctx->acc.ms_super_sort += ms[4];
    ctx->acc.ms_tile_lists += ms[5];
    ctx->acc.ms_blend += ms[6];
    ctx->ev_pending = -1;
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================

extern "C" {

const char *fgs_status_string(fgs_status s) {
    // a C caller may pass any int; read it as one (a C++ enum holding a value
    // outside its enumerators' range is undefined)
    int v = 0;
    static_assert(sizeof v == sizeof s, "fgs_status is int-sized");
    memcpy(&v, &s, sizeof v);
    switch (v) {
    case FGS_OK: return "ok";
    case FGS_ERR_INVALID_ARGUMENT: return "invalid argument";
    case FGS_ERR_OUT_OF_MEMORY: return "out of device memory";
    case FGS_ERR_CAPACITY: return "capacity exceeded";
    case FGS_ERR_DEVICE: return "device error";
    case FGS_ERR_NOT_SUPPORTED: return "not supported";
    case FGS_ERR_INTERNAL: return "internal error";
    }
    return "unknown status";
}

const char *fgs_last_error(const fgs_context *ctx) {
    return ctx ? ctx->err.c_str() : g_null_ctx_error.c_str();
}

void fgs_default_options(fgs_options *o) {
    if (!o) return;
    o->alpha_min = 1.0f / 255.0f;
    o->T_stop = 1e-4f;
    o->alpha_max = 0.99f;
    o->dilation = 0.3f;
    o->jac_clip = 1.3f;
    o->bg[0] = o->bg[1] = o->bg[2] = 0.0f;
    o->cap_3sigma = 1;
    o->binning = 0;
}

fgs_status fgs_validate(const fgs_scene *scene, const fgs_camera *cam, int32_t W, int32_t H,
                        const fgs_options *opt) {
    return validate(nullptr, scene, cam, W, H, opt);
}

fgs_status fgs_create(int device, fgs_context **out) {
    if (!out) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0)
        return fail(nullptr, FGS_ERR_DEVICE, "no HIP device available");
    if (device < 0 || device >= n) return fail(nullptr, FGS_ERR_DEVICE, "device %d of %d does not exist", device, n);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return fail(nullptr, FGS_ERR_DEVICE, "hipGetDeviceProperties failed");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(nullptr, FGS_ERR_DEVICE, "device %d is %s; this library is built for gfx950 only", device,
                    prop.gcnArchName);
    if (hipSetDevice(device) != hipSuccess) return fail(nullptr, FGS_ERR_DEVICE, "hipSetDevice failed");
    fgs_context *ctx = new fgs_context();
    ctx->device = device;
    if (hipMalloc((void **)&ctx->fc_dev, sizeof(FrameCounters)) != hipSuccess ||
        hipHostMalloc((void **)&ctx->fc_host, sizeof(FrameCounters), hipHostMallocDefault) != hipSuccess) {
        fgs_destroy(ctx);
        return fail(nullptr, FGS_ERR_OUT_OF_MEMORY, "cannot allocate frame counters");
    }
    if (hipEventCreateWithFlags(&ctx->front_done, hipEventDisableTiming) != hipSuccess ||
        ctx->side.create() != hipSuccess) {
        fgs_destroy(ctx);
        return fail(nullptr, FGS_ERR_DEVICE, "cannot create an event");
    }
    const hipError_t ne = noalloc_scratch(device, &ctx->noalloc_base);
    if (ne != hipSuccess) {
        fgs_destroy(ctx);
        return fail(nullptr, FGS_ERR_DEVICE, "cannot take the fixed scratch's device address: %s",
                    hipGetErrorString(ne));
    }
    *out = ctx;
    return FGS_OK;
}

void fgs_destroy(fgs_context *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    for (fgs_frame *f : ctx->frames) {
        free_frame_buffers(f->fb);
        if (f->done) (void)hipEventDestroy(f->done);
        delete f;
    }
    if (ctx->gacc) (void)hipFree(ctx->gacc);
    for (fgs_prepared *p : ctx->prepared) {
        free_prepared(p->pb);
        delete p;
    }
    for (FrameBuffers &b : ctx->pool) free_frame_buffers(b);
    free_frame_buffers(ctx->fb);
    for (auto &bc : ctx->batch) {
        free_frame_buffers(bc.fb);
        free_chunks(bc.ch);
        free_sort_scratch(bc.ss);
    }
    if (ctx->bfc_dev) (void)hipFree(ctx->bfc_dev);
    if (ctx->bfc_host) (void)hipHostFree(ctx->bfc_host);
    for (auto &set : ctx->ev)
        for (hipEvent_t &e : set)
            if (e) (void)hipEventDestroy(e);
    if (ctx->work_dev) (void)hipFree(ctx->work_dev);
    free_chunks(ctx->ch);
    free_sort_scratch(ctx->ss);
    if (ctx->fc_dev) (void)hipFree(ctx->fc_dev);
    if (ctx->fc_host) (void)hipHostFree(ctx->fc_host);
    if (ctx->front_done) (void)hipEventDestroy(ctx->front_done);
    ctx->side.destroy();
    delete ctx;
}

fgs_status fgs_reserve(fgs_context *ctx, int64_t max_gaussians, int64_t max_pairs, int32_t max_w, int32_t max_h) {
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "context is NULL");
    if (max_gaussians < 0 || max_pairs < 0 || max_w < 0 || max_h < 0 || max_w > 16384 || max_h > 16384)
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "negative or oversized reservation");
    if (max_gaussians > 0x7fffffffLL || max_pairs > 0xffffffffLL)
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "reservation beyond 32-bit indices");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, ensure_gauss(ctx->fb, (size_t)max_gaussians));
    HIP_TRY(ctx, ensure_pairs(ctx->fb, (size_t)max_pairs));
    const size_t tiles = (size_t)((max_w + kTile - 1) / kTile) * ((max_h + kTile - 1) / kTile);
    HIP_TRY(ctx, ensure_tiles(ctx->fb, tiles));
    HIP_TRY(ctx, ensure_chunks(ctx->ch, (size_t)max_gaussians / 8));
    HIP_TRY(ctx, ensure_sort_scratch(ctx->ss));
    return FGS_OK;
}

size_t fgs_scratch_bytes(const fgs_context *ctx) {
    if (!ctx) return 0;
    size_t b = ctx->fb.bytes() + sizeof(FrameCounters) + ctx->ch.bytes() + (ctx->ss.rhist ? SortScratch::bytes() : 0);
    b += 9 * ctx->gacc_stride * sizeof(float);
    for (const fgs_prepared *p : ctx->prepared) b += p->pb.bytes();
    for (const FrameBuffers &p : ctx->pool) b += p.bytes();
    for (const fgs_frame *f : ctx->frames) b += f->fb.bytes();
    for (const auto &bc : ctx->batch)
        b += bc.fb.bytes() + bc.ch.bytes() + (bc.ss.rhist ? SortScratch::bytes() : 0);
    if (ctx->bfc_dev) b += kMaxCams * sizeof(FrameCounters);
    return b;
}

}  // extern "C"

namespace {

// Planning only (fgs_plan): the front half runs, the pair count and the bytes
// a render needs are reported, nothing is blended.
struct PlanOut {
    int64_t *pairs;
    size_t *bytes;
};

fgs_status render_impl(fgs_context *ctx, const fgs_scene *scene, const fgs_prepared *prep, const fgs_camera *cam,
                       int32_t W, int32_t H, const fgs_options *opt_in, float *out_rgb, float *out_T,
                       uint32_t *out_last, fgs_frame **saved, fgs_stats *stats, void *stream_v,
                       const PlanOut *plan = nullptr) {
    if (saved) *saved = nullptr;
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "context is NULL");
    fgs_status st = validate(ctx, scene, cam, W, H, opt_in);
    if (st != FGS_OK) return st;
    if (!out_rgb && !plan) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "out_rgb is NULL");
    fgs_options opt;
    if (opt_in)
        opt = *opt_in;
    else
        fgs_default_options(&opt);
    if (prep && (opt.alpha_min != prep->opt.alpha_min || opt.cap_3sigma != prep->opt.cap_3sigma))
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "alpha_min / cap_3sigma differ from the scene's preparation");
    ctx->err.clear();
    hipStream_t s = (hipStream_t)stream_v;
    HIP_TRY(ctx, hipSetDevice(ctx->device));

    FrameBuffers &fb = ctx->fb;
    const int64_t P = scene->num_gaussians;
    const int tiles_x = (W + kTile - 1) / kTile, tiles_y = (H + kTile - 1) / kTile;
    const uint32_t ntiles = (uint32_t)tiles_x * (uint32_t)tiles_y;
    const size_t npix = (size_t)W * H;
    HIP_TRY(ctx, ensure_gauss(fb, (size_t)P));
    HIP_TRY(ctx, ensure_tiles(fb, ntiles));
    HIP_TRY(ctx, ensure_sort_scratch(ctx->ss));
    if (saved) HIP_TRY(ctx, ensure_pixels(fb, npix));
    HIP_TRY(ctx, ensure_chunks(ctx->ch, (size_t)P / 8));

    const DevScene dsc = to_dev(*scene);
    const DevCamera dcam = to_dev(*cam);
    const DevOptions dop = to_dev(opt);
    const bool timed = (ctx->instr & FGS_INSTR_STAGE_TIMES) != 0;
    const int es = ctx->ev_next;
    StageMarks mk;
    if (timed) mk.ev = ctx->ev[es];

    float *Tdst = saved ? fb.T : out_T;
    uint32_t *Ldst = saved ? fb.last : out_last;
    unsigned long long *work = (ctx->instr & FGS_INSTR_WORK) ? ctx->work_dev : nullptr;
    uint32_t V = 0, N = 0, big = 0, ncand = 0;
    size_t Ncap = 0;  // pair-array capacity the frame needs
    uint32_t E = 0;   // super-tile entries
    bool tiles_in_a = true;
    size_t spec_cap = 0;  // pair capacity of a second half already enqueued (0: none)
    for (int attempt = 0;; ++attempt) {
        const DevPrepared pdev = prep ? prep->pb.dev() : DevPrepared{};
        enqueue_front(dsc, prep ? &pdev : nullptr, dcam, dop, W, H, fb, ctx->ch, ctx->ss, ctx->fc_dev, ctx->fc_host,
                      s, ctx->side, mk, ctx->front_done, saved != nullptr);
        HIP_TRY(ctx, hipGetLastError());
        // The second half reads every count on the device and never writes
        // beyond the pair buffers, so it is enqueued at once with the buffers
        // at hand; the GPU goes on while the host reads the pair count.  If
        // the frame has more pairs than they hold, it runs again below.
        spec_cap = 0;
        if (!plan && !work && fb.capN > 0) {
            tiles_in_a = enqueue_back(W, H, dop, (uint32_t)P, fb, ctx->ch, ctx->ss, ctx->fc_dev, out_rgb, Tdst, Ldst,
                                      nullptr, s, mk, ctx->blend_variant);
            HIP_TRY(ctx, hipGetLastError());
            spec_cap = fb.capN;
        }
        // wait for the counters by polling (the first half takes about a
        // millisecond at 4K, where a blocking wait's wake-up would add a
        // large share of that)
        hipError_t q;
        while ((q = hipEventQuery(ctx->front_done)) == hipErrorNotReady) {
        }
        HIP_TRY(ctx, q);
        fold_events(ctx);  // the previous instrumented frame is complete after the wait
        if (ctx->fc_host->error & kErrChunkOverflow) {
            // the large-Gaussian chunk list was too small: size it exactly and
            // render the frame again (a second half already enqueued skipped
            // the large rectangles; it is redone)
            if (attempt > 0) return fail(ctx, FGS_ERR_INTERNAL, "chunk list overflow after resizing");
            if (spec_cap) HIP_TRY(ctx, hipStreamSynchronize(s));  // the list is in use
            HIP_TRY(ctx, ensure_chunks(ctx->ch, (size_t)ctx->fc_host->nchunks + (size_t)ctx->fc_host->nchunks / 8));
            continue;
        }
        V = ctx->fc_host->visible;
        N = ctx->fc_host->pairs;
        E = ctx->fc_host->entries;
        Ncap = pair_capacity_needed(N, E, W, H);
        big = ctx->fc_host->nchunks;
        ncand = prep ? ctx->fc_host->ncand : 0;
        break;
    }
    if (plan) {
        FrameBuffers need;
        need.capP = (size_t)P;
        need.capN = Ncap;
        need.capTiles = ntiles;
        ChunkList chunks_need;
        chunks_need.cap = std::max<size_t>((size_t)big + big / 8, 65536);
        if (plan->pairs) *plan->pairs = (int64_t)N;
        if (plan->bytes)
            *plan->bytes = need.bytes() + SortScratch::bytes() + chunks_need.bytes() + sizeof(FrameCounters);
        if (stats) {
            fgs_stats stt{};
            stt.visible = V;
            stt.pairs = N;
            stt.tiles_x = tiles_x;
            stt.tiles_y = tiles_y;
            stt.big_chunks = (int32_t)big;
            stt.candidates = prep ? (int64_t)ncand : (int64_t)P;
            stt.entries = E;
            stt.cull_batches = prep ? (int64_t)ctx->fc_host->cull_read : 0;
            *stats = stt;
        }
        return FGS_OK;
    }
    if (spec_cap == 0 || Ncap > spec_cap) {
        // no second half yet, or it ran out of pair buffer: grow the buffers
        // (after it has finished with them) and enqueue it again
        if (spec_cap) HIP_TRY(ctx, hipStreamSynchronize(s));
        HIP_TRY(ctx, ensure_pairs(fb, Ncap));
        tiles_in_a = enqueue_back(W, H, dop, (uint32_t)P, fb, ctx->ch, ctx->ss, ctx->fc_dev, out_rgb, Tdst, Ldst,
                                  work, s, mk, ctx->blend_variant);
    }
    HIP_TRY(ctx, hipGetLastError());
    if (timed) {
        ctx->ev_pending = es;
        ctx->ev_next = es ^ 1;
    }
    if (saved) {
        if (out_T) HIP_TRY(ctx, hipMemcpyAsync(out_T, fb.T, npix * sizeof(float), hipMemcpyDeviceToDevice, s));
        if (out_last)
            HIP_TRY(ctx, hipMemcpyAsync(out_last, fb.last, npix * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
    }

    fgs_stats stt{};
    stt.visible = V;
    stt.pairs = N;
    stt.tiles_x = tiles_x;
    stt.tiles_y = tiles_y;
    stt.big_chunks = (int32_t)big;
    stt.candidates = prep ? (int64_t)ncand : (int64_t)P;
    stt.entries = E;
    stt.cull_batches = prep ? (int64_t)ctx->fc_host->cull_read : 0;
    stt.sort_passes = 4 + super_sort_passes(W, H);
    if (stats) *stats = stt;

    if (saved) {
        fgs_frame *f = new fgs_frame();
        f->fb = fb;
        f->W = W;
        f->H = H;
        f->P = P;
        f->visible = V;
        f->pairs = N;
        f->dense = prep != nullptr;
        f->ncand = ncand;
        f->tiles_in_a = tiles_in_a;
        f->stream = s;
        f->stats = stt;
        f->cam = *cam;
        f->opt = opt;
        if (hipEventCreateWithFlags(&f->done, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(f->done, s) != hipSuccess) {
            if (f->done) (void)hipEventDestroy(f->done);
            delete f;
            return fail(ctx, FGS_ERR_DEVICE, "cannot record the saved frame's completion event");
        }
        ctx->frames.push_back(f);
        // the context continues with pooled or fresh buffers
        if (!ctx->pool.empty()) {
            ctx->fb = ctx->pool.back();
            ctx->pool.pop_back();
        } else {
            ctx->fb = FrameBuffers{};
        }
        *saved = f;
    }
    return FGS_OK;
}

}  // namespace

extern "C" {

fgs_status fgs_render(fgs_context *ctx, const fgs_scene *scene, const fgs_camera *cam, int32_t W, int32_t H,
                      const fgs_options *opt, float *out_rgb, float *out_T, uint32_t *out_last, fgs_frame **saved,
                      fgs_stats *stats, void *stream) {
    return render_impl(ctx, scene, nullptr, cam, W, H, opt, out_rgb, out_T, out_last, saved, stats, stream);
}

fgs_status fgs_plan(fgs_context *ctx, const fgs_scene *scene, const fgs_camera *cam, int32_t W, int32_t H,
                    const fgs_options *opt, int64_t *pairs_out, size_t *bytes_out, void *stream) {
    if (pairs_out) *pairs_out = 0;
    if (bytes_out) *bytes_out = 0;
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "context is NULL");
    if (!pairs_out && !bytes_out) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "pairs_out and bytes_out are NULL");
    const PlanOut plan{pairs_out, bytes_out};
    return render_impl(ctx, scene, nullptr, cam, W, H, opt, nullptr, nullptr, nullptr, nullptr, nullptr, stream,
                       &plan);
}

}  // extern "C"

namespace {

// Bump carving of the fixed scratch: 256-byte aligned pieces, in order.
struct Carve {
    unsigned char *base;
    size_t size, used = 0;
    bool overflow = false;
    template <class T>
    T *take(size_t n) {
        const size_t off = (used + 255) & ~size_t(255);
        const size_t b = n * sizeof(T);
        if (off > size || b > size - off) {
            overflow = true;
            return nullptr;
        }
        used = off + b;
        return reinterpret_cast<T *>(base + off);
    }
};

// One frame's buffers in the fixed scratch: counters, sort scratch, tile
// ranges, the per-Gaussian arrays for P, the chunk list, then four pair
// arrays sharing what is left.  False if the fixed part does not fit.
bool carve_noalloc(unsigned char *base, size_t P, size_t ntiles, FrameBuffers &fb, SortScratch &ss, ChunkList &ch,
                   FrameCounters *&fc, size_t &fixed_bytes) {
    Carve c{base, FGS_NOALLOC_SCRATCH_BYTES};
    fb = FrameBuffers{};
    fc = c.take<FrameCounters>(1);
    ss.rhist = c.take<uint32_t>((size_t)kSortBlocks * kRadixMax);
    ss.gsum = c.take<uint32_t>((size_t)kGsumSlots * kGsumWords);
    ss.sums = c.take<uint32_t>((size_t)kSortBlocks);
    fb.ranges = c.take<uint2>(ntiles);
    fb.sranges = c.take<uint2>(ntiles);
    fb.capTiles = ntiles;
    const size_t capP = std::max<size_t>(P, 1);
    fb.gs = c.take<GaussState>(capP);
    fb.conic = c.take<float4>(capP);
    fb.rect = c.take<uint4>(capP);
    fb.count = c.take<uint32_t>(capP);
    fb.count8 = c.take<uint8_t>(capP);
    fb.erec = c.take<uint4>(capP);
    fb.dkey = c.take<uint32_t>(capP);
    fb.dk_b = c.take<uint32_t>(capP);
    fb.dv_a = c.take<uint32_t>(capP);
    fb.dv_b = c.take<uint32_t>(capP);
    fb.offsets = c.take<uint32_t>(capP + 1);
    fb.seg_count = c.take<uint32_t>(2 * kCullBlocks);
    fb.gmap = c.take<uint32_t>(capP);
    fb.capP = capP;
    ch.cap = (std::max<size_t>(P / 8, 8192) + kChunkCapAlign - 1) / kChunkCapAlign * kChunkCapAlign;
    ch.chunks = c.take<uint2>(ch.cap);
    ch.mask = c.take<uint32_t>(ch.cap * (kChunkTiles / 32));
    ch.big = c.take<uint2>(ch.cap);
    fixed_bytes = c.used;
    if (c.overflow) return false;
    // the rest: the four pair arrays of equal capacity, one block
    const size_t rest = FGS_NOALLOC_SCRATCH_BYTES - ((c.used + 255) & ~size_t(255));
    const size_t capN = rest / (4 * sizeof(uint32_t)) / 64 * 64;
    if (capN == 0) return false;
    fb.tk_a = c.take<uint32_t>(4 * capN);
    fb.tk_b = fb.tk_a + capN;
    fb.tv_a = fb.tk_a + 2 * capN;
    fb.tv_b = fb.tk_a + 3 * capN;
    fb.capN = capN;
    fb.pairs_owned = false;
    return !c.overflow;
}

}  // namespace

extern "C" {

fgs_status fgs_render_noalloc(fgs_context *ctx, const fgs_scene *scene, const fgs_camera *cam, int32_t W,
                              int32_t H, const fgs_options *opt_in, float *out_rgb, float *out_T, uint32_t *out_last,
                              fgs_stats *stats, void *stream_v) {
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "context is NULL");
    fgs_status st = validate(ctx, scene, cam, W, H, opt_in);
    if (st != FGS_OK) return st;
    if (!out_rgb) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "out_rgb is NULL");
    if (!ctx->noalloc_base) return fail(ctx, FGS_ERR_DEVICE, "the fixed scratch has no device address");
    fgs_options opt;
    if (opt_in)
        opt = *opt_in;
    else
        fgs_default_options(&opt);
    const int64_t P = scene->num_gaussians;
    const int tiles_x = (W + kTile - 1) / kTile, tiles_y = (H + kTile - 1) / kTile;
    const size_t ntiles = (size_t)tiles_x * (size_t)tiles_y;
    FrameBuffers fb;
    SortScratch ss;
    ChunkList ch;
    FrameCounters *fc = nullptr;
    size_t fixed = 0;
    if (!carve_noalloc(ctx->noalloc_base, (size_t)P, ntiles, fb, ss, ch, fc, fixed))
        return fail(ctx, FGS_ERR_CAPACITY,
                    "%lld Gaussians at %dx%d need %zu bytes of per-Gaussian, tile, sort and chunk buffers "
                    "plus pair space; the fixed scratch holds %zu",
                    (long long)P, W, H, fixed, (size_t)FGS_NOALLOC_SCRATCH_BYTES);
    ctx->err.clear();
    hipStream_t s = (hipStream_t)stream_v;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const DevScene dsc = to_dev(*scene);
    const DevCamera dcam = to_dev(*cam);
    const DevOptions dop = to_dev(opt);
    const StageMarks mk;  // no stage events
    enqueue_front(dsc, nullptr, dcam, dop, W, H, fb, ch, ss, fc, ctx->fc_host, s, ctx->side, mk, ctx->front_done);
    HIP_TRY(ctx, hipGetLastError());
    // the second half reads the pair count on the device and stays within the
    // pair arrays, so it goes right behind the first
    enqueue_back(W, H, dop, (uint32_t)P, fb, ch, ss, fc, out_rgb, out_T, out_last, nullptr, s, mk,
                 ctx->blend_variant);
    HIP_TRY(ctx, hipGetLastError());
    hipError_t q;
    while ((q = hipEventQuery(ctx->front_done)) == hipErrorNotReady) {
    }
    HIP_TRY(ctx, q);
    const FrameCounters h = *ctx->fc_host;
    if (stats) {
        fgs_stats stt{};
        stt.visible = h.visible;
        stt.pairs = h.pairs;
        stt.tiles_x = tiles_x;
        stt.tiles_y = tiles_y;
        stt.big_chunks = (int32_t)h.nchunks;
        stt.candidates = P;
        stt.entries = h.entries;
        stt.sort_passes = 4 + super_sort_passes(W, H);
        *stats = stt;
    }
    if (h.error & kErrChunkOverflow)
        return fail(ctx, FGS_ERR_CAPACITY, "the frame needs %u large-rectangle chunks; the fixed scratch holds %zu",
                    h.nchunks, ch.cap);
    const size_t need = pair_capacity_needed(h.pairs, h.entries, W, H);
    if (need > fb.capN)
        return fail(ctx, FGS_ERR_CAPACITY, "the frame has %u pairs and %u super-tile entries, which need pair "
                    "arrays of %zu; the fixed scratch holds %zu beside its %zu bytes of per-Gaussian, tile, sort and "
                    "chunk buffers",
                    h.pairs, h.entries, need, fb.capN, fixed);
    return FGS_OK;
}

fgs_status fgs_prepare_scene(fgs_context *ctx, const fgs_scene *scene, const fgs_options *opt_in,
                             fgs_prepared **out, void *stream) {
    if (out) *out = nullptr;
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "context is NULL");
    if (!out) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "out is NULL");
    fgs_camera probe{};
    for (int i = 0; i < 3; ++i) probe.R[4 * i] = 1.0f;
    probe.fx = probe.fy = 1.0f;
    probe.near_z = 0.2f;
    fgs_status st = validate(ctx, scene, &probe, 1, 1, opt_in);
    if (st != FGS_OK) return st;
    fgs_options opt;
    if (opt_in)
        opt = *opt_in;
    else
        fgs_default_options(&opt);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    fgs_prepared *p = new fgs_prepared();
    p->scene = *scene;
    p->opt = opt;
    const hipError_t e = build_prepared(*scene, opt, p->pb, (hipStream_t)stream);
    if (e != hipSuccess) {
        free_prepared(p->pb);
        delete p;
        return hip_fail(ctx, e, "building the scene's precompute");
    }
    ctx->prepared.push_back(p);
    *out = p;
    return FGS_OK;
}

fgs_status fgs_prepared_release(fgs_context *ctx, fgs_prepared *p) {
    if (!p) return FGS_OK;
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "context is NULL");
    for (size_t i = 0; i < ctx->prepared.size(); ++i) {
        if (ctx->prepared[i] == p) {
            ctx->prepared.erase(ctx->prepared.begin() + (long)i);
            (void)hipSetDevice(ctx->device);
            (void)hipDeviceSynchronize();  // frames may still read it
            free_prepared(p->pb);
            delete p;
            return FGS_OK;
        }
    }
    return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "prepared scene does not belong to this context");
}

fgs_status fgs_render_prepared(fgs_context *ctx, const fgs_prepared *p, const fgs_camera *cam, int32_t W, int32_t H,
                               const fgs_options *opt, float *out_rgb, float *out_T, uint32_t *out_last,
                               fgs_frame **saved, fgs_stats *stats, void *stream) {
    if (saved) *saved = nullptr;
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "context is NULL");
    bool owned = false;
    for (const fgs_prepared *q : ctx->prepared) owned |= (q == p);
    if (!p || !owned) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "prepared scene is NULL or not of this context");
    return render_impl(ctx, &p->scene, p, cam, W, H, opt, out_rgb, out_T, out_last, saved, stats, stream);
}

static_assert(kMaxCams == FGS_MAX_BATCH_CAMERAS, "batch size limit of the ABI");

fgs_status fgs_render_prepared_batch(fgs_context *ctx, const fgs_prepared *p, const fgs_camera *cams, int32_t ncams,
                                     int32_t W, int32_t H, const fgs_options *opt_in, float *const *out_rgb,
                                     float *const *out_T, uint32_t *const *out_last, fgs_stats *stats, void *stream_v) {
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "context is NULL");
    bool owned = false;
    for (const fgs_prepared *q : ctx->prepared) owned |= (q == p);
    if (!p || !owned) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "prepared scene is NULL or not of this context");
    if (!cams || ncams < 1 || ncams > kMaxCams)
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "ncams must be 1..%d with cams given", kMaxCams);
    if (!out_rgb) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "out_rgb is NULL");
    for (int c = 0; c < ncams; ++c) {
        fgs_status st = validate(ctx, &p->scene, &cams[c], W, H, opt_in);
        if (st != FGS_OK) return st;
        if (!out_rgb[c]) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "out_rgb[%d] is NULL", c);
    }
    fgs_options opt;
    if (opt_in)
        opt = *opt_in;
    else
        fgs_default_options(&opt);
    if (opt.alpha_min != p->opt.alpha_min || opt.cap_3sigma != p->opt.cap_3sigma)
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "alpha_min / cap_3sigma differ from the scene's preparation");
    ctx->err.clear();
    hipStream_t s = (hipStream_t)stream_v;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const int64_t P = p->scene.num_gaussians;
    const int tiles_x = (W + kTile - 1) / kTile, tiles_y = (H + kTile - 1) / kTile;
    const uint32_t ntiles = (uint32_t)tiles_x * (uint32_t)tiles_y;
    if (!ctx->bfc_dev) HIP_TRY(ctx, hipMalloc((void **)&ctx->bfc_dev, kMaxCams * sizeof(FrameCounters)));
    if (!ctx->bfc_host)
        HIP_TRY(ctx, hipHostMalloc((void **)&ctx->bfc_host, kMaxCams * sizeof(FrameCounters), hipHostMallocDefault));
    if (ctx->batch.size() < (size_t)ncams) ctx->batch.resize(ncams);
    for (int c = 0; c < ncams; ++c) {
        auto &bc = ctx->batch[c];
        HIP_TRY(ctx, ensure_gauss(bc.fb, (size_t)P));
        HIP_TRY(ctx, ensure_tiles(bc.fb, ntiles));
        HIP_TRY(ctx, ensure_sort_scratch(bc.ss));
        HIP_TRY(ctx, ensure_chunks(bc.ch, (size_t)P / 8));
    }
    const DevScene dsc = to_dev(p->scene);
    const DevOptions dop = to_dev(opt);
    const DevPrepared pdev = p->pb.dev();
    const StageMarks nomk;
    size_t spec_cap[kMaxCams] = {};  // pair capacity of a second half already enqueued (0: none)
    for (int attempt = 0;; ++attempt) {
        // one cull and one preprocess for every camera; the candidate list
        // and the Gaussian of each list position live in camera 0's buffers
        MultiOut mo{};
        mo.n = ncams;
        for (int c = 0; c < ncams; ++c) {
            auto &bc = ctx->batch[c];
            CamOut &o = mo.c[c];
            o.cam = to_dev(cams[c]);
            o.cam64 = to_dev64(cams[c], opt, W, H);
            o.W = W;
            o.H = H;
            o.gs = bc.fb.gs;
            o.conic = bc.fb.conic;
            o.rect = bc.fb.rect;
            o.count = bc.fb.count;
            o.count8 = bc.fb.count8;
            o.erec = bc.fb.erec;
            o.dkey = bc.fb.dkey;
            o.gmap = bc.fb.gmap;
            o.chunks = bc.ch.chunks;
            o.chunk_cap = (uint32_t)std::min<size_t>(bc.ch.cap, 0xffffffffu);
            o.fc = ctx->bfc_dev + c;
            o.gsum_clear = bc.ss.slot(0);
        }
        FrameBuffers &fb0 = ctx->batch[0].fb;
        if (P <= 0) launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->bfc_dev), 0u, kMaxCams * sizeof(FrameCounters) / 4, s);
        launch_preprocess_multi(dsc, pdev, mo, dop, fb0.dv_b, fb0.seg_count, fb0.gmap, s);
        // each camera's depth order and scan, then (beside the host's wait
        // for the counters) each camera's second half
        for (int c = 0; c < ncams; ++c) {
            auto &bc = ctx->batch[c];
            enqueue_front_rest(true, (uint32_t)P, dop, W, H, bc.fb, bc.ch, bc.ss, ctx->bfc_dev + c, ctx->bfc_host + c,
                               s, ctx->side, nomk);
        }
        HIP_TRY(ctx, hipEventRecord(ctx->front_done, s));
        // the cameras' second halves share no buffer: odd cameras run on the
        // side stream beside the even ones (one camera's sort passes, bound by
        // HBM, overlap another's blend, bound by the VALU), and s joins the
        // side stream at the end
        hipStream_t s2 = s;
        if (ncams > 1 && ctx->side.side && hipEventRecord(ctx->side.fork, s) == hipSuccess &&
            hipStreamWaitEvent(ctx->side.side, ctx->side.fork, 0) == hipSuccess)
            s2 = ctx->side.side;
        for (int c = 0; c < ncams; ++c) {
            auto &bc = ctx->batch[c];
            spec_cap[c] = 0;
            if (bc.fb.capN > 0) {
                (void)enqueue_back(W, H, dop, (uint32_t)P, bc.fb, bc.ch, bc.ss, ctx->bfc_dev + c, out_rgb[c],
                                   out_T ? out_T[c] : nullptr, out_last ? out_last[c] : nullptr, nullptr,
                                   (c & 1) ? s2 : s, nomk, ctx->blend_variant);
                spec_cap[c] = bc.fb.capN;
            }
        }
        if (s2 != s) {
            HIP_TRY(ctx, hipEventRecord(ctx->side.join, s2));
            HIP_TRY(ctx, hipStreamWaitEvent(s, ctx->side.join, 0));
        }
        HIP_TRY(ctx, hipGetLastError());
        hipError_t q;
        while ((q = hipEventQuery(ctx->front_done)) == hipErrorNotReady) {
        }
        HIP_TRY(ctx, q);
        bool overflow = false;
        for (int c = 0; c < ncams; ++c) overflow |= (ctx->bfc_host[c].error & kErrChunkOverflow) != 0;
        if (!overflow) break;
        // a chunk list was too small: size it exactly and render the batch again
        if (attempt > 0) return fail(ctx, FGS_ERR_INTERNAL, "chunk list overflow after resizing");
        HIP_TRY(ctx, hipStreamSynchronize(s));  // the lists are in use (s has joined the side stream)
        for (int c = 0; c < ncams; ++c) {
            const size_t need = ctx->bfc_host[c].nchunks;
            HIP_TRY(ctx, ensure_chunks(ctx->batch[c].ch, need + need / 8));
        }
    }
    bool synced = false;
    for (int c = 0; c < ncams; ++c) {
        auto &bc = ctx->batch[c];
        const uint32_t N = ctx->bfc_host[c].pairs;
        const size_t Ncap = pair_capacity_needed(N, ctx->bfc_host[c].entries, W, H);
        if (spec_cap[c] == 0 || Ncap > spec_cap[c]) {
            // no second half yet, or it ran out of pair buffer: grow the
            // buffers (once every enqueued half has finished: s has joined
            // the side stream) and enqueue it on s
            if (!synced) HIP_TRY(ctx, hipStreamSynchronize(s));
            synced = true;
            HIP_TRY(ctx, ensure_pairs(bc.fb, Ncap));
            (void)enqueue_back(W, H, dop, (uint32_t)P, bc.fb, bc.ch, bc.ss, ctx->bfc_dev + c, out_rgb[c],
                               out_T ? out_T[c] : nullptr, out_last ? out_last[c] : nullptr, nullptr, s, nomk,
                               ctx->blend_variant);
        }
        if (stats) {
            fgs_stats stt{};
            stt.visible = ctx->bfc_host[c].visible;
            stt.pairs = N;
            stt.tiles_x = tiles_x;
            stt.tiles_y = tiles_y;
            stt.big_chunks = (int32_t)ctx->bfc_host[c].nchunks;
            stt.candidates = (int64_t)ctx->bfc_host[c].ncand;
            stt.entries = ctx->bfc_host[c].entries;
            stt.cull_batches = ctx->bfc_host[c].cull_read;
            stt.sort_passes = 4 + super_sort_passes(W, H);
            stats[c] = stt;
        }
    }
    HIP_TRY(ctx, hipGetLastError());
    return FGS_OK;
}

fgs_status fgs_frame_release(fgs_context *ctx, fgs_frame *frame) {
    if (!frame) return FGS_OK;
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "context is NULL");
    for (size_t i = 0; i < ctx->frames.size(); ++i) {
        if (ctx->frames[i] == frame) {
            ctx->frames.erase(ctx->frames.begin() + (long)i);
            (void)hipSetDevice(ctx->device);
            (void)hipStreamSynchronize(frame->stream);
            if (frame->done) {
                // a backward may have used the frame on another stream
                (void)hipEventSynchronize(frame->done);
                (void)hipEventDestroy(frame->done);
            }
            if (ctx->pool.size() < 4)
                ctx->pool.push_back(frame->fb);
            else
                free_frame_buffers(frame->fb);
            delete frame;
            return FGS_OK;
        }
    }
    return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "frame does not belong to this context");
}

fgs_status fgs_frame_stats(const fgs_frame *frame, fgs_stats *stats) {
    if (!frame || !stats) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "NULL argument");
    *stats = frame->stats;
    return FGS_OK;
}

size_t fgs_frame_field_bytes(const fgs_frame *f, fgs_field field) {
    if (!f) return 0;
    const size_t tiles = (size_t)f->stats.tiles_x * f->stats.tiles_y;
    switch (field) {
    case FGS_FIELD_GAUSS: return (size_t)f->P * kHostGaussFloats * sizeof(float);
    case FGS_FIELD_RECT: return (size_t)f->P * sizeof(uint4);
    case FGS_FIELD_COUNT: return (size_t)f->P * sizeof(uint32_t);
    case FGS_FIELD_ORDER: return (size_t)f->visible * sizeof(uint32_t);
    case FGS_FIELD_TILES: return (size_t)f->pairs * sizeof(uint32_t);
    case FGS_FIELD_VALUES: return (size_t)f->pairs * sizeof(uint32_t);
    case FGS_FIELD_RANGES: return tiles * sizeof(uint2);
    }
    return 0;
}

fgs_status fgs_frame_download(fgs_context *ctx, const fgs_frame *f, fgs_field field, void *host_dst, size_t bytes) {
    if (!ctx || !f || (!host_dst && bytes)) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "NULL argument");
    const size_t need = fgs_frame_field_bytes(f, field);
    if (bytes != need) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "field needs %zu bytes, got %zu", need, bytes);
    if (!bytes) return FGS_OK;
    const void *src = nullptr;
    const FrameBuffers &b = f->fb;
    switch (field) {
    case FGS_FIELD_GAUSS: break;  // assembled from the state and conic arrays below
    case FGS_FIELD_RECT: src = b.rect; break;
    case FGS_FIELD_COUNT: src = b.count; break;
    case FGS_FIELD_ORDER: src = b.dv_a; break;
    case FGS_FIELD_TILES: break;  // expanded from the ranges below
    case FGS_FIELD_VALUES: src = f->tiles_in_a ? b.tv_a : b.tv_b; break;
    case FGS_FIELD_RANGES: src = b.ranges; break;
    default: return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "unknown field %d", (int)field);
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(f->stream));
    if (field == FGS_FIELD_TILES) {
        // the tile lists keep only their ranges, not the tile id of each
        // pair: the id of pair i is the tile whose range holds i
        const size_t tiles = (size_t)f->stats.tiles_x * f->stats.tiles_y;
        std::vector<uint2> rg(tiles);
        HIP_TRY(ctx, hipMemcpy(rg.data(), b.ranges, tiles * sizeof(uint2), hipMemcpyDeviceToHost));
        uint32_t *dst = static_cast<uint32_t *>(host_dst);
        for (size_t i = 0; i < f->pairs; ++i) dst[i] = 0xffffffffu;
        for (size_t t = 0; t < tiles; ++t)
            for (uint32_t i = rg[t].x; i < rg[t].y && i < f->pairs; ++i) dst[i] = (uint32_t)t;
        return FGS_OK;
    }
    if (field == FGS_FIELD_GAUSS) {
        // state and canonical conic of every output slot (Gaussian, or list
        // position of a prepared scene's frame), assembled into host records
        const size_t n = f->dense ? (size_t)f->ncand : (size_t)f->P;
        std::vector<float> gsh(n * 12), cnh(n * 4), rec(n * kHostGaussFloats);
        if (n) {
            HIP_TRY(ctx, hipMemcpy(gsh.data(), b.gs, n * sizeof(GaussState), hipMemcpyDeviceToHost));
            HIP_TRY(ctx, hipMemcpy(cnh.data(), b.conic, n * sizeof(float4), hipMemcpyDeviceToHost));
        }
        gauss_to_host(gsh.data(), cnh.data(), n, rec.data());
        if (!f->dense) {
            memcpy(host_dst, rec.data(), bytes);
            return FGS_OK;
        }
        std::vector<uint32_t> gm(n);
        if (n) HIP_TRY(ctx, hipMemcpy(gm.data(), b.gmap, n * sizeof(uint32_t), hipMemcpyDeviceToHost));
        const size_t esz = kHostGaussFloats * sizeof(float);
        uint8_t *d = static_cast<uint8_t *>(host_dst);
        memset(d, 0, bytes);
        for (size_t c = 0; c < n; ++c)
            if ((size_t)gm[c] * esz + esz <= bytes) memcpy(d + (size_t)gm[c] * esz, rec.data() + c * kHostGaussFloats, esz);
        return FGS_OK;
    }
    if (f->dense && (field == FGS_FIELD_RECT || field == FGS_FIELD_COUNT ||
                     field == FGS_FIELD_ORDER || field == FGS_FIELD_VALUES)) {
        // a prepared scene's frame holds per-Gaussian data by candidate list
        // position: map positions to Gaussian indices
        std::vector<uint32_t> gm(f->ncand);
        if (f->ncand) HIP_TRY(ctx, hipMemcpy(gm.data(), b.gmap, f->ncand * sizeof(uint32_t), hipMemcpyDeviceToHost));
        if (field == FGS_FIELD_ORDER || field == FGS_FIELD_VALUES) {
            HIP_TRY(ctx, hipMemcpy(host_dst, src, bytes, hipMemcpyDeviceToHost));
            uint32_t *d = static_cast<uint32_t *>(host_dst);
            for (size_t i = 0; i < bytes / sizeof(uint32_t); ++i) d[i] = d[i] < f->ncand ? gm[d[i]] : 0xffffffffu;
            return FGS_OK;
        }
        const size_t esz = field == FGS_FIELD_RECT ? sizeof(uint4) : sizeof(uint32_t);
        std::vector<uint8_t> tmp((size_t)f->ncand * esz);
        if (f->ncand) HIP_TRY(ctx, hipMemcpy(tmp.data(), src, tmp.size(), hipMemcpyDeviceToHost));
        uint8_t *d = static_cast<uint8_t *>(host_dst);
        memset(d, 0, bytes);
        for (size_t c = 0; c < f->ncand; ++c)
            if ((size_t)gm[c] * esz + esz <= bytes) memcpy(d + (size_t)gm[c] * esz, tmp.data() + c * esz, esz);
        return FGS_OK;
    }
    HIP_TRY(ctx, hipMemcpy(host_dst, src, bytes, hipMemcpyDeviceToHost));
    if (field == FGS_FIELD_RANGES) {
        // an empty tile holds start == end on the device; report (0, 0)
        uint2 *r = static_cast<uint2 *>(host_dst);
        for (size_t t = 0; t < bytes / sizeof(uint2); ++t)
            if (r[t].x >= r[t].y) r[t] = make_uint2(0u, 0u);
    }
    return FGS_OK;
}

fgs_status fgs_set_instrumentation(fgs_context *ctx, int flags) {
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "context is NULL");
    if (flags & ~(FGS_INSTR_STAGE_TIMES | FGS_INSTR_WORK))
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "unknown instrumentation flags %d", flags);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipDeviceSynchronize());
    if (flags & FGS_INSTR_STAGE_TIMES)
        for (auto &set : ctx->ev)
            for (hipEvent_t &e : set)
                if (!e) HIP_TRY(ctx, hipEventCreate(&e));
    if ((flags & FGS_INSTR_WORK) && !ctx->work_dev)
        HIP_TRY(ctx, hipMalloc((void **)&ctx->work_dev, 2 * sizeof(unsigned long long)));
    if (ctx->work_dev) HIP_TRY(ctx, hipMemset(ctx->work_dev, 0, 2 * sizeof(unsigned long long)));
    ctx->instr = flags;
    ctx->ev_pending = -1;
    ctx->acc = fgs_timings{};
    return FGS_OK;
}

fgs_status fgs_set_blend_variant(fgs_context *ctx, int32_t variant) {
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "context is NULL");
    if (variant != FGS_BLEND_LDS_BATCHES && variant != FGS_BLEND_PREFETCH)
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "unknown blend variant %d", variant);
    ctx->blend_variant = variant;
    return FGS_OK;
}

fgs_status fgs_get_instrumentation(fgs_context *ctx, fgs_timings *out) {
    if (!ctx || !out) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "NULL argument");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (ctx->ev_pending >= 0) {
        HIP_TRY(ctx, hipEventSynchronize(ctx->ev[ctx->ev_pending][7]));  // the frame's last mark
        fold_events(ctx);
    }
    if (ctx->work_dev) {
        HIP_TRY(ctx, hipDeviceSynchronize());
        unsigned long long w[2] = {0, 0};
        HIP_TRY(ctx, hipMemcpy(w, ctx->work_dev, sizeof w, hipMemcpyDeviceToHost));
        ctx->acc.blend_evaluations = (int64_t)w[0];
        ctx->acc.blend_wave_steps = (int64_t)w[1];
    }
    *out = ctx->acc;
    return FGS_OK;
}

fgs_status fgs_measure_peaks(fgs_context *ctx, fgs_peaks *out) {
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "context is NULL");
    if (!out) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "out is NULL");
    *out = fgs_peaks{};
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipDeviceProp_t prop;
    HIP_TRY(ctx, hipGetDeviceProperties(&prop, ctx->device));
    out->compute_units = prop.multiProcessorCount;
    out->clock_mhz = prop.clockRate / 1000;
    const size_t copy_bytes = (size_t)1 << 30;
    float *sink = nullptr;
    void *a = nullptr, *b = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t s = ctx->side.side;
    fgs_status st = FGS_OK;
    auto cleanup = [&]() {
        (void)hipDeviceSynchronize();
        if (sink) (void)hipFree(sink);
        if (a) (void)hipFree(a);
        if (b) (void)hipFree(b);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
    };
    // best of `reps` timed launches (after one untimed) of `launch`, in ms
    auto best_ms = [&](int reps, auto launch, float *ms) -> hipError_t {
        hipError_t e;
        launch();
        *ms = 1e30f;
        for (int r = 0; r < reps; ++r) {
            if ((e = hipEventRecord(e0, s)) != hipSuccess) return e;
            launch();
            if ((e = hipEventRecord(e1, s)) != hipSuccess) return e;
            if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
            float t = 0.0f;
            if ((e = hipEventElapsedTime(&t, e0, e1)) != hipSuccess) return e;
            *ms = t < *ms ? t : *ms;
        }
        return hipGetLastError();
    };
    hipError_t e = hipMalloc((void **)&sink, sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&a, copy_bytes);
    if (e == hipSuccess) e = hipMalloc(&b, copy_bytes);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipMemsetAsync(a, 0, copy_bytes, s);
    const int blocks = 32 * (prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256);
    const int fma_iters = 4096, exp_iters = 1024;
    float ms = 0.0f;
    if (e == hipSuccess) e = best_ms(3, [&] { launch_peak_fma(blocks, fma_iters, sink, s); }, &ms);
    if (e == hipSuccess) {
        out->fma_lane_ops_per_s = (double)blocks * kBlock * fma_iters * kPeakChains / (ms * 1e-3);
        out->valu_wave_instr_per_s = out->fma_lane_ops_per_s / 64.0;
        e = best_ms(3, [&] { launch_peak_exp(blocks, exp_iters, sink, s); }, &ms);
    }
    if (e == hipSuccess) {
        out->exp_lane_ops_per_s = (double)blocks * kBlock * exp_iters * kPeakChains / (ms * 1e-3);
        e = best_ms(5, [&] { launch_peak_copy(a, b, copy_bytes, s); }, &ms);
    }
    if (e == hipSuccess) out->copy_bytes_per_s = 2.0 * (double)copy_bytes / (ms * 1e-3);
    if (e != hipSuccess) st = hip_fail(ctx, e, "peak-rate measurement");
    cleanup();
    return st;
}

fgs_status fgs_render_backward(fgs_context *ctx, const fgs_frame *frame, const fgs_scene *scene,
                               const fgs_camera *cam, const fgs_options *opt, const float *dL_drgb,
                               const fgs_scene_grad *grad, void *stream_v) {
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "context is NULL");
    if (!frame) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "frame is NULL");
    bool owned = false;
    for (const fgs_frame *f : ctx->frames) owned |= (f == frame);
    if (!owned) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "frame does not belong to this context");
    fgs_status st = validate(ctx, scene, cam ? cam : &frame->cam, frame->W, frame->H, opt ? opt : &frame->opt);
    if (st != FGS_OK) return st;
    if (scene->num_gaussians != frame->P)
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "scene has %lld Gaussians, the frame was rendered with %lld",
                    (long long)scene->num_gaussians, (long long)frame->P);
    if (cam && memcmp(cam, &frame->cam, sizeof(fgs_camera)) != 0)
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "camera differs from the forward call's");
    if (opt && memcmp(opt, &frame->opt, sizeof(fgs_options)) != 0)
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "options differ from the forward call's");
    if (frame->dense)
        return fail(ctx, FGS_ERR_NOT_SUPPORTED,
                    "the frame was rendered from a prepared scene; render from the parameters for gradients");
    if (!dL_drgb) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "dL_drgb is NULL");
    if (!grad) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "grad is NULL");
    const int64_t P = frame->P;
    if (grad->plane_stride < P)
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "grad.plane_stride %lld < num_gaussians %lld",
                    (long long)grad->plane_stride, (long long)P);
    if (P > 0 && (!grad->means || !grad->log_scales || !grad->quats || !grad->opacity_logits || !grad->sh))
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "a gradient pointer is NULL");
    ctx->err.clear();
    hipStream_t s = (hipStream_t)stream_v;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (s != frame->stream) HIP_TRY(ctx, hipStreamWaitEvent(s, frame->done, 0));
    if (P == 0) return FGS_OK;

    const size_t stride = (size_t)P;
    if (ctx->gacc_stride < stride || !ctx->gacc) {
        const size_t cap = stride + stride / 8 + 1024;
        if (ctx->gacc) {
            HIP_TRY(ctx, hipDeviceSynchronize());
            (void)hipFree(ctx->gacc);
            ctx->gacc = nullptr;
            ctx->gacc_stride = 0;
        }
        HIP_TRY(ctx, hipMalloc((void **)&ctx->gacc, 9 * cap * sizeof(float)));
        ctx->gacc_stride = cap;
    }
    const int64_t as = (int64_t)ctx->gacc_stride;
    // cleared with a fill kernel (no memset node if the caller captures a graph)
    launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->gacc), 0u, 9 * (size_t)as, s);

    const DevOptions dop = to_dev(frame->opt);
    const DevCamera dcam = to_dev(frame->cam);
    const FrameBuffers &fb = frame->fb;
    launch_blend_backward(fb.gs, frame->tiles_in_a ? fb.tv_a : fb.tv_b, fb.ranges, fb.T, fb.last, dL_drgb,
                          frame->W, frame->H, dop, ctx->gacc, as, s);
    const DevScene dsc = to_dev(*scene);
    launch_preprocess_backward(dsc, dcam, dop, frame->W, frame->H, fb.gs, ctx->gacc, as, grad->means,
                               grad->log_scales, grad->quats, grad->opacity_logits, grad->sh, grad->plane_stride, s);
    HIP_TRY(ctx, hipGetLastError());
    return FGS_OK;
}

}  // extern "C"
