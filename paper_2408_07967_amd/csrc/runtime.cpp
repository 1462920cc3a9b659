// Host runtime behind the C ABI of include/fgs.h: argument validation,
// context and scratch-arena management, and the orchestration of the
// preprocess -> depth sort -> count scan -> emit -> tile sort -> ranges ->
// blend kernels of one frame.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "fgs.h"
#include "fgs_internal.hpp"

using namespace fgs;

namespace {

thread_local std::string g_null_ctx_error;

// One frame's device buffers.  Everything is sized for a capacity and reused
// across frames (Sec. 5.3.1: no per-frame allocation once warmed up).
struct FrameBuffers {
    size_t capP = 0, capN = 0, capTiles = 0, capPix = 0;
    GaussState *gs = nullptr;
    uint4 *rect = nullptr;
    uint32_t *count = nullptr;
    uint2 *mask = nullptr;
    uint32_t *dkey = nullptr, *dk_b = nullptr, *dv_a = nullptr, *dv_b = nullptr;
    uint32_t *offsets = nullptr;
    uint32_t *tk_a = nullptr, *tk_b = nullptr, *tv_a = nullptr, *tv_b = nullptr;
    uint2 *ranges = nullptr;
    float *T = nullptr;
    uint32_t *last = nullptr;

    size_t bytes() const {
        return capP * (sizeof(GaussState) + sizeof(uint4) + sizeof(uint32_t) + sizeof(uint2) + 4 * sizeof(uint32_t)) +
               (capP + 1) * sizeof(uint32_t) + capN * 4 * sizeof(uint32_t) + capTiles * sizeof(uint2) +
               capPix * (sizeof(float) + sizeof(uint32_t));
    }
};

void free_p(void *&p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

void free_frame_buffers(FrameBuffers &b) {
    void **ps[] = {(void **)&b.gs, (void **)&b.rect, (void **)&b.count, (void **)&b.mask, (void **)&b.dkey,
                   (void **)&b.dk_b, (void **)&b.dv_a, (void **)&b.dv_b, (void **)&b.offsets, (void **)&b.tk_a,
                   (void **)&b.tk_b, (void **)&b.tv_a, (void **)&b.tv_b, (void **)&b.ranges, (void **)&b.T,
                   (void **)&b.last};
    for (void **p : ps) free_p(*p);
    b = FrameBuffers{};
}

}  // namespace

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
};

struct fgs_context {
    int device = 0;
    std::string err;
    FrameBuffers fb;
    std::vector<FrameBuffers> pool;
    std::vector<fgs_frame *> frames;
    FrameCounters *fc_dev = nullptr;
    FrameCounters *fc_host = nullptr;
    // radix-sort and scan scratch (fixed size)
    uint32_t *rhist = nullptr, *gsum = nullptr, *sums = nullptr;
    // chunk list of Gaussians with large rectangles (used within one render)
    uint2 *chunks = nullptr;
    uint32_t *chunk_hits = nullptr;
    size_t chunk_cap = 0;
    uint32_t *chunk_mask = nullptr;  // 256-bit hit mask per chunk
    // instrumentation
    int instr = 0;
    hipEvent_t ev[2][8] = {};
    int ev_pending = -1;  // event set of the last instrumented frame not yet folded in
    int ev_next = 0;
    hipStream_t ev_stream = nullptr;
    fgs_timings acc{};
    unsigned long long *work_dev = nullptr;
    // backward: per-Gaussian sums of the blend adjoint, 9 planes of gacc_stride
    float *gacc = nullptr;
    size_t gacc_stride = 0;
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

#define HIP_TRY(ctx, expr)                                                                                   \
    do {                                                                                                     \
        hipError_t e_ = (expr);                                                                              \
        if (e_ != hipSuccess)                                                                                \
            return fail(ctx, e_ == hipErrorOutOfMemory ? FGS_ERR_OUT_OF_MEMORY : FGS_ERR_DEVICE, "%s: %s", \
                        #expr, hipGetErrorString(e_));                                                       \
    } while (0)

// Add the stage times of a completed instrumented frame to the sums.
void fold_events(fgs_context *ctx) {
    if (ctx->ev_pending < 0) return;
    hipEvent_t *e = ctx->ev[ctx->ev_pending];
    float ms[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int i = 0; i < 7; ++i)
        if (hipEventElapsedTime(&ms[i], e[i], e[i + 1]) != hipSuccess) ms[i] = 0.0f;
    ctx->acc.frames += 1;
    ctx->acc.ms_preprocess += ms[0];
    ctx->acc.ms_depth_sort += ms[1];
    ctx->acc.ms_scan += ms[2];
    ctx->acc.ms_emit += ms[3];
    ctx->acc.ms_tile_sort += ms[4];
    ctx->acc.ms_ranges += ms[5];
    ctx->acc.ms_blend += ms[6];
    ctx->ev_pending = -1;
}

template <class T>
hipError_t grow(T *&p, size_t n_have, size_t n_need) {
    if (n_need <= n_have && p) return hipSuccess;
    if (p) {
        // the old buffer may still be read by queued work
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return e;
        (void)hipFree(p);
    }
    p = nullptr;
    return hipMalloc((void **)&p, (n_need ? n_need : 1) * sizeof(T));
}

fgs_status ensure_gauss(fgs_context *ctx, FrameBuffers &b, size_t P) {
    if (P <= b.capP && b.gs) return FGS_OK;
    size_t cap = P + P / 8 + 1024;
    HIP_TRY(ctx, grow(b.gs, 0, cap));
    HIP_TRY(ctx, grow(b.rect, 0, cap));
    HIP_TRY(ctx, grow(b.count, 0, cap));
    HIP_TRY(ctx, grow(b.mask, 0, cap));
    HIP_TRY(ctx, grow(b.dkey, 0, cap));
    HIP_TRY(ctx, grow(b.dk_b, 0, cap));
    HIP_TRY(ctx, grow(b.dv_a, 0, cap));
    HIP_TRY(ctx, grow(b.dv_b, 0, cap));
    HIP_TRY(ctx, grow(b.offsets, 0, cap + 1));
    b.capP = cap;
    return FGS_OK;
}

fgs_status ensure_pairs(fgs_context *ctx, FrameBuffers &b, size_t N) {
    if (N <= b.capN && b.tk_a) return FGS_OK;
    size_t cap = N + N / 4 + 4096;
    HIP_TRY(ctx, grow(b.tk_a, 0, cap));
    HIP_TRY(ctx, grow(b.tk_b, 0, cap));
    HIP_TRY(ctx, grow(b.tv_a, 0, cap));
    HIP_TRY(ctx, grow(b.tv_b, 0, cap));
    b.capN = cap;
    return FGS_OK;
}

fgs_status ensure_tiles(fgs_context *ctx, FrameBuffers &b, size_t tiles) {
    if (tiles <= b.capTiles && b.ranges) return FGS_OK;
    HIP_TRY(ctx, grow(b.ranges, 0, tiles));
    b.capTiles = tiles;
    return FGS_OK;
}

fgs_status ensure_pixels(fgs_context *ctx, FrameBuffers &b, size_t pix) {
    if (pix <= b.capPix && b.T) return FGS_OK;
    HIP_TRY(ctx, grow(b.T, 0, pix));
    HIP_TRY(ctx, grow(b.last, 0, pix));
    b.capPix = pix;
    return FGS_OK;
}

fgs_status ensure_sort_scratch(fgs_context *ctx) {
    if (ctx->rhist) return FGS_OK;
    HIP_TRY(ctx, grow(ctx->rhist, 0, (size_t)kSortBlocks * kRadix));
    HIP_TRY(ctx, grow(ctx->gsum, 0, (size_t)(kSortBlocks / kSortGroup) * kRadix));
    HIP_TRY(ctx, grow(ctx->sums, 0, (size_t)kSortBlocks));
    return FGS_OK;
}

fgs_status ensure_chunks(fgs_context *ctx, size_t need) {
    need = std::max<size_t>(need, 65536);
    if (need <= ctx->chunk_cap && ctx->chunks) return FGS_OK;
    HIP_TRY(ctx, grow(ctx->chunks, 0, need));
    HIP_TRY(ctx, grow(ctx->chunk_hits, 0, need));
    HIP_TRY(ctx, grow(ctx->chunk_mask, 0, need * (kChunkTiles / 32)));
    ctx->chunk_cap = need;
    return FGS_OK;
}

bool finite_all(const float *p, int n) {
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
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

int ceil_log2(uint64_t x) {
    int b = 0;
    while ((1ull << b) < x) ++b;
    return b;
}

// Split `bits` tile-id bits into passes of at most kRadixBits each.
int plan_tile_passes(int bits, int *shift, int *width) {
    if (bits <= 0) return 0;
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

// ============================================================================
// C ABI
// ============================================================================

extern "C" {

const char *fgs_status_string(fgs_status s) {
    switch (s) {
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

static fgs_status validate(fgs_context *ctx, const fgs_scene *sc, const fgs_camera *cam, int32_t W, int32_t H,
                           const fgs_options *opt) {
    if (!sc) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "scene is NULL");
    if (!cam) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "camera is NULL");
    if (sc->num_gaussians < 0 || sc->num_gaussians > 0x7fffffffLL)
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "num_gaussians %lld out of range [0, 2^31)",
                    (long long)sc->num_gaussians);
    if (sc->plane_stride < sc->num_gaussians)
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "plane_stride %lld < num_gaussians %lld",
                    (long long)sc->plane_stride, (long long)sc->num_gaussians);
    if (sc->sh_degree < 0 || sc->sh_degree > 3)
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "sh_degree %d outside 0..3", sc->sh_degree);
    if (sc->reserved != 0) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "scene.reserved must be 0");
    if (sc->num_gaussians > 0 &&
        (!sc->means || !sc->log_scales || !sc->quats || !sc->opacity_logits || !sc->sh))
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "a scene attribute pointer is NULL");
    if (W < 1 || W > 16384 || H < 1 || H > 16384)
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "image size %dx%d outside 1..16384", W, H);
    if (!finite_all(cam->R, 9) || !finite_all(cam->t, 3) || !finite_all(cam->eye, 3) ||
        !std::isfinite(cam->fx) || !std::isfinite(cam->fy) || !std::isfinite(cam->cx) || !std::isfinite(cam->cy) ||
        !std::isfinite(cam->near_z))
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "camera has a non-finite value");
    if (!(cam->fx > 0.0f) || !(cam->fy > 0.0f)) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "focal length <= 0");
    if (!(cam->near_z > 0.0f)) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "near_z <= 0");
    if (opt) {
        if (!(opt->alpha_min > 0.0f && opt->alpha_min < 1.0f))
            return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "alpha_min outside (0, 1)");
        if (!(opt->T_stop >= 0.0f && opt->T_stop < 1.0f))
            return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "T_stop outside [0, 1)");
        if (!(opt->alpha_max > 0.0f && opt->alpha_max < 1.0f))
            return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "alpha_max outside (0, 1)");
        if (!(opt->dilation >= 0.0f) || !std::isfinite(opt->dilation))
            return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "dilation must be finite and >= 0");
        if (!(opt->jac_clip > 0.0f) || !std::isfinite(opt->jac_clip))
            return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "jac_clip must be finite and > 0");
        if (!finite_all(opt->bg, 3)) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "background is not finite");
        if (opt->binning < 0 || opt->binning > 1)
            return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "binning %d not in {0, 1}", opt->binning);
    }
    return FGS_OK;
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
    for (FrameBuffers &b : ctx->pool) free_frame_buffers(b);
    free_frame_buffers(ctx->fb);
    for (auto &set : ctx->ev)
        for (hipEvent_t &e : set)
            if (e) (void)hipEventDestroy(e);
    if (ctx->work_dev) (void)hipFree(ctx->work_dev);
    if (ctx->chunks) (void)hipFree(ctx->chunks);
    if (ctx->chunk_mask) (void)hipFree(ctx->chunk_mask);
    if (ctx->rhist) (void)hipFree(ctx->rhist);
    if (ctx->gsum) (void)hipFree(ctx->gsum);
    if (ctx->sums) (void)hipFree(ctx->sums);
    if (ctx->chunk_hits) (void)hipFree(ctx->chunk_hits);
    if (ctx->fc_dev) (void)hipFree(ctx->fc_dev);
    if (ctx->fc_host) (void)hipHostFree(ctx->fc_host);
    delete ctx;
}

fgs_status fgs_reserve(fgs_context *ctx, int64_t max_gaussians, int64_t max_pairs, int32_t max_w, int32_t max_h) {
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "context is NULL");
    if (max_gaussians < 0 || max_pairs < 0 || max_w < 0 || max_h < 0 || max_w > 16384 || max_h > 16384)
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "negative or oversized reservation");
    if (max_gaussians > 0x7fffffffLL || max_pairs > 0xffffffffLL)
        return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "reservation beyond 32-bit indices");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    fgs_status s;
    if ((s = ensure_gauss(ctx, ctx->fb, (size_t)max_gaussians)) != FGS_OK) return s;
    if ((s = ensure_pairs(ctx, ctx->fb, (size_t)max_pairs)) != FGS_OK) return s;
    const size_t tiles = (size_t)((max_w + kTile - 1) / kTile) * ((max_h + kTile - 1) / kTile);
    if ((s = ensure_tiles(ctx, ctx->fb, tiles)) != FGS_OK) return s;
    if ((s = ensure_chunks(ctx, (size_t)max_gaussians / 8)) != FGS_OK) return s;
    return ensure_sort_scratch(ctx);
}

size_t fgs_scratch_bytes(const fgs_context *ctx) {
    if (!ctx) return 0;
    size_t b = ctx->fb.bytes() + sizeof(FrameCounters) + ctx->chunk_cap * (sizeof(uint2) + 9 * sizeof(uint32_t)) +
               ((size_t)kSortBlocks * kRadix + (size_t)(kSortBlocks / kSortGroup) * kRadix + kSortBlocks) *
                   sizeof(uint32_t);
    b += 9 * ctx->gacc_stride * sizeof(float);
    for (const FrameBuffers &p : ctx->pool) b += p.bytes();
    for (const fgs_frame *f : ctx->frames) b += f->fb.bytes();
    return b;
}

fgs_status fgs_render(fgs_context *ctx, const fgs_scene *scene, const fgs_camera *cam, int32_t W, int32_t H,
                      const fgs_options *opt_in, float *out_rgb, float *out_T, uint32_t *out_last, fgs_frame **saved,
                      fgs_stats *stats, void *stream_v) {
    if (saved) *saved = nullptr;
    if (!ctx) return fail(nullptr, FGS_ERR_INVALID_ARGUMENT, "context is NULL");
    fgs_status st = validate(ctx, scene, cam, W, H, opt_in);
    if (st != FGS_OK) return st;
    if (!out_rgb) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "out_rgb is NULL");
    fgs_options opt;
    if (opt_in)
        opt = *opt_in;
    else
        fgs_default_options(&opt);
    ctx->err.clear();
    hipStream_t s = (hipStream_t)stream_v;
    HIP_TRY(ctx, hipSetDevice(ctx->device));

    FrameBuffers &fb = ctx->fb;
    const int64_t P = scene->num_gaussians;
    const int tiles_x = (W + kTile - 1) / kTile, tiles_y = (H + kTile - 1) / kTile;
    const uint32_t ntiles = (uint32_t)tiles_x * (uint32_t)tiles_y;
    const size_t npix = (size_t)W * H;
    if ((st = ensure_gauss(ctx, fb, (size_t)P)) != FGS_OK) return st;
    if ((st = ensure_tiles(ctx, fb, ntiles)) != FGS_OK) return st;
    if ((st = ensure_sort_scratch(ctx)) != FGS_OK) return st;
    if (saved && (st = ensure_pixels(ctx, fb, npix)) != FGS_OK) return st;
    if ((st = ensure_chunks(ctx, (size_t)P / 8)) != FGS_OK) return st;

    DevScene dsc{};
    dsc.means = scene->means;
    dsc.log_scales = scene->log_scales;
    dsc.quats = scene->quats;
    dsc.logits = scene->opacity_logits;
    dsc.sh = scene->sh;
    dsc.P = P;
    dsc.stride = scene->plane_stride;
    dsc.D = scene->sh_degree;
    const DevCamera dcam = to_dev(*cam);
    const DevOptions dop = to_dev(opt);
    FrameCounters *fc = ctx->fc_dev;
    const bool timed = (ctx->instr & FGS_INSTR_STAGE_TIMES) != 0;
    const int es = ctx->ev_next;
    auto mark = [&](int i) {
        if (timed) (void)hipEventRecord(ctx->ev[es][i], s);
    };

    uint32_t V = 0, N = 0;
    for (int attempt = 0;; ++attempt) {
    const uint32_t chunk_cap = (uint32_t)std::min<size_t>(ctx->chunk_cap, 0xffffffffu);
    // ---- stage 1: preprocess + exact tile count ---------------------------
    launch_fill_u32(reinterpret_cast<uint32_t *>(fc), 0u, sizeof(FrameCounters) / 4, s);
    mark(0);
    launch_preprocess(dsc, dcam, dop, W, H, fb.gs, fb.rect, fb.count, fb.mask, fb.dkey, ctx->chunks, chunk_cap, fc,
                      s);
    launch_big_count(W, H, opt.binning, fb.gs, fb.rect, ctx->chunks, chunk_cap, ctx->chunk_hits, ctx->chunk_mask,
                     fb.count, fc, s);
    // ---- depth order of the visible Gaussians: 4 LSD passes over the depth
    // digits, hoisted before key duplication (the low half of the (tile |
    // depth) key is the same for every pair of a Gaussian) --------------------
    mark(1);
    const uint32_t P32 = (uint32_t)P;
    uint32_t *rh = ctx->rhist, *gs_ = ctx->gsum;
    launch_radix_pass(fb.dkey, nullptr, fb.dk_b, fb.dv_b, P32, nullptr, 0, 8, true, true, rh, gs_, s);
    launch_radix_pass(fb.dk_b, fb.dv_b, fb.dkey, fb.dv_a, P32, &fc->visible, 8, 8, false, true, rh, gs_, s);
    launch_radix_pass(fb.dkey, fb.dv_a, fb.dk_b, fb.dv_b, P32, &fc->visible, 16, 8, false, true, rh, gs_, s);
    launch_radix_pass(fb.dk_b, fb.dv_b, fb.dkey, fb.dv_a, P32, &fc->visible, 24, 8, false, false, rh, gs_, s);
    mark(2);
    // ---- stage 2a: scan of the tile counts in depth order -------------------
    launch_count_scan(fb.dv_a, fb.count, P32, &fc->visible, fb.dk_b, ctx->sums, fb.offsets, &fc->pairs, s);
    mark(3);
    HIP_TRY(ctx, hipGetLastError());
    HIP_TRY(ctx, hipMemcpyAsync(ctx->fc_host, fc, sizeof(uint32_t) * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(ctx, hipStreamSynchronize(s));
    fold_events(ctx);  // the previous instrumented frame is complete after the wait
    if (ctx->fc_host->error & kErrChunkOverflow) {
        // the large-Gaussian chunk list was too small: size it exactly and
        // render the frame again
        if (attempt > 0) return fail(ctx, FGS_ERR_INTERNAL, "chunk list overflow after resizing");
        if ((st = ensure_chunks(ctx, (size_t)ctx->fc_host->nchunks + (size_t)ctx->fc_host->nchunks / 8)) != FGS_OK)
            return st;
        continue;
    }
    V = ctx->fc_host->visible;
    N = ctx->fc_host->pairs;
    break;
    }  // attempts
    const uint32_t chunk_cap = (uint32_t)std::min<size_t>(ctx->chunk_cap, 0xffffffffu);

    // ---- stage 2b: key emission -------------------------------------------
    if ((st = ensure_pairs(ctx, fb, N)) != FGS_OK) return st;
    int shifts[3] = {0, 0, 0}, widths[3] = {0, 0, 0};
    const int npass = plan_tile_passes(ceil_log2(ntiles), shifts, widths);
    const uint32_t pair_cap = (uint32_t)std::min<size_t>(fb.capN, 0xffffffffu);
    launch_emit(W, H, fb.dv_a, V, fb.offsets, fb.rect, fb.count, fb.mask, fb.tk_a, fb.tv_a, pair_cap, s);
    launch_big_emit(W, fb.rect, fb.mask, ctx->chunks, chunk_cap, ctx->chunk_hits, ctx->chunk_mask, fb.tk_a, fb.tv_a,
                    pair_cap, fc, s);
    mark(4);
    // ---- stage 3: stable LSD sort of the pairs by tile id -------------------
    uint32_t *ki = fb.tk_a, *vi = fb.tv_a, *ko = fb.tk_b, *vo = fb.tv_b;
    for (int p = 0; p < npass; ++p) {
        launch_radix_pass(ki, vi, ko, vo, N, nullptr, shifts[p], widths[p], false, true, ctx->rhist, ctx->gsum, s);
        std::swap(ki, ko);
        std::swap(vi, vo);
    }
    mark(5);
    launch_tile_ranges(ki, N, fb.ranges, ntiles, s);
    mark(6);
    // ---- stage 4: blend -----------------------------------------------------
    float *Tdst = saved ? fb.T : out_T;
    uint32_t *Ldst = saved ? fb.last : out_last;
    launch_blend(fb.gs, vi, fb.ranges, W, H, dop, out_rgb, Tdst, Ldst,
                 (ctx->instr & FGS_INSTR_WORK) ? ctx->work_dev : nullptr, s);
    mark(7);
    HIP_TRY(ctx, hipGetLastError());
    if (timed) {
        ctx->ev_pending = es;
        ctx->ev_next = es ^ 1;
        ctx->ev_stream = s;
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
    stt.sort_passes = 4 + npass;
    if (stats) *stats = stt;

    if (saved) {
        fgs_frame *f = new fgs_frame();
        f->fb = fb;
        f->W = W;
        f->H = H;
        f->P = P;
        f->visible = V;
        f->pairs = N;
        f->tiles_in_a = (ki == fb.tk_a);
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
    case FGS_FIELD_GAUSS: return (size_t)f->P * sizeof(GaussState);
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
    case FGS_FIELD_GAUSS: src = b.gs; break;
    case FGS_FIELD_RECT: src = b.rect; break;
    case FGS_FIELD_COUNT: src = b.count; break;
    case FGS_FIELD_ORDER: src = b.dv_a; break;
    case FGS_FIELD_TILES: src = f->tiles_in_a ? b.tk_a : b.tk_b; break;
    case FGS_FIELD_VALUES: src = f->tiles_in_a ? b.tv_a : b.tv_b; break;
    case FGS_FIELD_RANGES: src = b.ranges; break;
    default: return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "unknown field %d", (int)field);
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipStreamSynchronize(f->stream));
    HIP_TRY(ctx, hipMemcpy(host_dst, src, bytes, hipMemcpyDeviceToHost));
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
        HIP_TRY(ctx, hipMalloc((void **)&ctx->work_dev, sizeof(unsigned long long)));
    if (ctx->work_dev) HIP_TRY(ctx, hipMemset(ctx->work_dev, 0, sizeof(unsigned long long)));
    ctx->instr = flags;
    ctx->ev_pending = -1;
    ctx->acc = fgs_timings{};
    return FGS_OK;
}

fgs_status fgs_get_instrumentation(fgs_context *ctx, fgs_timings *out) {
    if (!ctx || !out) return fail(ctx, FGS_ERR_INVALID_ARGUMENT, "NULL argument");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if (ctx->ev_pending >= 0) {
        HIP_TRY(ctx, hipEventSynchronize(ctx->ev[ctx->ev_pending][7]));
        fold_events(ctx);
    }
    if (ctx->work_dev) {
        HIP_TRY(ctx, hipDeviceSynchronize());
        unsigned long long w = 0;
        HIP_TRY(ctx, hipMemcpy(&w, ctx->work_dev, sizeof w, hipMemcpyDeviceToHost));
        ctx->acc.blend_evaluations = (int64_t)w;
    }
    *out = ctx->acc;
    return FGS_OK;
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
        HIP_TRY(ctx, grow(ctx->gacc, 0, 9 * cap));
        ctx->gacc_stride = cap;
    }
    const int64_t as = (int64_t)ctx->gacc_stride;
    // cleared with a fill kernel (no memset node if the caller captures a graph)
    launch_fill_u32(reinterpret_cast<uint32_t *>(ctx->gacc), 0u, 9 * (size_t)as, s);

    const fgs_options &op = frame->opt;
    const DevOptions dop = to_dev(op);
    const DevCamera dcam = to_dev(frame->cam);
    const FrameBuffers &fb = frame->fb;
    launch_blend_backward(fb.gs, frame->tiles_in_a ? fb.tv_a : fb.tv_b, fb.ranges, fb.T, fb.last, dL_drgb,
                          frame->W, frame->H, dop, ctx->gacc, as, s);
    DevScene dsc{};
    dsc.means = scene->means;
    dsc.log_scales = scene->log_scales;
    dsc.quats = scene->quats;
    dsc.logits = scene->opacity_logits;
    dsc.sh = scene->sh;
    dsc.P = P;
    dsc.stride = scene->plane_stride;
    dsc.D = scene->sh_degree;
    launch_preprocess_backward(dsc, dcam, dop, frame->W, frame->H, fb.gs, ctx->gacc, as, grad->means,
                               grad->log_scales, grad->quats, grad->opacity_logits, grad->sh, grad->plane_stride, s);
    HIP_TRY(ctx, hipGetLastError());
    return FGS_OK;
}

}  // extern "C"
