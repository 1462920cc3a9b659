/*
 * fgs.h - C ABI of the MI355X (gfx950) Gaussian-splatting rasterizer with
 * exact ellipse/tile intersection (FlashGS, arXiv 2408.07967).
 *
 * The library renders a set of 3D Gaussians (Alg. 1 / Alg. 4 inputs:
 * positions, scales, rotations, opacities, SH coefficients) through one
 * pinhole camera into an RGB image, in four stages that all run as HIP
 * kernels on the GPU:
 *   1. per-Gaussian preprocessing with the exact ellipse/tile test
 *      (Sec. 4.1, Alg. 3, Eq. 1-3 and Eq. 7, Alg. 4),
 *   2. key emission after a prefix scan of per-Gaussian tile counts
 *      (Alg. 2 offsets; Sec. 4.2 fusion of intersection and key generation),
 *   3. radix sort of (tile | depth) keys and per-tile ranges (Sec. 2.2):
 *      depth first, once per Gaussian, then the (super-tile, Gaussian, hit
 *      mask) entries by super-tile, expanded into the per-tile lists,
 *   4. per-tile front-to-back alpha blending with early termination
 *      (Sec. 2.2, Sec. 5.2).
 *
 * Conventions shared by every entry point:
 *   - Pointers marked "device" are HIP device memory owned by the caller;
 *     "host" pointers are ordinary host memory.  The library never frees
 *     caller memory.
 *   - Every call returns an fgs_status and never aborts or throws across the
 *     ABI.  Argument errors are detected on the host before any HIP call and
 *     return FGS_ERR_INVALID_ARGUMENT; fgs_last_error() then describes them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is stream-ordered; outputs are valid once the stream reaches the
 *     end of the call's work.
 *   - A context may be used by one host thread at a time.
 */
#ifndef FGS_H
#define FGS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FGS_OK = 0,
    FGS_ERR_INVALID_ARGUMENT = 1,
    FGS_ERR_OUT_OF_MEMORY = 2,
    FGS_ERR_CAPACITY = 3,
    FGS_ERR_DEVICE = 4,
    FGS_ERR_NOT_SUPPORTED = 5,
    FGS_ERR_INTERNAL = 6
} fgs_status;

typedef struct fgs_context fgs_context; /* device, scratch arena, error text */
typedef struct fgs_frame fgs_frame;     /* saved forward state for the backward */

/* Gaussian parameters, planar binary32 in device memory.  Plane c of an
 * attribute X is X + c * plane_stride, one float per Gaussian.
 * (Alg. 1 / Alg. 4 inputs: positions, scales s, rotations R, opacity, shs.) */
typedef struct {
    int64_t num_gaussians;      /* P >= 0; P == 0 renders the background   */
    int64_t plane_stride;       /* >= P                                      */
    int32_t sh_degree;          /* D in 0..3                                 */
    int32_t reserved;           /* must be 0                                 */
    const float *means;         /* device, 3 planes: world x, y, z           */
    const float *log_scales;    /* device, 3 planes: scale = exp(value)      */
    const float *quats;         /* device, 4 planes w, x, y, z; any non-zero
                                   norm (normalised inside)                  */
    const float *opacity_logits;/* device, 1 plane: opacity = sigmoid(value) */
    const float *sh;            /* device, 3 (D+1)^2 planes; plane 3 k + ch,
                                   k = l^2 + l + m (real SH, Condon-Shortley
                                   phase)                                    */
} fgs_scene;

/* Gradients with respect to the raw parameters above (same planar layout);
 * device memory owned by the caller, overwritten by fgs_render_backward. */
typedef struct {
    int64_t plane_stride;
    float *means, *log_scales, *quats, *opacity_logits, *sh;
} fgs_scene_grad;

/* Pinhole camera (Alg. 1 viewmatrix / focal inputs).  x_cam = R x + t with R
 * row-major; camera axes: x right, y down, z forward.  eye is the camera
 * centre in world space (direction for the SH colour).  Pixel (i, j) is
 * sampled at (i + 1/2, j + 1/2).  near_z: Gaussians need z_cam > near_z
 * (0.2 in Alg. 4). */
typedef struct {
    float R[9];
    float t[3];
    float eye[3];
    float fx, fy, cx, cy;
    float near_z;
} fgs_camera;

typedef struct {
    float alpha_min; /* tau: opacity cutoff and extent threshold, 1/255 (Sec. 4.1) */
    float T_stop;    /* transmittance at which a pixel stops, 1e-4                 */
    float alpha_max; /* per-Gaussian alpha clamp, 0.99                              */
    float dilation;  /* low-pass added to the 2D covariance diagonal, 0.3 px^2      */
    float jac_clip;  /* projection-Jacobian clamp, multiple of the half image, 1.3 */
    float bg[3];     /* background colour, black by default                        */
    int32_t cap_3sigma; /* 1: extent k^2 = min(9, 2 ln(o / tau)) (Eq. 1-3)          */
    int32_t binning;    /* 0: exact ellipse/tile test (Alg. 3); 1: every tile of the
                           tight box; 2: every tile of the square box of the 3 sigma
                           circle, radius ceil(3 sqrt(lambda_max)) (the 3DGS binning
                           of Alg. 1 / Alg. 2).  1 and 2 are comparison modes: more
                           pairs, the same image                                     */
} fgs_options;

typedef struct {
    int64_t visible;   /* Gaussians that survived preprocessing          */
    int64_t pairs;     /* Gaussian-tile key/value pairs emitted          */
    int32_t tiles_x, tiles_y;
    int32_t sort_passes; /* radix passes: 4 over the depth keys, then those
                           over the super-tile ids of the entries (one of up
                           to 9 bits, else 8 bits each)                      */
    int32_t big_chunks; /* 256-tile chunks of the rectangles of more than 64
                           tiles, tested by wavefronts across the GPU        */
    int64_t candidates; /* Gaussians preprocessed: the cull's candidates of a
                           prepared scene, every Gaussian otherwise          */
    int64_t entries;    /* (Gaussian, 8 x 8-tile super-tile) entries emitted:
                           one per super-tile a Gaussian's rectangle overlaps */
    int64_t cull_batches; /* prepared scene: batches of 256 precompute slots its
                           cull read (the others' bounds showed that every
                           member would be culled); 0 for raw parameters    */
} fgs_stats;

/* ---- context --------------------------------------------------------- */

/* Create a context on HIP device `device`.  *out receives the handle, or NULL
 * with FGS_ERR_DEVICE when the device is missing / not gfx950. */
fgs_status fgs_create(int device, fgs_context **out);

/* Destroy a context and every frame it still owns (NULL is ignored). */
void fgs_destroy(fgs_context *ctx);

/* Static description of a status code. */
const char *fgs_status_string(fgs_status s);

/* Text of the last error on this context ("" if none); valid until the next
 * call on the context.  With ctx == NULL: the last error of a call that was
 * given no context. */
const char *fgs_last_error(const fgs_context *ctx);

/* Fill *opt with the defaults listed in fgs_options. */
void fgs_default_options(fgs_options *opt);

/* Host-only validation of render arguments (no HIP call).  Returns
 * FGS_ERR_INVALID_ARGUMENT for: null pointers, P < 0, plane_stride < P,
 * sh_degree outside 0..3, W or H outside 1..16384, non-finite camera values,
 * fx or fy <= 0, near_z <= 0, or out-of-range options. */
fgs_status fgs_validate(const fgs_scene *scene, const fgs_camera *cam, int32_t W, int32_t H,
                        const fgs_options *opt);

/* Pre-size the context's device scratch so that later renders up to these
 * sizes allocate nothing (Sec. 5.3.1: allocation hoisted out of the frame
 * loop). */
fgs_status fgs_reserve(fgs_context *ctx, int64_t max_gaussians, int64_t max_pairs, int32_t max_w,
                       int32_t max_h);

/* Bytes of device scratch currently held by the context. */
size_t fgs_scratch_bytes(const fgs_context *ctx);

/* ---- forward ------------------------------------------------------------ */

/* Render scene through cam at W x H.
 *   out_rgb  device, [3][H][W] float (planar RGB), required.
 *   out_T    device, [H][W] float final transmittance, or NULL.
 *   out_last device, [H][W] uint32: 1 + position, within its tile's sorted
 *            list, of the last Gaussian that contributed to the pixel (0 if
 *            none), or NULL.
 *   saved    if non-NULL, receives a frame handle that keeps the per-Gaussian
 *            state, the sorted list, the tile ranges, T_final and last for
 *            fgs_render_backward / fgs_frame_download; release it with
 *            fgs_frame_release.
 *   stats    host, or NULL: counts of the frame.
 * The call enqueues the whole frame, then waits once on `stream` for the
 * number of pairs (busy-polling an event, so the calling thread spins for the
 * first half of the frame); if the context's pair buffers were too small for
 * it, they grow and the second half is enqueued again.  It returns with the
 * second half still in flight.  opt == NULL means defaults. */
fgs_status fgs_render(fgs_context *ctx, const fgs_scene *scene, const fgs_camera *cam, int32_t W, int32_t H,
                      const fgs_options *opt, float *out_rgb, float *out_T, uint32_t *out_last,
                      fgs_frame **saved, fgs_stats *stats, void *stream);

/* Plan one frame without rendering it: the first half of fgs_render runs
 * (preprocess with the exact tile count, depth order, scan of the counts;
 * Alg. 4 and Alg. 2 up to the pair count) and the call waits for it.
 *   pairs_out  host, or NULL: number of Gaussian-tile pairs of the frame
 *   bytes_out  host, or NULL: device bytes the context needs to render it
 *              (per-Gaussian, pair, tile, sort and chunk buffers; without the
 *              output image and without a saved frame's per-pixel buffers)
 * At least one of the two must be non-NULL.  The context keeps the
 * per-Gaussian buffers it grew; pair buffers are not allocated. */
fgs_status fgs_plan(fgs_context *ctx, const fgs_scene *scene, const fgs_camera *cam, int32_t W, int32_t H,
                    const fgs_options *opt, int64_t *pairs_out, size_t *bytes_out, void *stream);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid hipMalloc): fgs_render without a saved frame, whose
 * kernels take every scratch buffer (per-Gaussian state, depth order, count
 * scan, super-tile entries and their sort ping-pong, pairs, tile ranges, large-rectangle chunk
 * list, frame counters) from one fixed device array of
 * FGS_NOALLOC_SCRATCH_BYTES per GPU, part of the library's code object: each
 * GPU the library runs on holds it until the process ends.  The call makes no
 * hipMalloc, hipFree or other allocating call (the context's events, second
 * stream and pinned counter copy come from fgs_create, which also takes the
 * array's device address).  Arguments, outputs and the single wait for the
 * pair count are those of fgs_render; the image is bit-identical to it.
 * Limits: the per-Gaussian part (about 130 B per Gaussian), the tile ranges
 * (16 B per tile), the sort scratch and a chunk list of max(P / 8, 8192)
 * entries are carved first and must fit, else FGS_ERR_CAPACITY before any
 * device work; the rest holds the pairs (16 B each, which also hold the
 * super-tile entries: 28 B each).  A frame with more pairs or entries than
 * that, or with more large-rectangle chunks than the list holds, returns
 * FGS_ERR_CAPACITY after its device work (the image is then incomplete).
 * Every call on one GPU, from any context, uses that GPU's one array, which
 * keeps the previous call's contents (each frame clears what must start at
 * zero): calls that overlap on one GPU race (different streams, threads or
 * contexts without ordering between them), and a call returns with its
 * second half still in flight on `stream`, so a later call on another stream
 * must wait for that one first. */
#define FGS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
fgs_status fgs_render_noalloc(fgs_context *ctx, const fgs_scene *scene, const fgs_camera *cam, int32_t W,
                              int32_t H, const fgs_options *opt, float *out_rgb, float *out_T, uint32_t *out_last,
                              fgs_stats *stats, void *stream);

/* ---- prepared (resident) scenes ------------------------------------------ */

/* The paper moves preprocessing shared by the viewpoints of one scene to an
 * initial stage (Sec. 5.3.1).  fgs_prepare_scene computes, once, the
 * view-independent part of every Gaussian: opacity (0 for a Gaussian that can
 * never be visible), scales and unit quaternion, extent k^2, a bound of the
 * screen extent (trace of the 3D covariance), and the SH coefficients
 * Gaussian-major, so a frame reads 24 bytes for every Gaussian of the
 * 256-slot batches its cull reads, 48 more for the candidates of its cull and
 * one contiguous run of SH for the visible ones.  The precompute stores the
 * Gaussians in a spatial order (Morton order of the means, computed and
 * sorted here), so that the candidates of a frame's cull, which see one
 * region of the scene, are read as few contiguous runs; per batch it keeps
 * bounds (box of the means, greatest opacity, trace and k^2) from which the
 * cull skips the batches whose every member it would cull.  Frames re-order
 * equal depths by Gaussian index, so the pair order is still the method's.
 * Device memory owned by the context: 60 B + 4 ceil4(3 (D+1)^2) B per
 * Gaussian (252 B at degree 3) and 48 B per batch, plus 16 B per Gaussian and
 * the sort scratch during the call.  It depends on the
 * scene's values (copy of the fgs_scene struct kept; the planes must stay
 * valid and unchanged for backward passes) and on opt->alpha_min and
 * opt->cap_3sigma.  Frames rendered from it are bit-identical to fgs_render
 * of the scene.  Runs on `stream` and waits for it before returning. */
typedef struct fgs_prepared fgs_prepared;
fgs_status fgs_prepare_scene(fgs_context *ctx, const fgs_scene *scene, const fgs_options *opt, fgs_prepared **out,
                             void *stream);
/* Waits for the device, then frees the precompute (NULL is ignored). */
fgs_status fgs_prepared_release(fgs_context *ctx, fgs_prepared *prepared);
/* fgs_render from a prepared scene.  opt: NULL means defaults; its
 * alpha_min and cap_3sigma must equal those of the preparation. */
fgs_status fgs_render_prepared(fgs_context *ctx, const fgs_prepared *prepared, const fgs_camera *cam, int32_t W,
                               int32_t H, const fgs_options *opt, float *out_rgb, float *out_T, uint32_t *out_last,
                               fgs_frame **saved, fgs_stats *stats, void *stream);
/* Several viewpoints of one prepared scene in one call (Sec. 5.3.1 carried
 * one step further: the preprocessing of every viewpoint of the batch shares
 * one pass).  One cull keeps the union of the cameras' candidates and one
 * preprocess pass walks that list, evaluating each Gaussian for every camera
 * in turn, so its precompute comes from HBM once per batch, not once per
 * camera; sorting and blending then run per camera.
 *   cams      host, ncams cameras, 1 <= ncams <= FGS_MAX_BATCH_CAMERAS; one
 *             W, H and opt (as for fgs_render_prepared) for all of them.
 *   out_rgb   host array of ncams device pointers, each [3][H][W] float.
 *   out_T, out_last  NULL, or host arrays of ncams device pointers (an
 *             entry may be NULL), [H][W] float / uint32.
 *   stats     NULL or host array of ncams fgs_stats.
 * Camera c's image, T_final and last contributor are bit for bit those of
 * fgs_render_prepared for camera c alone.  No frame is saved (a batch has
 * no backward) and a batch collects neither stage times nor work counts.
 * Device memory: one set of frame buffers per camera slot, grown on demand
 * (fgs_reserve does not size them) and kept by the context for later batches.  Enqueued on `stream`: the second halves of odd
 * cameras run on the context's own second stream, which `stream` waits for
 * on the device, so later work on `stream` sees every output.  Like
 * fgs_render_prepared it returns once the frame counters are on the host.
 * Errors as for fgs_render_prepared, and INVALID_ARGUMENT for ncams out of
 * range. */
#define FGS_MAX_BATCH_CAMERAS 8
fgs_status fgs_render_prepared_batch(fgs_context *ctx, const fgs_prepared *prepared, const fgs_camera *cams,
                                     int32_t ncams, int32_t W, int32_t H, const fgs_options *opt,
                                     float *const *out_rgb, float *const *out_T, uint32_t *const *out_last,
                                     fgs_stats *stats, void *stream);

/* ---- backward ----------------------------------------------------------- */

/* Gradients of a scalar loss L with respect to the raw scene parameters
 * (the paper calls its rasterizer differentiable and leaves the adjoint out;
 * this one replays each pixel's blend back to front from its saved final
 * transmittance and last contributor, with wavefront-reduced atomics as in
 * the DISTWAR work the paper cites).
 *   frame    a frame saved by fgs_render of this context (not released);
 *            a frame of fgs_render_prepared gives FGS_ERR_NOT_SUPPORTED.
 *   scene    the forward call's scene, same pointers and unchanged values.
 *   cam, opt NULL, or identical to the forward call's (else INVALID_ARGUMENT).
 *   dL_drgb  device, [3][H][W] float, H and W of the frame.
 *   grad     device gradient planes, planar like the scene with
 *            grad->plane_stride >= P; every plane of Gaussians 0..P-1 is
 *            overwritten (zero for culled Gaussians).  The derivative through
 *            a clamped alpha, a colour channel clamped at 0 or a clamped
 *            Jacobian view direction is zero.  Camera gradients are not
 *            computed.
 * Enqueued on `stream`, which first waits for the forward's work if it ran
 * on another stream.  Floating-point atomics make the summation order, and so
 * the last bits of the gradients, vary from run to run.  The context's
 * accumulation buffer (9 floats per Gaussian) grows on first use. */
fgs_status fgs_render_backward(fgs_context *ctx, const fgs_frame *frame, const fgs_scene *scene,
                               const fgs_camera *cam, const fgs_options *opt, const float *dL_drgb,
                               const fgs_scene_grad *grad, void *stream);

/* Release a saved frame (NULL is ignored). */
fgs_status fgs_frame_release(fgs_context *ctx, fgs_frame *frame);

/* Introspection of a saved frame for tests and tools: copies one field to
 * host memory (synchronising the frame's stream).  Fields and layouts:
 *   FGS_FIELD_GAUSS   [P][16] float: u, v, conic A, B, C, k^2, log2(o),
 *                     r, g, b, depth, o, blend conic Ab, Bb, Cb, 0 (valid
 *                     Gaussians only; others are 0 for a prepared scene's
 *                     frame and unspecified otherwise).  A, B, C is the
 *                     canonical binary32 conic that decides the pairs; the
 *                     blend evaluates pixels with Ab, Bb, Cb, the same conic
 *                     computed in binary64 and rounded once
 *   FGS_FIELD_RECT    [P][4] int32: tx0, tx1, ty0, ty1 (valid only)
 *   FGS_FIELD_COUNT   [P] uint32 exact tile count (0 for culled Gaussians)
 *   FGS_FIELD_ORDER   [visible] uint32 Gaussian indices in (depth, index) order
 *   FGS_FIELD_TILES   [pairs] uint32 tile id of each sorted pair (the sort keeps only
 *                     the ranges; the ids are expanded from them on the host)
 *   FGS_FIELD_VALUES  [pairs] uint32 Gaussian index of each sorted pair
 *   FGS_FIELD_RANGES  [tiles][2] uint32 [start, end) of each tile's list ((0, 0) if empty)
 * `bytes` must equal the field's size (fgs_frame_field_bytes). */
typedef enum {
    FGS_FIELD_GAUSS = 0,
    FGS_FIELD_RECT = 1,
    FGS_FIELD_COUNT = 2,
    FGS_FIELD_ORDER = 3,
    FGS_FIELD_TILES = 4,
    FGS_FIELD_VALUES = 5,
    FGS_FIELD_RANGES = 6
} fgs_field;

/* ---- instrumentation (measurement only; off by default) ------------------ */

#define FGS_INSTR_STAGE_TIMES 1 /* HIP events around every stage on the render stream */
#define FGS_INSTR_WORK 2        /* count blend evaluations (a slower blend variant)   */

typedef struct {
    int64_t frames;            /* instrumented frames folded into the sums below     */
    double ms_preprocess;      /* summed stage times over those frames (ms); the
                                  preprocess kernel alone (a prepared scene's cull
                                  is ms_cull)                                        */
    double ms_depth_sort;
    double ms_scan;
    double ms_emit;            /* super-tile entries (key emission)                  */
    double ms_super_sort;      /* radix sort of the entries by super-tile            */
    double ms_tile_lists;      /* per-tile lists and ranges from the sorted entries  */
    double ms_blend;
    int64_t blend_evaluations; /* with FGS_INSTR_WORK: sum over pixels of the number of
                                  list entries the pixel examines (up to and including
                                  the entry at which it stops, else the whole list),
                                  summed over the instrumented frames                */
    double ms_cull;            /* the cull of a prepared scene (0 for raw parameters) */
    int64_t blend_wave_steps;  /* with FGS_INSTR_WORK: (wavefront, list entry) steps the
                                  blend executes; each evaluates one entry at the
                                  wavefront's 128 pixels (entries that miss the
                                  wavefront's half tile are skipped)                 */
} fgs_timings;

/* Select instrumentation flags for later fgs_render calls and clear the sums. */
fgs_status fgs_set_instrumentation(fgs_context *ctx, int flags);

/* ---- blend variants (Sec. 5.3.2) --------------------------------------------
 * Two kernels render the same image, bit for bit:
 *   FGS_BLEND_LDS_BATCHES (default): the workgroup of a tile stages batches of
 *       its sorted list in LDS and each wavefront skips the entries whose
 *       ellipse misses its half of the tile;
 *   FGS_BLEND_PREFETCH: each wavefront walks the list on its own with a
 *       software prefetch pipeline (the state of entry i + 1 and the index of
 *       entry i + 2 in flight while entry i is blended), no LDS, no skipping.
 * Applies to later fgs_render / fgs_render_prepared calls of ctx (the
 * evaluation count of FGS_INSTR_WORK always uses the default).  Returns
 * FGS_ERR_INVALID_ARGUMENT for another value. */
#define FGS_BLEND_LDS_BATCHES 0
#define FGS_BLEND_PREFETCH 1
fgs_status fgs_set_blend_variant(fgs_context *ctx, int32_t variant);

/* Wait for the last instrumented frame and return the sums. */
fgs_status fgs_get_instrumentation(fgs_context *ctx, fgs_timings *out);

/* Measured peak rates of the context's device (measurement only): kernels
 * that do nothing but one operation over enough wavefronts to fill every
 * SIMD, timed with HIP events (best of several runs).  They give the
 * measured denominators of the rooflines beside the published peaks.
 * Allocates and frees 2 GiB of device memory for the copy; synchronises the
 * device.  Takes a few tens of milliseconds. */
typedef struct {
    double fma_lane_ops_per_s;    /* binary32 FMAs (non-packed), lane operations per second */
    double valu_wave_instr_per_s; /* the same as wave64 VALU instructions per second        */
    double exp_lane_ops_per_s;    /* v_exp_f32, lane operations per second                   */
    double copy_bytes_per_s;      /* device-to-device copy, bytes read plus written per second */
    int32_t compute_units;
    int32_t clock_mhz;            /* the device's reported peak engine clock                 */
} fgs_peaks;
fgs_status fgs_measure_peaks(fgs_context *ctx, fgs_peaks *out);

size_t fgs_frame_field_bytes(const fgs_frame *frame, fgs_field field);
fgs_status fgs_frame_download(fgs_context *ctx, const fgs_frame *frame, fgs_field field, void *host_dst,
                              size_t bytes);
fgs_status fgs_frame_stats(const fgs_frame *frame, fgs_stats *stats);

/* ---- render server: continuous batching over a resident scene ---------- */
/* The paper renders one frame at a time from statically allocated buffers
 * (Sec. 5.3.1).  The server keeps one scene resident and serves camera
 * requests of mixed resolutions concurrently.  A request takes a slot (its
 * own stream and per-Gaussian buffers) and runs the first half of the frame
 * (preprocess, exact tile counts, depth order, count scan), which yields its
 * exact pair count N and its super-tile entries; requests that start
 * together share the cull and preprocess of that half (batch_fronts).  It is
 * then admitted when its pair and sort buffers (16 bytes per unit of the pair
 * capacity those need) fit in the free part of a device byte budget: FIFO, a
 * request that does not fit may be overtaken by at most max_bypass later
 * ones.  The second half (emission, super-tile sort, tile lists, blend) then
 * runs as a hipGraph captured once per (slot, resolution) and replayed.  A slot that
 * still holds the pair region of an earlier request enqueues that graph right
 * behind the first half, before the pair count is known (its kernels read
 * the count on the device and stay within the region), so that the host's
 * wait for the count is off the request's path; a frame with more pairs than
 * the region is admitted and run again.  Requests
 * in different slots overlap on the device.  One worker thread owned by the
 * server issues all of its GPU work.  The server keeps the scene's
 * view-independent precompute (see fgs_prepare_scene).  Images are
 * bit-identical to fgs_render of the same request alone. */
typedef struct fgs_server fgs_server;

typedef struct {
    int64_t budget_bytes;   /* pair and sort buffers of admitted requests (>= 1 MiB) */
    int32_t max_inflight;   /* slots, 1..32                                          */
    int32_t max_width;      /* largest request, 1..16384                             */
    int32_t max_height;
    int32_t max_bypass;     /* >= 0                                                  */
    int32_t use_graphs;     /* 1: replay a captured graph per (slot, W, H); 0: launch */
    int32_t share_queue;    /* >= 0.  0: waiting requests start on every free slot;
                               k >= 1: a request starts beside others still in flight
                               only while at least k requests are waiting, so at light
                               load requests run one at a time on the whole GPU      */
    int32_t batch_fronts;   /* 0 or 1.  1: requests that start together (up to
                               FGS_MAX_BATCH_CAMERAS, any mix of resolutions) share one
                               cull and one preprocess pass, which reads each
                               candidate's precompute once for all of them; 0: every
                               request runs its own                                  */
} fgs_server_config;

typedef struct {
    uint64_t id;
    int32_t status;         /* FGS_OK; FGS_ERR_CAPACITY if the request can never fit
                               the budget; FGS_ERR_DEVICE on a device error        */
    int32_t width, height;
    int32_t slot;
    const float *rgb;       /* device [3][H][W]; valid until fgs_server_release(id) */
    int64_t arrival_ns;     /* fgs_clock_ns() clock, as submitted                   */
    int64_t start_ns;       /* first half enqueued                                  */
    int64_t admit_ns;       /* second half enqueued                                 */
    int64_t done_ns;        /* completion observed by the worker                    */
    int64_t visible, pairs;
} fgs_server_result;

typedef struct {
    int64_t submitted, completed, rejected;
    int64_t graphs_captured, graph_launches;
    int64_t region_allocs, region_evictions, bypasses;
    int64_t peak_bytes_in_use;  /* of the budget                                       */
    int64_t budget_bytes;
    int64_t slot_bytes;         /* buffers outside the budget: all slots and the
                                   scene's view-independent precompute             */
    int64_t batched_fronts;     /* first halves run as one batch (batch_fronts)     */
    int64_t batched_requests;   /* requests whose first half ran in such a batch    */
    int64_t spec_launches;      /* second halves enqueued right behind the first on
                                   a slot's cached pair region                     */
    int64_t spec_misses;        /* of those, frames with more pairs than the region:
                                   the request was admitted and run again          */
} fgs_server_stats;

/* Monotonic clock (ns) of the server's timestamps. */
int64_t fgs_clock_ns(void);

/* scene: device planes that stay valid and unchanged while the server lives.
 * opt: NULL means defaults; fixed for all requests. */
fgs_status fgs_server_create(int device, const fgs_scene *scene, const fgs_options *opt,
                             const fgs_server_config *cfg, fgs_server **out);
/* Stops the worker after the work in flight; frees everything. */
void fgs_server_destroy(fgs_server *srv);
const char *fgs_server_last_error(const fgs_server *srv);
/* Queue a request (thread-safe).  W, H within the configured maximum.
 * out_rgb: NULL (the image stays in the slot until fgs_server_release), or
 * caller-owned device memory of 3 W H floats that receives a copy of the
 * image before the request is reported complete. */
fgs_status fgs_server_submit(fgs_server *srv, uint64_t id, const fgs_camera *cam, int32_t W, int32_t H,
                             int64_t arrival_ns, float *out_rgb);
/* Move up to max completed requests into out, waiting up to wait_ns for the
 * first; returns their number (>= 0) or a negative fgs_status. */
int32_t fgs_server_poll(fgs_server *srv, fgs_server_result *out, int32_t max, int64_t wait_ns);
/* The image of a completed request may be overwritten; its slot is reused. */
fgs_status fgs_server_release(fgs_server *srv, uint64_t id);
fgs_status fgs_server_get_stats(fgs_server *srv, fgs_server_stats *out);

/* One request of a recorded trace: arrival relative to the replay's start. */
typedef struct {
    uint64_t id;
    fgs_camera cam;
    int32_t width, height;
    int64_t arrival_offset_ns;
} fgs_trace_request;

/* Replay a trace through the server: submit each request at its arrival
 * time, release every image as soon as it completes.  results[i] belongs to
 * trace[i]. */
fgs_status fgs_server_replay(fgs_server *srv, const fgs_trace_request *trace, int64_t n,
                             fgs_server_result *results);

/* The same trace through the plain renderer: one request at a time in
 * arrival order, fgs_render into rgb_scratch (device, >= 3 W H floats of the
 * largest request), waiting for each frame before the next. */
fgs_status fgs_replay_plain(fgs_context *ctx, const fgs_scene *scene, const fgs_options *opt,
                            const fgs_trace_request *trace, int64_t n, float *rgb_scratch,
                            fgs_server_result *results, void *stream);

/* The same replay from a prepared scene of ctx (fgs_render_prepared per
 * request): the plain renderer with the resident precompute the server
 * keeps, so that a comparison with the server measures the serving machinery
 * alone.  INVALID_ARGUMENT also for a NULL prepared scene. */
fgs_status fgs_replay_plain_prepared(fgs_context *ctx, const fgs_prepared *prepared, const fgs_options *opt,
                                     const fgs_trace_request *trace, int64_t n, float *rgb_scratch,
                                     fgs_server_result *results, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* FGS_H */
