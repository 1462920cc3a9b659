// Render server: continuous batching of camera requests over one resident
// scene (declared in include/fgs.h).
//
// Request life cycle, driven by one worker thread that issues all GPU work:
//   QUEUED  -> FRONT  a free slot runs the first half of the frame on its
//                     own stream (preprocess, exact tile counts, depth order,
//                     count scan) and copies the frame counters to the host;
//                     requests that start together share one cull and one
//                     preprocess pass (then sort and scan on their own slots)
//   FRONT   -> WAIT   the counters arrived: N pairs are known
//   WAIT    -> BACK   admitted: 16 C bytes (+ headroom) of the byte budget
//                     back the slot's pair and sort buffers (C: the pair
//                     capacity the frame's pairs and super-tile entries
//                     need); the second half (emission, super-tile sort,
//                     tile lists, blend) is a graph captured
//                     once per (slot, W, H) while the slot's buffers stay put
//   BACK    -> DONE   the image is complete; the client polls the result
//   DONE    -> IDLE   the client released the image
// Admission is FIFO over the waiting requests in arrival order; a request
// that does not fit may be overtaken by at most max_bypass later ones.
// Slots keep their pair region between requests (so their graphs stay
// valid); regions of slots that are not blending are evicted when a waiting
// request needs the space.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fgs.h"
#include "fgs_internal.hpp"
#include "arena.hpp"
#include "pipeline.hpp"

using namespace fgs;

namespace {

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

size_t align_up(size_t x) { return arena_align(x); }

struct Request {
    uint64_t id = 0;
    fgs_camera cam{};
    int W = 0, H = 0;
    int64_t arrival_ns = 0;
    uint64_t seq = 0;  // submission order
    float *out = nullptr;  // optional caller copy of the image
};

enum class SlotState { IDLE, FRONT, WAIT, BACK, DONE };

struct GraphEntry {
    int W, H;
    hipGraphExec_t exec;
};

struct Slot {
    int idx = 0;
    SlotState state = SlotState::IDLE;
    hipStream_t stream = nullptr;
    hipEvent_t evA = nullptr, evB = nullptr;
    hipEvent_t evP = nullptr;  // a batched front half's shared preprocess is complete
    SideStream side;
    FrameBuffers fb;
    ChunkList ch;
    SortScratch ss;
    FrameCounters *fc_dev = nullptr, *fc_host = nullptr;
    float *img = nullptr;
    // pair region in the arena
    bool has_region = false;
    size_t reg_off = 0, reg_bytes = 0;
    std::vector<GraphEntry> graphs;
    // a second half enqueued right behind the first, on the slot's cached
    // pair region, before the pair count is known; its region stays in use
    // until evB has passed
    bool spec = false;
    // current request
    Request req;
    int attempts = 0;
    int bypassed = 0;
    int64_t start_ns = 0, admit_ns = 0, done_ns = 0;
    uint32_t V = 0, N = 0;
    size_t Ncap = 0;  // pair-array capacity the request needs (pairs and super-tile entries)
};

}  // namespace

struct fgs_server {
    int device = 0;
    fgs_scene scene{};
    DevScene dsc{};
    fgs_options opt{};
    DevOptions dop{};
    fgs_server_config cfg{};
    std::string err;  // guarded by mu
    uint8_t *arena_base = nullptr;
    Arena arena;
    PreparedBuffers prep;  // view-independent precompute of the resident scene
    DevPrepared pdev{};
    std::vector<Slot> slots;
    // shared with client threads
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request> incoming;
    std::deque<fgs_server_result> done;
    std::vector<uint64_t> releases;
    bool stop = false;
    uint64_t next_seq = 0;
    fgs_server_stats st{};   // guarded by mu
    fgs_server_stats wst{};  // the worker's own counters, published into st under mu
    std::thread worker;
    bool worker_failed = false;
};

namespace {

void set_error(fgs_server *srv, const char *msg) {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->err = msg;
}

void drop_graphs(Slot &s) {
    for (GraphEntry &g : s.graphs) (void)hipGraphExecDestroy(g.exec);
    s.graphs.clear();
}

void drop_region(fgs_server *srv, Slot &s) {
    if (!s.has_region) return;
    drop_graphs(s);
    srv->arena.release(s.reg_off, s.reg_bytes);
    s.has_region = false;
    s.reg_bytes = 0;
    s.fb.tk_a = s.fb.tk_b = s.fb.tv_a = s.fb.tv_b = nullptr;
    s.fb.capN = 0;
    srv->wst.region_evictions += 1;
}

void point_pairs(fgs_server *srv, Slot &s) {
    const size_t cap = (s.reg_bytes / 16) / 64 * 64;
    uint32_t *base = reinterpret_cast<uint32_t *>(srv->arena_base + s.reg_off);
    s.fb.tk_a = base;
    s.fb.tk_b = base + cap;
    s.fb.tv_a = base + 2 * cap;
    s.fb.tv_b = base + 3 * cap;
    s.fb.capN = cap;
    s.fb.pairs_owned = false;
}

size_t bytes_for_pairs(size_t N) { return align_up(16 * (N + N / 8 + 4096)); }

// Try to give slot s a region for its pairs and entries (Ncap); evicts cached regions of
// slots that are not blending.  Returns false if the budget cannot hold it now.
bool ensure_region(fgs_server *srv, Slot &s) {
    if (s.has_region && s.reg_bytes / 16 >= s.Ncap + 64) return true;
    const size_t need = bytes_for_pairs(s.Ncap);
    drop_region(srv, s);
    size_t off = 0;
    bool ok = srv->arena.alloc(need, &off);
    for (size_t i = 0; !ok && i < srv->slots.size(); ++i) {
        Slot &o = srv->slots[i];
        if (&o == &s || !o.has_region || o.state == SlotState::BACK || o.spec) continue;
        drop_region(srv, o);
        ok = srv->arena.alloc(need, &off);
    }
    if (!ok) return false;
    s.has_region = true;
    s.reg_off = off;
    s.reg_bytes = need;
    point_pairs(srv, s);
    srv->wst.region_allocs += 1;
    srv->wst.peak_bytes_in_use = std::max<int64_t>(srv->wst.peak_bytes_in_use, (int64_t)srv->arena.used());
    return true;
}

void speculate_back(fgs_server *srv, Slot &s);

void start_front(fgs_server *srv, Slot &s) {
    const DevCamera dcam = to_dev(s.req.cam);
    enqueue_front(srv->dsc, &srv->pdev, dcam, srv->dop, s.req.W, s.req.H, s.fb, s.ch, s.ss, s.fc_dev, s.fc_host,
                  s.stream, s.side, StageMarks{});
    (void)hipEventRecord(s.evA, s.stream);
    s.state = SlotState::FRONT;
    speculate_back(srv, s);
}

// First halves of several requests that start together (each on its own
// slot, any mix of resolutions): one cull keeps the union of their
// candidates and one preprocess pass evaluates every candidate for each
// camera, reading its precompute once (Sec. 5.3.1's unified preprocessing
// across viewpoints); each slot then sorts by depth and scans on its own
// stream.  The union list lives in the first slot's buffers.
void start_front_batch(fgs_server *srv, const std::vector<Slot *> &b) {
    MultiOut mo{};
    mo.n = (int)b.size();
    for (size_t c = 0; c < b.size(); ++c) {
        Slot &s = *b[c];
        CamOut &o = mo.c[c];
        o.cam = to_dev(s.req.cam);
        o.cam64 = to_dev64(s.req.cam, srv->opt, s.req.W, s.req.H);
        o.W = s.req.W;
        o.H = s.req.H;
        o.gs = s.fb.gs;
        o.conic = s.fb.conic;
        o.rect = s.fb.rect;
        o.count = s.fb.count;
        o.count8 = s.fb.count8;
        o.erec = s.fb.erec;
        o.dkey = s.fb.dkey;
        o.gmap = s.fb.gmap;
        o.chunks = s.ch.chunks;
        o.chunk_cap = (uint32_t)std::min<size_t>(s.ch.cap, 0xffffffffu);
        o.fc = s.fc_dev;
        o.gsum_clear = s.ss.slot(0);
    }
    Slot &s0 = *b[0];
    const uint32_t P = (uint32_t)srv->scene.num_gaussians;
    if (P == 0)
        for (Slot *s : b) launch_fill_u32(reinterpret_cast<uint32_t *>(s->fc_dev), 0u, sizeof(FrameCounters) / 4, s0.stream);
    launch_preprocess_multi(srv->dsc, srv->pdev, mo, srv->dop, s0.fb.dv_b, s0.fb.seg_count, s0.fb.gmap, s0.stream);
    (void)hipEventRecord(s0.evP, s0.stream);
    for (size_t c = 0; c < b.size(); ++c) {
        Slot &s = *b[c];
        if (c > 0) (void)hipStreamWaitEvent(s.stream, s0.evP, 0);
        enqueue_front_rest(true, P, srv->dop, s.req.W, s.req.H, s.fb, s.ch, s.ss, s.fc_dev, s.fc_host, s.stream,
                           s.side, StageMarks{});
        (void)hipEventRecord(s.evA, s.stream);
        s.state = SlotState::FRONT;
        speculate_back(srv, s);
    }
    srv->wst.batched_fronts += 1;
    srv->wst.batched_requests += (int64_t)b.size();
}

// Enqueue the second half (and the caller's image copy) on the slot's stream
// and record evB behind it.
hipError_t launch_back(fgs_server *srv, Slot &s) {
    const int W = s.req.W, H = s.req.H;
    const uint32_t P = (uint32_t)srv->scene.num_gaussians;
    if (srv->cfg.use_graphs) {
        hipGraphExec_t exec = nullptr;
        for (GraphEntry &g : s.graphs)
            if (g.W == W && g.H == H) exec = g.exec;
        if (!exec) {
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamBeginCapture(s.stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess) return e;
            enqueue_back(W, H, srv->dop, P, s.fb, s.ch, s.ss, s.fc_dev, s.img, nullptr, nullptr, nullptr, s.stream,
                         StageMarks{});
            e = hipStreamEndCapture(s.stream, &graph);
            if (e != hipSuccess) return e;
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return e;
            s.graphs.push_back(GraphEntry{W, H, exec});
            srv->wst.graphs_captured += 1;
        }
        hipError_t e = hipGraphLaunch(exec, s.stream);
        if (e != hipSuccess) return e;
        srv->wst.graph_launches += 1;
    } else {
        enqueue_back(W, H, srv->dop, P, s.fb, s.ch, s.ss, s.fc_dev, s.img, nullptr, nullptr, nullptr, s.stream,
                     StageMarks{});
    }
    if (s.req.out) {
        const hipError_t c = hipMemcpyAsync(s.req.out, s.img, 3 * (size_t)W * H * sizeof(float),
                                            hipMemcpyDeviceToDevice, s.stream);
        if (c != hipSuccess) return c;
    }
    return hipEventRecord(s.evB, s.stream);
}

hipError_t start_back(fgs_server *srv, Slot &s) {
    const hipError_t e = launch_back(srv, s);
    if (e != hipSuccess) return e;
    s.state = SlotState::BACK;
    return hipSuccess;
}

// Whether a slot's region holds its pairs and entries (the admission criterion
// of ensure_region).
bool region_fits(const Slot &s) { return s.has_region && s.reg_bytes / 16 >= s.Ncap + 64; }

// A slot that kept its pair region from an earlier request enqueues the
// second half right behind the first (as fgs_render does): its kernels read
// the pair count on the device and stay within the region, so no host round
// trip sits between the halves.  If the frame turns out to have more pairs
// than the region holds, the request waits for that half to finish and is
// admitted as usual.
void speculate_back(fgs_server *srv, Slot &s) {
    s.spec = false;
    if (!s.has_region) return;
    if (launch_back(srv, s) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    s.spec = true;
    s.admit_ns = now_ns();
    srv->wst.spec_launches += 1;
}

fgs_server_result make_result(const Slot &s, int32_t status) {
    fgs_server_result r{};
    r.id = s.req.id;
    r.status = status;
    r.width = s.req.W;
    r.height = s.req.H;
    r.slot = s.idx;
    r.rgb = status == FGS_OK ? s.img : nullptr;
    r.arrival_ns = s.req.arrival_ns;
    r.start_ns = s.start_ns;
    r.admit_ns = s.admit_ns;
    r.done_ns = s.done_ns;
    r.visible = s.V;
    r.pairs = s.N;
    return r;
}

void finish(fgs_server *srv, Slot &s, int32_t status) {
    s.done_ns = now_ns();
    const fgs_server_result r = make_result(s, status);
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->done.push_back(r);
        if (status == FGS_OK)
            srv->st.completed += 1;
        else
            srv->st.rejected += 1;
    }
    srv->cv_done.notify_all();
    // a failed request holds no image: its slot is free again at once
    s.state = status == FGS_OK ? SlotState::DONE : SlotState::IDLE;
}

void worker_main(fgs_server *srv) {
    if (hipSetDevice(srv->device) != hipSuccess) {
        srv->worker_failed = true;
        return;
    }
    std::deque<Request> pending;
    const int max_bypass = srv->cfg.max_bypass;
    constexpr int64_t kSpinIdleNs = 50'000'000;  // 50 ms
    int64_t idle_since = now_ns();
    for (;;) {
        bool progress = false;
        bool in_flight = false;
        {
            std::unique_lock<std::mutex> lk(srv->mu);
            for (uint64_t id : srv->releases)
                for (Slot &s : srv->slots)
                    if (s.state == SlotState::DONE && s.req.id == id) s.state = SlotState::IDLE;
            srv->releases.clear();
            while (!srv->incoming.empty()) {
                pending.push_back(srv->incoming.front());
                srv->incoming.pop_front();
            }
            if (srv->stop) {
                // shutting down: queued requests are dropped, finished images
                // are no longer held for the client
                pending.clear();
                for (Slot &s : srv->slots)
                    if (s.state == SlotState::DONE) s.state = SlotState::IDLE;
            }
            for (const Slot &s : srv->slots)
                in_flight |= (s.state == SlotState::FRONT || s.state == SlotState::WAIT || s.state == SlotState::BACK);
            if (srv->stop && pending.empty() && !in_flight) return;
            if (!in_flight && pending.empty()) {
                // idle: keep polling (yielding the core) for a while so a new
                // request starts without a sleep/wake-up delay, then sleep
                if (now_ns() - idle_since > kSpinIdleNs) {
                    srv->cv_work.wait_for(lk, std::chrono::milliseconds(2));
                } else {
                    lk.unlock();
                    std::this_thread::yield();
                }
                continue;
            }
            idle_since = now_ns();
        }
        // 1. start the first half of queued requests on free slots (FIFO); with
        // share_queue = k, beside requests already in flight only while k or
        // more are waiting (a lone request gets the whole GPU)
        int active = 0;
        for (const Slot &s : srv->slots)
            active += (s.state == SlotState::FRONT || s.state == SlotState::WAIT || s.state == SlotState::BACK);
        std::vector<Slot *> starting;
        for (Slot &s : srv->slots) {
            if (pending.empty() || (int)starting.size() == kMaxCams) break;
            if (s.state != SlotState::IDLE) continue;
            const int k = srv->cfg.share_queue;
            if (active > 0 && k > 0 && (int64_t)pending.size() < (int64_t)k) break;
            ++active;
            s.req = pending.front();
            pending.pop_front();
            s.attempts = 0;
            s.bypassed = 0;
            s.start_ns = now_ns();
            starting.push_back(&s);
        }
        // requests that start together share one cull and preprocess pass
        if (starting.size() == 1 || (starting.size() > 1 && !srv->cfg.batch_fronts)) {
            for (Slot *s : starting) start_front(srv, *s);
        } else if (starting.size() > 1) {
            start_front_batch(srv, starting);
        }
        progress |= !starting.empty();
        // 2. first halves that finished: their pair counts are known
        for (Slot &s : srv->slots) {
            if (s.state != SlotState::FRONT) continue;
            const hipError_t q = hipEventQuery(s.evA);
            if (q == hipErrorNotReady) continue;
            progress = true;
            if (q != hipSuccess) {
                set_error(srv, hipGetErrorString(q));
                s.spec = false;
                finish(srv, s, FGS_ERR_DEVICE);
                continue;
            }
            if ((s.fc_host->error & kErrChunkOverflow) && s.attempts == 0) {
                // large-Gaussian chunk list too small: grow it (its graphs
                // reference it) and run the first half again
                s.attempts += 1;
                if (s.spec) (void)hipEventSynchronize(s.evB);  // that half reads the chunk list
                s.spec = false;
                drop_graphs(s);
                if (ensure_chunks(s.ch, (size_t)s.fc_host->nchunks + (size_t)s.fc_host->nchunks / 8) != hipSuccess) {
                    finish(srv, s, FGS_ERR_OUT_OF_MEMORY);
                    continue;
                }
                start_front(srv, s);
                continue;
            }
            if (s.fc_host->error & kErrChunkOverflow) {
                if (s.spec) (void)hipEventSynchronize(s.evB);
                s.spec = false;
                finish(srv, s, FGS_ERR_INTERNAL);
                continue;
            }
            s.V = s.fc_host->visible;
            s.N = s.fc_host->pairs;
            s.Ncap = pair_capacity_needed(s.N, s.fc_host->entries, s.req.W, s.req.H);
            if (s.spec && region_fits(s)) {
                // the second half enqueued with the first holds every pair
                s.spec = false;
                s.state = SlotState::BACK;
                continue;
            }
            if (bytes_for_pairs(s.Ncap) > srv->arena.size()) {
                if (s.spec) (void)hipEventSynchronize(s.evB);  // the region is in use until then
                s.spec = false;
                finish(srv, s, FGS_ERR_CAPACITY);  // can never fit the budget
                continue;
            }
            if (s.spec) srv->wst.spec_misses += 1;
            s.state = SlotState::WAIT;
        }
        // 3. admission: FIFO over waiting requests, bounded bypass
        {
            std::vector<Slot *> waiting;
            for (Slot &s : srv->slots)
                if (s.state == SlotState::WAIT) waiting.push_back(&s);
            std::sort(waiting.begin(), waiting.end(), [](Slot *a, Slot *b) { return a->req.seq < b->req.seq; });
            auto try_admit = [&](Slot *s) {
                if (s->spec) {
                    // its speculative second half ran out of pairs: the
                    // region is free to grow once that half has finished
                    const hipError_t q = hipEventQuery(s->evB);
                    if (q == hipErrorNotReady) return false;
                    s->spec = false;
                }
                if (!ensure_region(srv, *s)) return false;
                s->admit_ns = now_ns();
                const hipError_t e = start_back(srv, *s);
                progress = true;
                if (e != hipSuccess) {
                    set_error(srv, hipGetErrorString(e));
                    finish(srv, *s, FGS_ERR_DEVICE);
                }
                return true;
            };
            auto bypassed = [](Slot *s) -> int & { return s->bypassed; };
            (void)admit_fifo_bounded_bypass(waiting, max_bypass, try_admit, bypassed, &srv->wst.bypasses);
        }
        // 4. completed images
        for (Slot &s : srv->slots) {
            if (s.state != SlotState::BACK) continue;
            const hipError_t q = hipEventQuery(s.evB);
            if (q == hipErrorNotReady) continue;
            progress = true;
            if (q != hipSuccess) set_error(srv, hipGetErrorString(q));
            finish(srv, s, q == hipSuccess ? FGS_OK : FGS_ERR_DEVICE);
        }
        if (progress) {
            std::lock_guard<std::mutex> lk(srv->mu);
            srv->st.graphs_captured = srv->wst.graphs_captured;
            srv->st.graph_launches = srv->wst.graph_launches;
            srv->st.region_allocs = srv->wst.region_allocs;
            srv->st.region_evictions = srv->wst.region_evictions;
            srv->st.bypasses = srv->wst.bypasses;
            srv->st.peak_bytes_in_use = srv->wst.peak_bytes_in_use;
            srv->st.batched_fronts = srv->wst.batched_fronts;
            srv->st.batched_requests = srv->wst.batched_requests;
            srv->st.spec_launches = srv->wst.spec_launches;
            srv->st.spec_misses = srv->wst.spec_misses;
        } else if (in_flight) {
            std::this_thread::yield();  // completions are polled: stay on the core
        } else {
            // queued work waits for a slot to be released
            std::unique_lock<std::mutex> lk(srv->mu);
            srv->cv_work.wait_for(lk, std::chrono::milliseconds(1));
        }
    }
}

fgs_status server_fail(fgs_server *srv, fgs_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (srv) set_error(srv, buf);
    return s;
}

thread_local std::string g_server_error_copy;

void free_server(fgs_server *srv) {
    (void)hipSetDevice(srv->device);
    (void)hipDeviceSynchronize();
    for (Slot &s : srv->slots) {
        drop_graphs(s);
        s.fb.tk_a = s.fb.tk_b = s.fb.tv_a = s.fb.tv_b = nullptr;  // arena-owned
        free_frame_buffers(s.fb);
        free_chunks(s.ch);
        free_sort_scratch(s.ss);
        if (s.fc_dev) (void)hipFree(s.fc_dev);
        if (s.fc_host) (void)hipHostFree(s.fc_host);
        if (s.img) (void)hipFree(s.img);
        if (s.evA) (void)hipEventDestroy(s.evA);
        if (s.evB) (void)hipEventDestroy(s.evB);
        if (s.evP) (void)hipEventDestroy(s.evP);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        s.side.destroy();
    }
    if (srv->arena_base) (void)hipFree(srv->arena_base);
    free_prepared(srv->prep);
    delete srv;
}

}  // namespace

extern "C" {

int64_t fgs_clock_ns(void) { return now_ns(); }

fgs_status fgs_server_create(int device, const fgs_scene *scene, const fgs_options *opt,
                             const fgs_server_config *cfg, fgs_server **out) {
    if (!out) return FGS_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    if (!cfg) return FGS_ERR_INVALID_ARGUMENT;
    if (cfg->budget_bytes < (1 << 20) || cfg->max_inflight < 1 || cfg->max_inflight > 32 || cfg->max_width < 1 ||
        cfg->max_width > 16384 || cfg->max_height < 1 || cfg->max_height > 16384 || cfg->max_bypass < 0 ||
        cfg->share_queue < 0 || (cfg->batch_fronts != 0 && cfg->batch_fronts != 1))
        return FGS_ERR_INVALID_ARGUMENT;
    fgs_camera probe{};
    for (int i = 0; i < 3; ++i) probe.R[4 * i] = 1.0f;
    probe.fx = probe.fy = 1.0f;
    probe.near_z = 0.2f;
    std::string m;
    if (check_args(scene, &probe, cfg->max_width, cfg->max_height, opt, m) != FGS_OK) return FGS_ERR_INVALID_ARGUMENT;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return FGS_ERR_DEVICE;
    if (hipSetDevice(device) != hipSuccess) return FGS_ERR_DEVICE;

    fgs_server *srv = new fgs_server();
    srv->device = device;
    srv->scene = *scene;
    srv->dsc = to_dev(*scene);
    if (opt)
        srv->opt = *opt;
    else
        fgs_default_options(&srv->opt);
    srv->dop = to_dev(srv->opt);
    srv->cfg = *cfg;
    srv->st.budget_bytes = cfg->budget_bytes;
    // occupancy queries happen outside any graph capture
    (void)preprocess_grid(1);
    (void)emit_grid(1);

    const size_t P = (size_t)scene->num_gaussians;
    const size_t tiles =
        (size_t)((cfg->max_width + kTile - 1) / kTile) * (size_t)((cfg->max_height + kTile - 1) / kTile);
    const size_t pix = (size_t)cfg->max_width * cfg->max_height;
    hipError_t e = hipMalloc((void **)&srv->arena_base, (size_t)cfg->budget_bytes);
    if (e == hipSuccess) e = build_prepared(*scene, srv->opt, srv->prep, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    srv->pdev = srv->prep.dev();
    srv->arena.init((size_t)cfg->budget_bytes);
    srv->slots.resize((size_t)cfg->max_inflight);
    size_t slot_bytes = 0;
    for (int i = 0; i < cfg->max_inflight && e == hipSuccess; ++i) {
        Slot &s = srv->slots[(size_t)i];
        s.idx = i;
        // default priority (no priority streams)
        if ((e = hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking)) != hipSuccess) break;
        if ((e = hipEventCreateWithFlags(&s.evA, hipEventDisableTiming)) != hipSuccess) break;
        if ((e = hipEventCreateWithFlags(&s.evB, hipEventDisableTiming)) != hipSuccess) break;
        if ((e = hipEventCreateWithFlags(&s.evP, hipEventDisableTiming)) != hipSuccess) break;
        if ((e = s.side.create()) != hipSuccess) break;
        if ((e = ensure_gauss(s.fb, P)) != hipSuccess) break;
        if ((e = ensure_tiles(s.fb, tiles)) != hipSuccess) break;
        if ((e = ensure_chunks(s.ch, P / 8)) != hipSuccess) break;
        if ((e = ensure_sort_scratch(s.ss)) != hipSuccess) break;
        if ((e = hipMalloc((void **)&s.fc_dev, sizeof(FrameCounters))) != hipSuccess) break;
        if ((e = hipHostMalloc((void **)&s.fc_host, sizeof(FrameCounters), hipHostMallocDefault)) != hipSuccess) break;
        if ((e = hipMalloc((void **)&s.img, 3 * pix * sizeof(float))) != hipSuccess) break;
        s.fb.pairs_owned = false;
        slot_bytes += s.fb.bytes() + s.ch.bytes() + SortScratch::bytes() + 3 * pix * sizeof(float);
    }
    if (e != hipSuccess) {
        free_server(srv);
        return e == hipErrorOutOfMemory ? FGS_ERR_OUT_OF_MEMORY : FGS_ERR_DEVICE;
    }
    srv->st.slot_bytes = (int64_t)(slot_bytes + srv->prep.bytes());
    srv->worker = std::thread(worker_main, srv);
    *out = srv;
    return FGS_OK;
}

void fgs_server_destroy(fgs_server *srv) {
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
        // images still held by the client are released at shutdown
        for (Slot &s : srv->slots)
            if (s.state == SlotState::DONE) srv->releases.push_back(s.req.id);
    }
    srv->cv_work.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    free_server(srv);
}

const char *fgs_server_last_error(const fgs_server *srv) {
    if (!srv) return "server is NULL";
    fgs_server *m = const_cast<fgs_server *>(srv);
    std::lock_guard<std::mutex> lk(m->mu);
    g_server_error_copy = m->err;  // stable for the calling thread
    return g_server_error_copy.c_str();
}

fgs_status fgs_server_submit(fgs_server *srv, uint64_t id, const fgs_camera *cam, int32_t W, int32_t H,
                             int64_t arrival_ns, float *out_rgb) {
    if (!srv) return FGS_ERR_INVALID_ARGUMENT;
    std::string m;
    if (check_args(&srv->scene, cam, W, H, &srv->opt, m) != FGS_OK)
        return server_fail(srv, FGS_ERR_INVALID_ARGUMENT, "%s", m.c_str());
    if (W > srv->cfg.max_width || H > srv->cfg.max_height)
        return server_fail(srv, FGS_ERR_INVALID_ARGUMENT, "request %dx%d exceeds the server's %dx%d", W, H,
                           srv->cfg.max_width, srv->cfg.max_height);
    if (srv->worker_failed) return server_fail(srv, FGS_ERR_DEVICE, "worker thread could not start");
    Request r;
    r.id = id;
    r.cam = *cam;
    r.W = W;
    r.H = H;
    r.arrival_ns = arrival_ns;
    r.out = out_rgb;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) {
            srv->err = "server is stopping";
            return FGS_ERR_INVALID_ARGUMENT;
        }
        r.seq = srv->next_seq++;
        srv->incoming.push_back(r);
        srv->st.submitted += 1;
    }
    srv->cv_work.notify_one();
    return FGS_OK;
}

int32_t fgs_server_poll(fgs_server *srv, fgs_server_result *out, int32_t max, int64_t wait_ns) {
    if (!srv || (!out && max > 0) || max < 0) return -(int32_t)FGS_ERR_INVALID_ARGUMENT;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->done.empty() && wait_ns > 0)
        srv->cv_done.wait_for(lk, std::chrono::nanoseconds(wait_ns), [&] { return !srv->done.empty(); });
    int32_t k = 0;
    while (k < max && !srv->done.empty()) {
        out[k++] = srv->done.front();
        srv->done.pop_front();
    }
    return k;
}

fgs_status fgs_server_release(fgs_server *srv, uint64_t id) {
    if (!srv) return FGS_ERR_INVALID_ARGUMENT;
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->releases.push_back(id);
    }
    srv->cv_work.notify_one();
    return FGS_OK;
}

fgs_status fgs_server_get_stats(fgs_server *srv, fgs_server_stats *out) {
    if (!srv || !out) return FGS_ERR_INVALID_ARGUMENT;
    std::lock_guard<std::mutex> lk(srv->mu);
    *out = srv->st;
    return FGS_OK;
}

fgs_status fgs_server_replay(fgs_server *srv, const fgs_trace_request *trace, int64_t n,
                             fgs_server_result *results) {
    if (!srv || (n > 0 && (!trace || !results)) || n < 0) return FGS_ERR_INVALID_ARGUMENT;
    std::map<uint64_t, int64_t> index;
    for (int64_t i = 0; i < n; ++i) {
        if (!index.emplace(trace[i].id, i).second)
            return server_fail(srv, FGS_ERR_INVALID_ARGUMENT, "duplicate request id in the trace");
        if (i > 0 && trace[i].arrival_offset_ns < trace[i - 1].arrival_offset_ns)
            return server_fail(srv, FGS_ERR_INVALID_ARGUMENT, "trace arrivals are not in order");
    }
    const int64_t t0 = now_ns() + 1000000;  // 1 ms to set up
    int64_t next = 0, got = 0;
    std::vector<fgs_server_result> buf(64);
    while (got < n) {
        const int64_t t = now_ns();
        while (next < n && t0 + trace[next].arrival_offset_ns <= t) {
            const fgs_trace_request &q = trace[next];
            const fgs_status s =
                fgs_server_submit(srv, q.id, &q.cam, q.width, q.height, t0 + q.arrival_offset_ns, nullptr);
            if (s != FGS_OK) return s;
            ++next;
        }
        // sleep until shortly before the next arrival (a timed wait wakes up
        // late by tens of microseconds), then poll without waiting so that
        // the request is submitted at its arrival time
        constexpr int64_t kSlack = 150000;
        int64_t wait = 0;
        if (next < n) wait = std::max<int64_t>(0, t0 + trace[next].arrival_offset_ns - now_ns() - kSlack);
        else wait = 5000000;
        wait = std::min<int64_t>(wait, 200000);  // stay responsive to arrivals
        const int32_t k = fgs_server_poll(srv, buf.data(), (int32_t)buf.size(), wait);
        if (k == 0 && wait == 0) std::this_thread::yield();
        if (k < 0) return (fgs_status)(-k);
        for (int32_t j = 0; j < k; ++j) {
            auto it = index.find(buf[(size_t)j].id);
            if (it == index.end()) continue;  // not from this trace
            results[it->second] = buf[(size_t)j];
            results[it->second].rgb = nullptr;  // released at once
            if (buf[(size_t)j].status == FGS_OK) (void)fgs_server_release(srv, buf[(size_t)j].id);
            ++got;
        }
    }
    return FGS_OK;
}

}  // extern "C"

namespace {

// The plain renderer's replay: each request at its arrival time, one at a
// time in arrival order, waiting for each frame before the next (completion
// observed by polling an event, as the server's worker does).  render(q, st)
// renders request q into the caller's scratch image.
template <class Render>
fgs_status replay_plain_impl(const fgs_trace_request *trace, int64_t n, fgs_server_result *results, void *stream,
                             Render render) {
    for (int64_t i = 1; i < n; ++i)
        if (trace[i].arrival_offset_ns < trace[i - 1].arrival_offset_ns) return FGS_ERR_INVALID_ARGUMENT;
    hipEvent_t done = nullptr;
    if (hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) return FGS_ERR_DEVICE;
    struct EventGuard {
        hipEvent_t e;
        ~EventGuard() { (void)hipEventDestroy(e); }
    } guard{done};
    const int64_t t0 = now_ns() + 1000000;
    for (int64_t i = 0; i < n; ++i) {
        const fgs_trace_request &q = trace[i];
        const int64_t arrive = t0 + q.arrival_offset_ns;
        while (now_ns() < arrive) std::this_thread::yield();
        fgs_server_result &r = results[i];
        r = fgs_server_result{};
        r.id = q.id;
        r.width = q.width;
        r.height = q.height;
        r.slot = 0;
        r.arrival_ns = arrive;
        r.start_ns = now_ns();
        fgs_stats stt{};
        fgs_status s = render(q, &stt);
        r.admit_ns = now_ns();  // the render call returns once the second half is enqueued
        if (s == FGS_OK) {
            hipError_t q2 = hipEventRecord(done, (hipStream_t)stream);
            if (q2 == hipSuccess)
                while ((q2 = hipEventQuery(done)) == hipErrorNotReady) {
                }
            if (q2 != hipSuccess) s = FGS_ERR_DEVICE;
        }
        r.done_ns = now_ns();
        r.status = s;
        r.visible = stt.visible;
        r.pairs = stt.pairs;
        if (s != FGS_OK) return s;
    }
    return FGS_OK;
}

}  // namespace

extern "C" {

fgs_status fgs_replay_plain(fgs_context *ctx, const fgs_scene *scene, const fgs_options *opt,
                            const fgs_trace_request *trace, int64_t n, float *rgb_scratch,
                            fgs_server_result *results, void *stream) {
    if (!ctx || (n > 0 && (!trace || !results || !rgb_scratch)) || n < 0) return FGS_ERR_INVALID_ARGUMENT;
    return replay_plain_impl(trace, n, results, stream, [&](const fgs_trace_request &q, fgs_stats *st) {
        return fgs_render(ctx, scene, &q.cam, q.width, q.height, opt, rgb_scratch, nullptr, nullptr, nullptr, st,
                          stream);
    });
}

fgs_status fgs_replay_plain_prepared(fgs_context *ctx, const fgs_prepared *prepared, const fgs_options *opt,
                                     const fgs_trace_request *trace, int64_t n, float *rgb_scratch,
                                     fgs_server_result *results, void *stream) {
    if (!ctx || !prepared || (n > 0 && (!trace || !results || !rgb_scratch)) || n < 0)
        return FGS_ERR_INVALID_ARGUMENT;
    return replay_plain_impl(trace, n, results, stream, [&](const fgs_trace_request &q, fgs_stats *st) {
        return fgs_render_prepared(ctx, prepared, &q.cam, q.width, q.height, opt, rgb_scratch, nullptr, nullptr,
                                   nullptr, st, stream);
    });
}

}  // extern "C"
