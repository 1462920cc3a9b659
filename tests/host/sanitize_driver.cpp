// Host-side checks of the runtime under AddressSanitizer and UBSan (built
// without the kernel files; see launch_stubs.cpp).  Exercises the C ABI's
// argument validation and error paths on a machine without a GPU, and the
// server's admission arena under a long random alloc/free sequence checked
// against a granule map.  Prints "sanitize ok" and exits 0 when every check
// holds; a sanitizer report or a failed check exits non-zero.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <random>
#include <string>
#include <vector>

#include "arena.hpp"
#include "fgs.h"

namespace {

int failures = 0;

void check(bool ok, const char *what) {
    if (!ok) {
        std::fprintf(stderr, "FAILED: %s\n", what);
        ++failures;
    }
}

struct Planes {
    std::vector<float> buf = std::vector<float>(64, 0.0f);
};

fgs_scene valid_scene(Planes &p) {
    fgs_scene s{};
    s.num_gaussians = 4;
    s.plane_stride = 4;
    s.sh_degree = 0;
    s.means = p.buf.data();
    s.log_scales = p.buf.data() + 12;
    s.quats = p.buf.data() + 24;
    s.opacity_logits = p.buf.data() + 40;
    s.sh = p.buf.data() + 44;
    return s;
}

fgs_camera valid_camera() {
    fgs_camera c{};
    c.R[0] = c.R[4] = c.R[8] = 1.0f;
    c.fx = c.fy = 100.0f;
    c.cx = c.cy = 32.0f;
    c.near_z = 0.2f;
    return c;
}

void validation() {
    Planes p;
    fgs_options o;
    fgs_default_options(&o);
    fgs_scene s = valid_scene(p);
    fgs_camera c = valid_camera();
    check(fgs_validate(&s, &c, 64, 64, &o) == FGS_OK, "valid arguments accepted");
    check(fgs_validate(&s, &c, 64, 64, nullptr) == FGS_OK, "NULL options mean defaults");

    struct Case {
        const char *name;
        void (*mutate)(fgs_scene &, fgs_camera &, fgs_options &, int &, int &);
    };
    const Case cases[] = {
        {"P < 0", [](fgs_scene &s, fgs_camera &, fgs_options &, int &, int &) { s.num_gaussians = -1; }},
        {"stride < P", [](fgs_scene &s, fgs_camera &, fgs_options &, int &, int &) { s.plane_stride = 3; }},
        {"sh degree 4", [](fgs_scene &s, fgs_camera &, fgs_options &, int &, int &) { s.sh_degree = 4; }},
        {"sh degree -1", [](fgs_scene &s, fgs_camera &, fgs_options &, int &, int &) { s.sh_degree = -1; }},
        {"reserved != 0", [](fgs_scene &s, fgs_camera &, fgs_options &, int &, int &) { s.reserved = 1; }},
        {"null means", [](fgs_scene &s, fgs_camera &, fgs_options &, int &, int &) { s.means = nullptr; }},
        {"null sh", [](fgs_scene &s, fgs_camera &, fgs_options &, int &, int &) { s.sh = nullptr; }},
        {"W = 0", [](fgs_scene &, fgs_camera &, fgs_options &, int &W, int &) { W = 0; }},
        {"H = 16385", [](fgs_scene &, fgs_camera &, fgs_options &, int &, int &H) { H = 16385; }},
        {"NaN rotation", [](fgs_scene &, fgs_camera &c, fgs_options &, int &, int &) { c.R[3] = NAN; }},
        {"inf eye", [](fgs_scene &, fgs_camera &c, fgs_options &, int &, int &) { c.eye[1] = INFINITY; }},
        {"fx = 0", [](fgs_scene &, fgs_camera &c, fgs_options &, int &, int &) { c.fx = 0.0f; }},
        {"fy < 0", [](fgs_scene &, fgs_camera &c, fgs_options &, int &, int &) { c.fy = -1.0f; }},
        {"near = 0", [](fgs_scene &, fgs_camera &c, fgs_options &, int &, int &) { c.near_z = 0.0f; }},
        {"alpha_min = 1", [](fgs_scene &, fgs_camera &, fgs_options &o, int &, int &) { o.alpha_min = 1.0f; }},
        {"T_stop < 0", [](fgs_scene &, fgs_camera &, fgs_options &o, int &, int &) { o.T_stop = -1e-4f; }},
        {"alpha_max NaN", [](fgs_scene &, fgs_camera &, fgs_options &o, int &, int &) { o.alpha_max = NAN; }},
        {"dilation inf", [](fgs_scene &, fgs_camera &, fgs_options &o, int &, int &) { o.dilation = INFINITY; }},
        {"jac_clip 0", [](fgs_scene &, fgs_camera &, fgs_options &o, int &, int &) { o.jac_clip = 0.0f; }},
        {"bg NaN", [](fgs_scene &, fgs_camera &, fgs_options &o, int &, int &) { o.bg[2] = NAN; }},
        {"binning 3", [](fgs_scene &, fgs_camera &, fgs_options &o, int &, int &) { o.binning = 3; }},
    };
    for (const Case &k : cases) {
        fgs_scene s2 = valid_scene(p);
        fgs_camera c2 = valid_camera();
        fgs_options o2 = o;
        int W = 64, H = 64;
        k.mutate(s2, c2, o2, W, H);
        const fgs_status st = fgs_validate(&s2, &c2, W, H, &o2);
        check(st == FGS_ERR_INVALID_ARGUMENT, k.name);
        check(std::strlen(fgs_last_error(nullptr)) > 0, "error text for a rejected argument");
    }
    check(fgs_validate(nullptr, &c, 64, 64, &o) == FGS_ERR_INVALID_ARGUMENT, "NULL scene");
    check(fgs_validate(&s, nullptr, 64, 64, &o) == FGS_ERR_INVALID_ARGUMENT, "NULL camera");
    fgs_scene empty = s;
    empty.num_gaussians = 0;
    empty.plane_stride = 0;
    empty.means = empty.log_scales = empty.quats = empty.opacity_logits = empty.sh = nullptr;
    check(fgs_validate(&empty, &c, 1, 1, &o) == FGS_OK, "an empty scene needs no planes");
}

void error_paths() {
    for (int s = 0; s <= 6; ++s) check(std::strlen(fgs_status_string((fgs_status)s)) > 0, "status text");
    check(std::strlen(fgs_status_string((fgs_status)99)) > 0, "unknown status text");
    fgs_context *ctx = reinterpret_cast<fgs_context *>(0x1);
    const fgs_status cs = fgs_create(0, &ctx);
    // no GPU here: the device check fails and no context is handed out
    check(cs == FGS_ERR_DEVICE || cs == FGS_OK, "fgs_create reports a missing device");
    if (cs == FGS_OK) {
        fgs_destroy(ctx);
    } else {
        check(ctx == nullptr, "no context on failure");
    }
    check(fgs_create(0, nullptr) == FGS_ERR_INVALID_ARGUMENT, "fgs_create with NULL out");
    check(fgs_create(-1, &ctx) != FGS_OK, "negative device");
    fgs_destroy(nullptr);
    check(fgs_scratch_bytes(nullptr) == 0, "scratch bytes of NULL");
    check(fgs_reserve(nullptr, 1, 1, 1, 1) == FGS_ERR_INVALID_ARGUMENT, "reserve without a context");
    Planes p;
    fgs_scene s = valid_scene(p);
    fgs_camera c = valid_camera();
    float dummy = 0.0f;
    check(fgs_render(nullptr, &s, &c, 8, 8, nullptr, &dummy, nullptr, nullptr, nullptr, nullptr, nullptr) ==
              FGS_ERR_INVALID_ARGUMENT,
          "render without a context");
    fgs_frame *fr = reinterpret_cast<fgs_frame *>(0x1);
    check(fgs_render(nullptr, &s, &c, 8, 8, nullptr, &dummy, nullptr, nullptr, &fr, nullptr, nullptr) ==
                  FGS_ERR_INVALID_ARGUMENT &&
              fr == nullptr,
          "saved frame cleared on failure");
    int64_t pairs = 7;
    size_t bytes = 7;
    check(fgs_plan(nullptr, &s, &c, 8, 8, nullptr, &pairs, &bytes, nullptr) == FGS_ERR_INVALID_ARGUMENT &&
              pairs == 0 && bytes == 0,
          "plan without a context");
    fgs_prepared *pr = reinterpret_cast<fgs_prepared *>(0x1);
    check(fgs_prepare_scene(nullptr, &s, nullptr, &pr, nullptr) == FGS_ERR_INVALID_ARGUMENT && pr == nullptr,
          "prepare without a context");
    check(fgs_prepared_release(nullptr, nullptr) == FGS_OK, "release of a NULL prepared scene");
    check(fgs_frame_release(nullptr, nullptr) == FGS_OK, "release of a NULL frame");
    check(fgs_set_instrumentation(nullptr, 0) == FGS_ERR_INVALID_ARGUMENT, "instrumentation without a context");
    check(fgs_set_blend_variant(nullptr, 0) == FGS_ERR_INVALID_ARGUMENT, "blend variant without a context");
    fgs_timings t{};
    check(fgs_get_instrumentation(nullptr, &t) == FGS_ERR_INVALID_ARGUMENT, "timings without a context");
    check(fgs_frame_stats(nullptr, nullptr) == FGS_ERR_INVALID_ARGUMENT, "stats of a NULL frame");
    check(fgs_frame_field_bytes(nullptr, FGS_FIELD_GAUSS) == 0, "field bytes of a NULL frame");
    check(fgs_render_backward(nullptr, nullptr, &s, &c, nullptr, nullptr, nullptr, nullptr) ==
              FGS_ERR_INVALID_ARGUMENT,
          "backward without a context");
    check(fgs_render_prepared_batch(nullptr, nullptr, &c, 1, 8, 8, nullptr, nullptr, nullptr, nullptr, nullptr,
                                    nullptr) == FGS_ERR_INVALID_ARGUMENT,
          "batch without a context");

    // server: configuration checks come before any device call
    fgs_server_config cfg{};
    cfg.budget_bytes = 64 << 20;
    cfg.max_inflight = 2;
    cfg.max_width = 64;
    cfg.max_height = 64;
    cfg.max_bypass = 1;
    cfg.use_graphs = 1;
    cfg.share_queue = 0;
    fgs_server *srv = reinterpret_cast<fgs_server *>(0x1);
    check(fgs_server_create(0, &s, nullptr, nullptr, &srv) == FGS_ERR_INVALID_ARGUMENT && srv == nullptr,
          "server without a configuration");
    const fgs_server_config base = cfg;
    auto bad_cfg = [&](void (*m)(fgs_server_config &), const char *what) {
        fgs_server_config k = base;
        m(k);
        check(fgs_server_create(0, &s, nullptr, &k, &srv) == FGS_ERR_INVALID_ARGUMENT, what);
    };
    bad_cfg([](fgs_server_config &k) { k.budget_bytes = 1000; }, "server budget below 1 MiB");
    bad_cfg([](fgs_server_config &k) { k.max_inflight = 0; }, "server without slots");
    bad_cfg([](fgs_server_config &k) { k.max_inflight = 33; }, "server with 33 slots");
    bad_cfg([](fgs_server_config &k) { k.max_width = 16385; }, "server width");
    bad_cfg([](fgs_server_config &k) { k.max_bypass = -1; }, "server bypass");
    bad_cfg([](fgs_server_config &k) { k.share_queue = -1; }, "server share threshold");
    bad_cfg([](fgs_server_config &k) { k.batch_fronts = 2; }, "server batching flag");
    Planes bad;
    fgs_scene bs = valid_scene(bad);
    bs.sh_degree = 9;
    check(fgs_server_create(0, &bs, nullptr, &cfg, &srv) == FGS_ERR_INVALID_ARGUMENT, "server scene check");
    const fgs_status ss = fgs_server_create(0, &s, nullptr, &cfg, &srv);
    check(ss == FGS_ERR_DEVICE || ss == FGS_OK, "server without a device");
    if (ss == FGS_OK) fgs_server_destroy(srv);
    fgs_server_destroy(nullptr);
    check(fgs_clock_ns() > 0, "monotonic clock");
}

void arena() {
    // random first-fit traffic, checked against a map of 256-byte granules
    const size_t size = (size_t)1 << 22;
    fgs::Arena a;
    a.init(size + 100);  // rounded down to the alignment
    check(a.size() == size, "arena size rounded to the alignment");
    std::vector<int> owner(size / fgs::kArenaAlign, -1);
    std::map<int, std::pair<size_t, size_t>> live;  // id -> (offset, requested bytes)
    std::mt19937_64 rng(12345);
    int next_id = 0;
    size_t used = 0;
    for (int step = 0; step < 200000; ++step) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const size_t req = (rng() % 4 == 0) ? 0 : (size_t)(rng() % 70000);
            size_t off = 0;
            const size_t g = (fgs::arena_align(req) ? fgs::arena_align(req) : fgs::kArenaAlign) / fgs::kArenaAlign;
            if (a.alloc(req, &off)) {
                check(off % fgs::kArenaAlign == 0 && off + g * fgs::kArenaAlign <= size, "allocation in range");
                for (size_t i = 0; i < g; ++i) {
                    if (owner[off / fgs::kArenaAlign + i] != -1) {
                        check(false, "allocations overlap");
                        break;
                    }
                    owner[off / fgs::kArenaAlign + i] = next_id;
                }
                live[next_id++] = {off, req};
                used += g * fgs::kArenaAlign;
            } else {
                // first fit failed: no free run of g granules may exist
                size_t run = 0, best = 0;
                for (int o : owner) {
                    run = (o == -1) ? run + 1 : 0;
                    best = std::max(best, run);
                }
                check(best < g, "first fit missed a free range");
                check(a.largest_free() < g * fgs::kArenaAlign, "largest free range consistent");
            }
        } else {
            auto it = live.begin();
            std::advance(it, (long)(rng() % live.size()));
            const size_t g = (fgs::arena_align(it->second.second) ? fgs::arena_align(it->second.second)
                                                                  : fgs::kArenaAlign) /
                             fgs::kArenaAlign;
            for (size_t i = 0; i < g; ++i) owner[it->second.first / fgs::kArenaAlign + i] = -1;
            a.release(it->second.first, it->second.second);
            used -= g * fgs::kArenaAlign;
            live.erase(it);
        }
        check(a.used() == used, "used bytes tracked");
        if (failures) return;
    }
    for (auto &kv : live) a.release(kv.second.first, kv.second.second);
    check(a.used() == 0 && a.free_ranges() == 1 && a.largest_free() == size, "arena coalesces back to one range");

    // bounded bypass: the head never fits; later requests overtake it at most twice
    std::vector<int> waiting = {0, 1, 2, 3, 4};
    std::vector<int> counters(5, 0);
    int64_t bypasses = 0;
    const int n = fgs::admit_fifo_bounded_bypass(
        waiting, 2, [](int w) { return w != 0; }, [&](int w) -> int & { return counters[(size_t)w]; }, &bypasses);
    check(n == 2 && bypasses == 2 && counters[0] == 2, "bounded bypass admits two later requests");
}

}  // namespace

int main() {
    validation();
    error_paths();
    arena();
    if (failures) {
        std::fprintf(stderr, "%d checks failed\n", failures);
        return 1;
    }
    std::printf("sanitize ok\n");
    return 0;
}
