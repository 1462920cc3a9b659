#!/usr/bin/env python3
"""Benchmark of the renderer on one MI355X.

Default workload: the 10,000,000-Gaussian ground-plane scene (SH degree 3)
rendered at 3840x2160 through the camera at 80 m altitude pitched 30 deg
down (synthetic stand-in for the paper's large-scale aerial 4K case).
A step is one full frame through the C ABI: cull, preprocess with the exact
ellipse/tile test, depth sort, count scan, key emission (super-tile
entries), their sort by super-tile, the per-tile lists and ranges, and
blending, with the scene already resident in HBM together with
its view-independent precompute (opacity, scales and rotation, extent, and
SH coefficients Gaussian-major; built once, Sec. 5.3.1).  The frame rate
from the raw parameters is reported beside it.

Prints one JSON line: frames/s, per-stage times and roofline fractions
(HIP events on the render stream; the dominant kernel in `roofline`), the
image against the binary64 oracle with a pass flag, the CPU oracle timed on
the host, the other workloads (10k at 256x256, 1M at 1080p through eight
cameras, the 8K stress case), the multi-camera batch, the serving workload
(batched server against the plain renderer on the same resident scene) and
the forward + backward timing.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "4K frames/s (10M Gaussians); served p50/p99 latency vs plain renderer"
WORKLOADS = {
    "city4k": dict(kind="city", W=3840, H=2160, name="city-10M-gaussians-3840x2160"),
    "city8k": dict(kind="city", W=7680, H=4320, name="city-10M-gaussians-7680x4320"),
    "medium": dict(kind="medium", W=1920, H=1080, name="medium-1M-gaussians-1920x1080"),
    "small": dict(kind="small", W=256, H=256, name="small-10k-gaussians-256x256"),
}
HBM_PEAK_GBS = 8000.0
# FP32 vector issue of MI355X: the published 157.3 TFLOP/s counts packed FMAs
# (two lanes' worth and two FLOP per instruction slot of a lane); one
# non-packed FP32 instruction slot per lane is a quarter of it, 39.3 T
# lane-slots/s (256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz).  An add, multiply or
# FMA takes one slot; v_exp_f32 issues at half rate (two slots, measured by
# fgs_measure_peaks).
VALU_PEAK_TSLOTS = 157.3 / 4
# FP32 slots the blend spends per (pixel, Gaussian) evaluation in its
# two-pixels-per-lane form: 10.6 add / multiply / FMA instructions (the
# kernel's instruction mix, SQ_INSTS_VALU_{ADD,MUL,FMA}_F32 per executed
# step of 128 pixel evaluations, committed under profiles/) and one
# v_exp_f32 at two slots
BLEND_SLOTS_PER_EVAL = 12.6
PROFILE_SOURCES = {
    "k_blend": ("k_blend.hip", "blend_common.hpp", "fgs_internal.hpp"),
    "k_preprocess": ("k_project.hip", "fgs_internal.hpp", "sh_basis.hpp"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash(kernel):
    """Hash of a kernel's sources with comments and blank lines left out, so
    that a change of wording alone does not void the counters taken on it."""
    h = hashlib.sha256()
    for f in PROFILE_SOURCES[kernel]:
        src = open(os.path.join(ROOT, "paper_2408_07967_amd", "csrc", f)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        lines = (re.sub(r"//.*$", "", ln).rstrip() for ln in src.splitlines())
        h.update("\n".join(ln for ln in lines if ln.strip()).encode())
    return h.hexdigest()[:16]


def profile_record(kernel, workload):
    """A committed rocprofv3 summary of the kernel on the workload
    (profiles/<kernel>_<workload>_counters.json), or None if absent or taken
    on different kernel sources."""
    p = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("kernel_sha") != kernel_source_hash(kernel):
        return None
    return d


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_frame(scene, cam, W, H, opts, mode="f64"):
    """One oracle frame (binary64, or its binary32 mode): (seconds, pairs,
    image [3, H, W])."""
    from oracle import oracle as orc
    prep = orc.Prepared(scene, cam, W, H, opts, mode)
    t0 = time.perf_counter()
    state, ints, n = orc.preprocess(prep)
    tiles, vals, rng = orc.pairs(prep, state, ints, n)
    rgb, _, _ = orc.blend_tiled(prep, state, vals, rng)
    return time.perf_counter() - t0, int(n), rgb


def cpu_baseline(scene, cam, W, H, opts):
    """The CPU oracle, untuned, timed on the host: one full frame of the
    timed workload in binary64 (the baseline) and in its binary32 mode, one
    frame of each smaller workload, and the 10k-Gaussian frame on one thread.
    Returns the record and the binary64 and binary32 images of the frame."""
    from oracle import oracle as orc
    from paper_2408_07967_amd import scenes
    threads = int(orc._lib().orc_num_threads())
    dt, npairs, rgb = oracle_frame(scene, cam, W, H, opts)
    dt32, _, rgb32 = oracle_frame(scene, cam, W, H, opts, "f32")
    res = dict(value=round(1.0 / dt, 5), unit="frames/s", cores=threads, kind="oracle",
               sample=f"one full {W}x{H} frame of the same scene and camera, binary64 "
                      f"(preprocess + pairs + sort + blend; input conversion excluded); {dt:.2f} s",
               cpu_model=cpu_model(), host_cpus=os.cpu_count(), pairs_per_s=round(npairs / dt, 1),
               binary32_mode=dict(frames_per_s=round(1.0 / dt32, 5), seconds=round(dt32, 3)))
    other = {}
    for kind, name in (("small", WORKLOADS["small"]["name"]), ("medium", WORKLOADS["medium"]["name"])):
        sc2 = scenes.make_scene(kind)
        cam2 = scenes.camera_for(kind, 0)
        dt2, n2, _ = oracle_frame(sc2, cam2, cam2.W, cam2.H, opts)
        other[name] = dict(frames_per_s=round(1.0 / dt2, 3), pairs_per_s=round(n2 / dt2, 1), seconds=round(dt2, 3),
                           cores=threads)
        if kind == "small":
            orc._lib().orc_set_num_threads(1)
            try:
                reps = 5
                t0 = time.perf_counter()
                for _ in range(reps):
                    dt1, n1, _ = oracle_frame(sc2, cam2, cam2.W, cam2.H, opts)
                dt1 = (time.perf_counter() - t0) / reps
            finally:
                orc._lib().orc_set_num_threads(threads)
            other[name + "-one-thread"] = dict(frames_per_s=round(1.0 / dt1, 3), pairs_per_s=round(n1 / dt1, 1),
                                               seconds=round(dt1, 4), cores=1)
    res["other_workloads"] = other
    return res, rgb, rgb32


def image_parity(gpu_rgb, ref_rgb, tol=2e-3, frac_bar=0.999, mean_bar=1e-5):
    """Per-pixel comparison with the binary64 oracle's image: a pixel is
    within tolerance when all three channels are; pass = both bars met."""
    import numpy as np
    d = np.abs(gpu_rgb.astype(np.float64) - ref_rgb.astype(np.float64))
    px = d.max(axis=0)
    frac, mean = float((px <= tol).mean()), float(d.mean())
    return dict(reference="oracle binary64, same scene and camera", tolerance=tol,
                frac_pixels_within=round(frac, 6), max_abs=float(px.max()), mean_abs=mean,
                bar=f"frac_pixels_within >= {frac_bar} and mean_abs <= {mean_bar}",
                passed=bool(frac >= frac_bar and mean <= mean_bar))


def visible_bounds(scene, cam):
    """P_z: Gaussians whose camera-space depth exceeds the near plane (the
    Gaussians whose remaining attributes the method reads, Alg. 4)."""
    import numpy as np
    m = scene.means.astype(np.float64)
    R = np.asarray(cam.R, np.float64)
    z = R[2] @ m + float(cam.t[2])
    return int(np.count_nonzero(z > cam.near))


def super_sort_bytes(E, nsuper):
    """Bytes the design's sort of the super-tile entries moves: one LSD pass
    of up to 9 bits (else passes of 8 bits) over the uint16 super-tile ids;
    per pass the upsweep reads the ids and the downsweep reads the ids and
    the 12-byte payload (Gaussian index, 64-bit tile mask) and writes the
    payload, and the ids too except in the last pass."""
    bits = max(1, math.ceil(math.log2(max(nsuper, 2))))
    passes = 0 if nsuper <= 1 else (1 if bits <= 9 else math.ceil(bits / 8))
    b = 0
    for p in range(passes):
        last = p == passes - 1
        b += E * (2 + 2 + 12 + 12 + (0 if last else 2))
    return b, passes


def stage_rooflines(stage_ms, stats, P, P_z, W, H, evals, steps_exec, peaks=None):
    """Per-stage achieved bandwidth or VALU rate against the MI355X peaks.
    Algorithmic bytes: the method's (what it reads and writes per Gaussian)
    for the preprocess; the design's own for the sorts, the
    emission and the tile lists (it sorts the depth digits once per Gaussian
    and the super-tile entries by super-tile, then expands the entries'
    masks into the per-tile lists)."""
    V, N, cand = stats["visible"], stats["pairs"], stats["candidates"]
    E, C = stats["entries"], stats["big_chunks"]
    ntiles = stats["tiles_x"] * stats["tiles_y"]
    nsuper = math.ceil(stats["tiles_x"] / 8) * math.ceil(stats["tiles_y"] / 8)
    ssort, spasses = super_sort_bytes(E, nsuper)
    rows = {}

    def hbm(name, nbytes, ms, note):
        if ms <= 0:
            return
        gbs = nbytes / (ms * 1e-3) / 1e9
        rows[name] = dict(bound="hbm", bytes=int(nbytes), ms=round(ms, 4), achieved_gbs=round(gbs, 1),
                          frac=round(gbs / HBM_PEAK_GBS, 4), bytes_are=note)

    nb = (P + 255) // 256
    read = stats.get("cull_batches", 0)
    if read:
        hbm("cull", 48 * nb + 24 * min(P, 256 * read), stage_ms["cull"],
            f"design: 48 B of bounds per 256-slot batch ({nb}), and 24 B per Gaussian (position, opacity, trace of "
            f"the covariance, k^2) of the {read} batches the bounds keep")
    else:
        hbm("cull", 24 * P, stage_ms["cull"], "24 B per Gaussian: position, opacity, trace of the covariance, k^2")
    hbm("preprocess", 32 * P_z + 232 * V, stage_ms["preprocess"],
        "method: 32 P_z (scales, rotation, opacity of the Gaussians past the near plane) + 192 P_vis (SH) + "
        "40 P_vis (state written)")
    hbm("cull_and_preprocess", 12 * P + 32 * P_z + 232 * V, stage_ms["cull"] + stage_ms["preprocess"],
        "method: 12 P (means) + 32 P_z + 232 P_vis")
    hbm("depth_sort", 80 * V, stage_ms["depth_sort"],
        "design: 4 LSD passes over the visible (depth, index) pairs, 20 B per pair and pass")
    hbm("super_sort", ssort, stage_ms["super_sort"],
        f"design: {spasses} LSD pass(es) over the super-tile entries: ids read twice, 12-byte payload read "
        "and written (ids written too before the last pass)")
    hbm("sort", 80 * V + ssort, stage_ms["depth_sort"] + stage_ms["super_sort"],
        "design: depth sort + super-tile sort (the method's full-key sort would move 8 N + 24 N per 8-bit "
        "key pass over the pairs)")
    hbm("emit", 24 * V + 32 * C + 14 * E + 8 * nsuper, stage_ms["emit"],
        "design: order, offset and 16-byte record per visible Gaussian, a 256-tile chunk mask per large "
        "rectangle chunk read; a 14-byte entry per overlapped super-tile written")
    hbm("tile_lists", 20 * E + 4 * N + 8 * ntiles, stage_ms["tile_lists"],
        "design: masks read twice and Gaussian indices once per entry, a 4-byte value per pair and the "
        "ranges per tile written")
    hbm("scan", 17 * V, stage_ms["scan"], "design: order (4 B) and count (1 B) gathered, 12 B per visible "
                                           "Gaussian written and read")
    if evals and stage_ms["blend"] > 0:
        slots = evals * BLEND_SLOTS_PER_EVAL
        tops = slots / (stage_ms["blend"] * 1e-3) / 1e12
        rows["blend"] = dict(bound="alu", slots=int(slots), ms=round(stage_ms["blend"], 4),
                             achieved_tops=round(tops, 3), peak_tops=round(VALU_PEAK_TSLOTS, 2),
                             frac=round(tops / VALU_PEAK_TSLOTS, 4),
                             slots_are=f"method evaluations (every pixel's examined list entries) x "
                                       f"{BLEND_SLOTS_PER_EVAL} FP32 lane-slots (10.6 add/mul/fma + v_exp_f32 at 2)",
                             executed_steps=steps_exec)
        if peaks:
            m = peaks["fma_lane_ops_per_s"] / 1e12
            rows["blend"].update(measured_peak_tops=round(m, 2), frac_of_measured=round(tops / m, 4))
    if peaks:
        cb = peaks["copy_bytes_per_s"] / 1e9
        for r in rows.values():
            if r["bound"] == "hbm":
                r["frac_of_measured_copy"] = round(r["achieved_gbs"] / cb, 4)
    return rows


def dominant_roofline(rows, stage_ms, workload):
    """The `roofline` object: the kernel with the longest launch of the frame
    (the preprocess or the blend), with the HBM traffic of its committed
    counter run when that run was taken on the current kernel sources."""
    cands = [k for k in ("preprocess", "blend") if k in rows]
    if not cands:
        return None
    k = max(cands, key=lambda c: stage_ms[c])
    r = rows[k]
    kernel = "k_preprocess" if k == "preprocess" else "k_blend"
    prof = profile_record(kernel, workload)
    traffic = prof.get("hbm_bytes_per_launch") if prof else None
    if r["bound"] == "hbm":
        out = dict(bound="hbm", achieved=r["achieved_gbs"], peak=HBM_PEAK_GBS, unit="GB/s", frac=r["frac"],
                   traffic=traffic, kernel=kernel, algorithmic_bytes_per_launch=r["bytes"],
                   avg_launch_ms=r["ms"], bytes_are=r["bytes_are"])
        if "frac_of_measured_copy" in r:
            out["frac_of_measured_copy"] = r["frac_of_measured_copy"]
    else:
        out = dict(bound="alu", achieved=r["achieved_tops"], peak=r["peak_tops"], unit="T FP32 lane-slots/s",
                   frac=r["frac"], traffic=traffic, kernel=kernel, valu_slots_per_launch=r["slots"],
                   avg_launch_ms=r["ms"], slots_are=r["slots_are"],
                   peak_is="published 157.3 TFLOP/s FP32 vector / 4 (packed FMA counted as 2 lanes x 2 FLOP)")
        for k2 in ("measured_peak_tops", "frac_of_measured"):
            if k2 in r:
                out[k2] = r[k2]
    if prof:
        out["counters"] = {k2: v for k2, v in prof.items() if k2 not in ("commands", "kernel_sha")}
    return out


SERVE_BUDGET = 3 << 30   # pair and sort buffers of admitted requests
SERVE_SLOTS = 4
SERVE_SHARE = 2          # a request runs beside others only while two or more wait


def serving_leg(args):
    """Serving workload: resident 6M-Gaussian scene of the large-scene
    distributions, Poisson camera requests on the 200 m orbit with mixed
    resolutions, replayed natively through the render server (continuous
    batching, byte-budget admission, graph replay) and through the plain
    one-request-at-a-time renderer on the same GPU, both from the scene's
    resident precompute (the plain renderer from the raw parameters as a
    second reference)."""
    import torch
    from paper_2408_07967_amd import scenes
    from paper_2408_07967_amd.render import GaussianScene, Renderer
    from paper_2408_07967_amd.serve import RenderServer, make_trace, replay_plain, latency_summary
    t0 = time.perf_counter()
    sc = scenes.make_scene("serve")
    gsc = GaussianScene.from_numpy(sc, "cuda:0")
    del sc
    trace = make_trace(args.serve_rate, args.serve_seconds, seed=5)
    warm = make_trace(400.0, 0.25, seed=6)
    log(f"[bench] serving: P={gsc.P}, {len(trace)} requests over {args.serve_seconds:.0f} s at "
        f"{args.serve_rate:.0f}/s (setup {time.perf_counter() - t0:.1f}s)")
    rnd = lambda d: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in d.items()}
    R = Renderer(0)
    prep = R.prepare(gsc)

    def plain(tr, raw=False):
        replay_plain(R, gsc, None, warm, prepared=None if raw else prep)
        return latency_summary(replay_plain(R, gsc, None, tr, prepared=None if raw else prep))

    def server():
        return RenderServer(gsc, budget_bytes=SERVE_BUDGET, max_inflight=SERVE_SLOTS, max_bypass=4,
                            share_queue=SERVE_SHARE)

    def served(tr):
        srv = server()
        try:
            srv.replay(warm)
            res = srv.replay(tr)
            st = srv.stats()
        finally:
            srv.close()
        return latency_summary(res), st

    ps = plain(trace)
    log(f"[bench] plain renderer (prepared scene): {ps}")
    ss, st = served(trace)
    log(f"[bench] server: {ss} stats {st}")
    # the raw-parameter plain renderer on a shorter stretch of the same trace
    tr_raw = [q for q in trace if q["t_ns"] < min(args.serve_seconds, 10.0) * 1e9]
    pr = plain(tr_raw, raw=True)
    log(f"[bench] plain renderer (raw parameters, first {len(tr_raw)} requests): {pr}")
    sweep = []
    for rate, secs in ((500.0, 8.0), (800.0, 5.0)):
        tr = make_trace(rate, min(args.serve_seconds, secs), seed=7)
        hp = plain(tr)
        hs, _ = served(tr)
        log(f"[bench] at {rate:.0f}/s: plain {hp} server {hs}")
        sweep.append(dict(rate_per_s=rate, requests=len(tr), server=rnd(hs), plain=rnd(hp),
                          p50_ratio_plain_over_server=round(hp["p50_ms"] / hs["p50_ms"], 3),
                          p99_ratio_plain_over_server=round(hp["p99_ms"] / hs["p99_ms"], 3)))
    R.release_prepared(prep)
    R.close()
    del gsc
    torch.cuda.empty_cache()
    return dict(workload=f"serve-6M-gaussians-poisson{args.serve_rate:.0f}-{args.serve_seconds:.0f}s-"
                         f"720p-1080p-1440p-2160p",
                requests=len(trace), server=rnd(ss), plain=rnd(ps),
                plain_is="fgs_render_prepared one request at a time on the same resident precompute",
                plain_raw_parameters=dict(rnd(pr), requests=len(tr_raw)),
                p50_ratio_plain_over_server=round(ps["p50_ms"] / ss["p50_ms"], 3),
                p99_ratio_plain_over_server=round(ps["p99_ms"] / ss["p99_ms"], 3),
                load_sweep=sweep,
                budget_bytes=SERVE_BUDGET, slots=SERVE_SLOTS, share_queue=SERVE_SHARE,
                server_stats={k: st[k] for k in ("peak_bytes_in_use", "graphs_captured", "graph_launches",
                                                 "bypasses", "region_evictions")})


def differentiation_leg(steps):
    """Forward + backward on the differentiation workload: 1M Gaussians of the
    1080p orbit scene at 1920x1080, L1 loss against the image of the same scene
    with means perturbed by N(0, 0.01).  Times the forward (saved frame) and
    the backward (blend adjoint + preprocess adjoint) with HIP-synchronised
    wall clocks."""
    import torch
    from paper_2408_07967_amd import scenes
    from paper_2408_07967_amd.render import GaussianScene, Renderer
    sc = scenes.make_scene("medium")
    gsc = GaussianScene.from_numpy(sc, "cuda:0")
    tgt_sc = GaussianScene.from_numpy(scenes.perturb_means(sc), "cuda:0")
    del sc
    cam = scenes.camera_for("medium", W=1920, H=1080)
    R = Renderer(0)
    target = R.render(tgt_sc, cam, 1920, 1080)["rgb"].clone()
    del tgt_sc
    fwd = bwd = 0.0
    for it in range(steps + 2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = R.render(gsc, cam, 1920, 1080, save=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dL = torch.sign(out["rgb"] - target) / out["rgb"].numel()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        R.backward(out["frame"], gsc, cam, 1920, 1080, None, dL)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        R.release(out["frame"])
        if it >= 2:
            fwd += t1 - t0
            bwd += t3 - t2
    R.close()
    return dict(workload="medium-1M-gaussians-1920x1080-l1", forward_ms=round(fwd / steps * 1e3, 3),
                backward_ms=round(bwd / steps * 1e3, 3), pairs=int(out["stats"]["pairs"]))


def batch_leg(R, gsc, prep, W, H, opts, ncams, steps):
    """Multi-camera batches of the resident scene: ncams viewpoints of a
    camera rig (the workload camera with its eye moved sideways in 2 m steps,
    same orientation) rendered by one batch call, against the same cameras
    rendered one call each.  Both sides have every input resident in HBM;
    frames/s counts camera images."""
    import numpy as np
    import torch
    from paper_2408_07967_amd import scenes
    base = scenes.camera_for("city", W=W, H=H)
    cams = []
    for i in range(ncams):
        dx = 2.0 * (i - (ncams - 1) / 2.0)
        eye = np.asarray(base.eye, np.float64) + np.array([dx, 0.0, 0.0])
        fwd = np.array([0.0, math.sin(math.radians(-30.0)), math.cos(math.radians(-30.0))])
        cams.append(scenes.look_at(eye, eye + fwd, W, H, 70.0))
    outs = [torch.empty((3, H, W), dtype=torch.float32, device="cuda:0") for _ in cams]
    for _ in range(2):
        got = R.render_batch(prep, gsc, cams, W, H, opts)
        for c, o in zip(cams, outs):
            R.render(gsc, c, W, H, opts, out=o, prepared=prep)
    torch.cuda.synchronize()
    same = all(torch.equal(g["rgb"].view(torch.int32), o.view(torch.int32)) for g, o in zip(got, outs))
    t0 = time.perf_counter()
    for _ in range(steps):
        for c, o in zip(cams, outs):
            R.render(gsc, c, W, H, opts, out=o, prepared=prep)
    torch.cuda.synchronize()
    single = steps * ncams / (time.perf_counter() - t0)
    t0 = time.perf_counter()
    for _ in range(steps):
        got = R.render_batch(prep, gsc, cams, W, H, opts)
    torch.cuda.synchronize()
    batched = steps * ncams / (time.perf_counter() - t0)
    return dict(cameras=ncams, rig="eye moved sideways in 2 m steps", batched_frames_per_s=round(batched, 2),
                one_call_per_camera_frames_per_s=round(single, 2), speedup=round(batched / single, 4),
                union_candidates=int(got[0]["stats"]["candidates"]), bit_identical=bool(same))


def time_frames(R, gsc, cams, W, H, opts, steps, prepared):
    """Frames/s of `steps` passes over `cams`, one request at a time (each
    render call enqueues its frame; the stream orders them), and the stats
    of the last frame of each camera."""
    import torch
    out = torch.empty((3, H, W), dtype=torch.float32, device="cuda:0")
    stats = [R.render(gsc, c, W, H, opts, out=out, prepared=prepared)["stats"] for c in cams]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for c in cams:
            R.render(gsc, c, W, H, opts, out=out, prepared=prepared)
    torch.cuda.synchronize()
    return steps * len(cams) / (time.perf_counter() - t0), stats, out


def workloads_leg(R, city_sc, city_gsc, city_prep, opts, steps, with_parity):
    """Frames/s and pairs/s of the other benchmark workloads, each from the
    prepared scene and from the raw parameters: 10k Gaussians at 256x256;
    1M Gaussians at 1920x1080 through the eight orbit cameras, one request
    at a time; the 10M city scene at 7680x4320.  With parity: camera 0 of
    the 1M workload and the 8K frame against the binary64 oracle."""
    import numpy as np
    import torch
    from paper_2408_07967_amd import scenes
    from paper_2408_07967_amd.render import GaussianScene
    out = {}
    for key in ("small", "medium", "city8k"):
        wl = WORKLOADS[key]
        W, H = wl["W"], wl["H"]
        if key == "city8k":
            sc, gsc, prep, owns = city_sc, city_gsc, city_prep, False
        else:
            sc = scenes.make_scene(wl["kind"])
            gsc = GaussianScene.from_numpy(sc, "cuda:0")
            prep, owns = R.prepare(gsc, opts), True
        cams = [scenes.camera_for(wl["kind"], k, W=W, H=H) for k in range(8 if key == "medium" else 1)]
        n = max(3, steps // (8 if key == "medium" else 1) // (4 if key == "city8k" else 1))
        fps_p, st_p, img = time_frames(R, gsc, cams, W, H, opts, n, prep)
        fps_r, _, _ = time_frames(R, gsc, cams, W, H, opts, max(2, n // 2), None)
        pairs = [int(s["pairs"]) for s in st_p]
        row = dict(workload=wl["name"], cameras=len(cams), frames_per_s=round(fps_p, 2),
                   raw_params_frames_per_s=round(fps_r, 2),
                   pairs_per_frame=pairs if len(pairs) > 1 else pairs[0],
                   pairs_per_s=round(float(np.mean(pairs)) * fps_p, 1),
                   visible=[int(s["visible"]) for s in st_p] if len(st_p) > 1 else int(st_p[0]["visible"]))
        if with_parity and key in ("medium", "city8k"):
            cam0 = cams[0]
            o = R.render(gsc, cam0, W, H, opts, prepared=prep)["rgb"]
            torch.cuda.synchronize()
            _, _, ref = oracle_frame(sc, cam0, W, H, opts)
            row["parity_camera0"] = image_parity(o.cpu().numpy(), ref)
            del ref
        log(f"[bench] workload {wl['name']}: {row}")
        out[key] = row
        if owns:
            R.release_prepared(prep)
            del gsc
        torch.cuda.empty_cache()
    return out


def compare_binning(steps):
    """Pair redundancy of the binning modes (the paper's pair-count and
    stage-breakdown comparison, on the synthetic workloads): exact ellipse/tile
    test, every tile of the tight box, every tile of the 3DGS 3 sigma square."""
    import torch
    from paper_2408_07967_amd import scenes
    from paper_2408_07967_amd import binding as B
    from paper_2408_07967_amd.render import GaussianScene, Renderer
    out = {}
    for key in ("medium", "city4k"):
        wl = WORKLOADS[key]
        sc = scenes.make_scene(wl["kind"])
        gsc = GaussianScene.from_numpy(sc, "cuda:0")
        del sc
        cam = scenes.camera_for(wl["kind"], W=wl["W"], H=wl["H"])
        R = Renderer(0)
        img = torch.empty((3, wl["H"], wl["W"]), dtype=torch.float32, device="cuda:0")
        rows = {}
        for mode, name in ((0, "exact"), (1, "tight_box"), (2, "3sigma_square")):
            o = dict(scenes.DEFAULT_OPTIONS, binning=mode)
            prep = R.prepare(gsc, o)
            st = None
            for _ in range(2):
                st = R.render(gsc, cam, wl["W"], wl["H"], o, out=img, prepared=prep)["stats"]
            R.set_instrumentation(B.INSTR_STAGE_TIMES)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                R.render(gsc, cam, wl["W"], wl["H"], o, out=img, prepared=prep)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / steps
            inst = R.instrumentation()
            R.set_instrumentation(0)
            nf = max(1, inst["frames"])
            rows[name] = dict(pairs=int(st["pairs"]), visible=int(st["visible"]),
                              pairs_per_visible=round(st["pairs"] / max(1, st["visible"]), 3),
                              ms_per_frame=round(dt * 1e3, 4),
                              stage_ms={k[3:]: round(inst[k] / nf, 4) for k in inst if k.startswith("ms_")})
            R.release_prepared(prep)
            log(f"[bench] {key} {name}: {rows[name]}")
        ex = rows["exact"]
        for name in ("tight_box", "3sigma_square"):
            rows[name]["pair_reduction_by_exact"] = round(1.0 - ex["pairs"] / rows[name]["pairs"], 4)
            rows[name]["speedup_of_exact"] = round(rows[name]["ms_per_frame"] / ex["ms_per_frame"], 3)
        out[wl["name"]] = rows
        R.close()
        del gsc, img
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="city4k", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-work-count", action="store_true")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-backward", action="store_true", help="skip the forward + backward timing")
    ap.add_argument("--no-workloads", action="store_true", help="skip the 10k, 1M x 8 cameras and 8K legs")
    ap.add_argument("--blend-variant", type=int, default=0, choices=(0, 1),
                    help="0: LDS-batched blend (default); 1: prefetch-pipeline blend (same image)")
    ap.add_argument("--compare-binning", action="store_true",
                    help="also report pairs and stage times of the three binning modes")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="length of the Poisson request trace")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--batch-cameras", type=int, default=4,
                    help="cameras of the multi-camera batch leg (0 skips it)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after the timed region, run one device copy of 256 MiB (read 256 MiB, write 256 MiB) "
                         "whose FETCH_SIZE / WRITE_SIZE counters scale the kernels' counters")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this renderer runs on a single MI355X; "
              "multi-GPU sharding is a design note, not a measured path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2408_07967_amd import scenes
    from paper_2408_07967_amd import binding as B
    from paper_2408_07967_amd.render import GaussianScene, Renderer

    wl = WORKLOADS[args.workload]
    W, H = wl["W"], wl["H"]
    t0 = time.perf_counter()
    sc = scenes.make_scene(wl["kind"])
    cam = scenes.camera_for(wl["kind"], W=W, H=H)
    P_z = visible_bounds(sc, cam)
    log(f"[bench] scene {wl['kind']} P={sc.P} drawn in {time.perf_counter() - t0:.1f}s; {P_z} past the near plane")
    torch.cuda.set_device(0)
    gsc = GaussianScene.from_numpy(sc, "cuda:0")
    R = Renderer(0)
    peaks = R.measure_peaks()
    log(f"[bench] measured peaks: FP32 FMA {peaks['fma_lane_ops_per_s'] / 1e12:.2f} T lane-ops/s, v_exp_f32 "
        f"{peaks['exp_lane_ops_per_s'] / 1e12:.2f} T, copy {peaks['copy_bytes_per_s'] / 1e12:.2f} TB/s")
    R.set_blend_variant(args.blend_variant)
    opts = scenes.DEFAULT_OPTIONS
    out = torch.empty((3, H, W), dtype=torch.float32, device="cuda:0")
    stats = None
    # the raw-parameter path, timed for reference
    for _ in range(max(1, args.warmup)):
        stats = R.render(gsc, cam, W, H, opts, out=out)["stats"]
    torch.cuda.synchronize()
    n_raw = max(1, args.steps // 2)
    t0 = time.perf_counter()
    for _ in range(n_raw):
        R.render(gsc, cam, W, H, opts, out=out)
    torch.cuda.synchronize()
    raw_fps = n_raw / (time.perf_counter() - t0)
    log(f"[bench] raw parameters: {raw_fps:.2f} frames/s; visible {stats['visible']} pairs {stats['pairs']}")
    # the resident scene's view-independent precompute (Sec. 5.3.1), once
    t0 = time.perf_counter()
    prep = R.prepare(gsc, opts)
    torch.cuda.synchronize()
    prep_ms = (time.perf_counter() - t0) * 1e3
    for _ in range(max(1, args.warmup)):
        stats = R.render(gsc, cam, W, H, opts, out=out, prepared=prep)["stats"]
    torch.cuda.synchronize()
    log(f"[bench] prepared in {prep_ms:.1f} ms; warmup done")

    evals = steps_exec = None
    if not args.no_work_count:
        R.set_instrumentation(B.INSTR_WORK)
        R.render(gsc, cam, W, H, opts, out=out, prepared=prep)
        inst = R.instrumentation()
        evals, steps_exec = int(inst["blend_evaluations"]), int(inst["blend_wave_steps"])
        R.set_instrumentation(0)
        log(f"[bench] blend: {evals} evaluations per frame (method), {steps_exec} wavefront steps executed "
            f"({steps_exec * 128} pixel evaluations)")

    # the timed frames run without instrumentation
    R.set_instrumentation(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        R.render(gsc, cam, W, H, opts, out=out, prepared=prep)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dt = t1 - t0
    fps = args.steps / dt
    # stage times (HIP events recorded on the render stream between stages,
    # which adds a marker per stage) over a second run of the same frames
    R.set_instrumentation(B.INSTR_STAGE_TIMES)
    for _ in range(args.steps):
        R.render(gsc, cam, W, H, opts, out=out, prepared=prep)
    torch.cuda.synchronize()
    inst = R.instrumentation()
    R.set_instrumentation(0)
    nf = max(1, inst["frames"])
    stage_ms = {k[3:]: round(inst[k] / nf, 4) for k in inst if k.startswith("ms_")}
    log(f"[bench] {args.steps} frames in {dt:.3f}s -> {fps:.2f} frames/s; stages {stage_ms}")
    # single-frame latency: each frame waited for on its own
    lat = []
    for _ in range(args.steps):
        t0 = time.perf_counter()
        R.render(gsc, cam, W, H, opts, out=out, prepared=prep)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t0) * 1e3)
    lat = np.sort(np.asarray(lat))
    frame_ms = dict(p10=round(float(np.percentile(lat, 10)), 4), p50=round(float(np.percentile(lat, 50)), 4),
                    p90=round(float(np.percentile(lat, 90)), 4))
    log(f"[bench] single-frame latency ms {frame_ms}")

    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    rows = stage_rooflines(stage_ms, stats, sc.P, P_z, W, H, evals, steps_exec, peaks)
    roof = dominant_roofline(rows, stage_ms, args.workload)
    log(f"[bench] rooflines {rows}")

    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle ...")
        cpu, ref_rgb, f32_rgb = cpu_baseline(sc, cam, W, H, opts)
        log(f"[bench] cpu baseline {cpu}")
        parity = image_parity(out.cpu().numpy(), ref_rgb)
        # the same comparison for the oracle's own binary32 mode
        parity["oracle_binary32_vs_binary64"] = {k: v for k, v in image_parity(f32_rgb, ref_rgb).items()
                                                 if k in ("frac_pixels_within", "max_abs", "mean_abs", "passed")}
        del ref_rgb, f32_rgb
        log(f"[bench] image parity {parity}")

    batch = None
    if args.batch_cameras > 0:
        batch = batch_leg(R, gsc, prep, W, H, opts, args.batch_cameras, max(3, args.steps // 10))
        log(f"[bench] multi-camera batch: {batch}")
    others = None
    if not args.no_workloads and args.workload == "city4k":
        others = workloads_leg(R, sc, gsc, prep, opts, max(20, args.steps // 2), with_parity=not args.no_cpu_baseline)
    R.release_prepared(prep)
    R.close()
    del gsc, out
    torch.cuda.empty_cache()
    serving = None
    if not args.no_serve:
        serving = serving_leg(args)
    binning_modes = compare_binning(max(5, args.steps // 5)) if args.compare_binning else None
    differentiation = None if args.no_backward else differentiation_leg(10)
    if differentiation:
        log(f"[bench] forward + backward: {differentiation}")

    res = dict(metric=METRIC, value=round(fps, 3), unit="frames/s", n_gpus=1, steps=args.steps,
               warmup=args.warmup, ms_per_step=round(dt / args.steps * 1e3, 4), higher_is_better=True,
               scaling="weak", vs_baseline=None, dtype="f32", data="synthetic",
               config=dict(workload=wl["name"], gaussians=sc.P, width=W, height=H, sh_degree=sc.sh_degree,
                           tile=16, scene_format="prepared (view-independent precompute, done once per scene)",
                           blend_variant="prefetch pipeline" if args.blend_variant else "LDS batches",
                           raw_params_frames_per_s=round(raw_fps, 3), prepare_ms=round(prep_ms, 2),
                           visible=int(stats["visible"]), pairs=int(stats["pairs"]),
                           candidates=int(stats["candidates"]), cull_batches_read=int(stats["cull_batches"]),
                           past_near_plane=P_z,
                           big_rect_chunks=int(stats["big_chunks"]), super_tile_entries=int(stats["entries"]),
                           pairs_per_s=round(stats["pairs"] * fps, 1), stage_ms=stage_ms,
                           single_frame_ms=frame_ms,
                           blend_evaluations=evals, blend_wave_steps=steps_exec),
               roofline=roof, stage_roofline=rows,
               measured_peaks=dict(fp32_fma_tlane_ops=round(peaks["fma_lane_ops_per_s"] / 1e12, 3),
                                   v_exp_f32_tlane_ops=round(peaks["exp_lane_ops_per_s"] / 1e12, 3),
                                   copy_gbs=round(peaks["copy_bytes_per_s"] / 1e9, 1),
                                   how="fgs_measure_peaks: FMA chains, v_exp_f32 chains, 1 GiB device copy; "
                                       "best of several runs"),
               cpu_baseline=cpu, parity=parity, workloads=others,
               serving=serving, differentiation=differentiation, multi_camera=batch)
    if binning_modes is not None:
        res["binning_modes"] = binning_modes
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
