"""Python face of the render server in libfgs.so (argument marshalling only).

The server keeps one scene resident, admits camera requests by the bytes
their pair and sort buffers need, replays a captured graph per (slot,
resolution) for the second half of each frame, and overlaps requests on the
device.  This module also draws the serving workload's request trace and
replays it through the server and through the plain renderer."""
import ctypes as C

import numpy as np

from . import binding as B
from .render import GaussianScene, camera_abi, options_abi
from . import scenes


def clock_ns():
    return int(B.lib().fgs_clock_ns())


class RenderServer:
    def __init__(self, scene, opts=None, budget_bytes=8 << 30, max_inflight=6, max_width=3840, max_height=2160,
                 max_bypass=4, use_graphs=True, share_queue=0, batch_fronts=True, device=0):
        if not isinstance(scene, GaussianScene):
            raise TypeError("scene must be a GaussianScene")
        self.scene = scene  # keeps the device planes alive
        self._sc = scene.abi()
        self._op = options_abi(opts)
        cfg = B.FgsServerConfig(int(budget_bytes), int(max_inflight), int(max_width), int(max_height),
                                int(max_bypass), 1 if use_graphs else 0, int(share_queue),
                                1 if batch_fronts else 0)
        h = C.c_void_p()
        st = B.lib().fgs_server_create(int(device), C.byref(self._sc), C.byref(self._op), C.byref(cfg), C.byref(h))
        if st != B.FGS_OK:
            raise B.FgsError(st, "fgs_server_create failed")
        self.handle = h
        self._buf = (B.FgsServerResult * 64)()

    def _check(self, st):
        if st != B.FGS_OK:
            raise B.FgsError(st, B.lib().fgs_server_last_error(self.handle).decode())

    def submit(self, rid, cam, W, H, arrival_ns=None, out=None):
        """Queue a request; `out` (a contiguous float32 CUDA tensor of 3 W H
        elements, kept alive by the caller until completion) receives a copy
        of the image."""
        cm = cam if isinstance(cam, B.FgsCamera) else camera_abi(cam)
        t = clock_ns() if arrival_ns is None else int(arrival_ns)
        if out is not None and (out.numel() != 3 * W * H or not out.is_contiguous()):
            raise ValueError("out must be a contiguous tensor of 3 * W * H floats")
        self._check(B.lib().fgs_server_submit(self.handle, int(rid), C.byref(cm), int(W), int(H), t,
                                              out.data_ptr() if out is not None else None))

    def poll(self, wait_s=0.0):
        k = B.lib().fgs_server_poll(self.handle, self._buf, len(self._buf), int(wait_s * 1e9))
        if k < 0:
            self._check(-k)
        return [_result_dict(self._buf[i]) for i in range(k)]

    def release(self, rid):
        self._check(B.lib().fgs_server_release(self.handle, int(rid)))

    def stats(self):
        s = B.FgsServerStats()
        self._check(B.lib().fgs_server_get_stats(self.handle, C.byref(s)))
        return {k: int(getattr(s, k)) for k, _ in B.FgsServerStats._fields_}

    def replay(self, trace):
        arr = _trace_array(trace)
        res = (B.FgsServerResult * len(trace))()
        self._check(B.lib().fgs_server_replay(self.handle, arr, len(trace), res))
        return [_result_dict(r) for r in res]

    def close(self):
        if self.handle:
            B.lib().fgs_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _result_dict(r):
    return dict(id=int(r.id), status=int(r.status), width=int(r.width), height=int(r.height), slot=int(r.slot),
                rgb=r.rgb, arrival_ns=int(r.arrival_ns), start_ns=int(r.start_ns), admit_ns=int(r.admit_ns),
                done_ns=int(r.done_ns), visible=int(r.visible), pairs=int(r.pairs))


def _trace_array(trace):
    arr = (B.FgsTraceRequest * len(trace))()
    for i, q in enumerate(trace):
        arr[i].id = int(q["id"])
        arr[i].cam = camera_abi(q["cam"])
        arr[i].width = int(q["W"])
        arr[i].height = int(q["H"])
        arr[i].arrival_offset_ns = int(q["t_ns"])
    return arr


def make_trace(rate_hz, seconds, seed=5):
    """Poisson arrivals at rate_hz over `seconds`; each request draws a pose on
    the 200 m orbit at 50-150 m altitude and a resolution uniformly from
    1280x720, 1920x1080, 2560x1440, 3840x2160."""
    rng = np.random.default_rng(seed)
    t, out, i = 0.0, [], 0
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= seconds:
            break
        cam = scenes.serve_pose(rng)
        out.append(dict(id=i, cam=cam, W=cam.W, H=cam.H, t_ns=int(t * 1e9)))
        i += 1
    return out


def replay_plain(renderer, scene, opts, trace, stream=None, prepared=None):
    """The trace through the plain renderer (one request at a time, FIFO),
    from the raw parameters or, with prepared (a handle of
    renderer.prepare(scene)), from the resident precompute."""
    import torch
    W = max(q["W"] for q in trace)
    H = max(q["H"] for q in trace)
    scratch = torch.empty(3 * W * H, dtype=torch.float32, device=scene.means.device)
    sc = scene.abi()
    op = options_abi(opts)
    arr = _trace_array(trace)
    res = (B.FgsServerResult * len(trace))()
    s = torch.cuda.current_stream(scene.means.device).cuda_stream if stream is None else stream
    if prepared is not None:
        renderer.ctx.check(B.lib().fgs_replay_plain_prepared(renderer.ctx.handle, prepared, C.byref(op), arr,
                                                             len(trace), scratch.data_ptr(), res, s))
    else:
        renderer.ctx.check(B.lib().fgs_replay_plain(renderer.ctx.handle, C.byref(sc), C.byref(op), arr, len(trace),
                                                    scratch.data_ptr(), res, s))
    return [_result_dict(r) for r in res]


def latency_summary(results):
    """p50 / p99 / mean latency (ms) and throughput of completed requests."""
    ok = [r for r in results if r["status"] == B.FGS_OK]
    if not ok:
        return dict(completed=0)
    lat = np.array([(r["done_ns"] - r["arrival_ns"]) * 1e-6 for r in ok])
    t0 = min(r["arrival_ns"] for r in ok)
    t1 = max(r["done_ns"] for r in ok)
    return dict(completed=len(ok), rejected=len(results) - len(ok), p50_ms=float(np.percentile(lat, 50)),
                p99_ms=float(np.percentile(lat, 99)), mean_ms=float(lat.mean()), max_ms=float(lat.max()),
                frames_per_s=len(ok) / max((t1 - t0) * 1e-9, 1e-9))
