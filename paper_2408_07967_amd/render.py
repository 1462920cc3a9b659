"""PyTorch-facing wrapper over the C ABI.  PyTorch supplies device memory and
the current HIP stream; every stage of the rasterizer runs in libfgs.so."""
import ctypes as C
import weakref

import numpy as np
import torch

from . import binding as B


class GaussianScene:
    """Planar float32 Gaussian parameters on a GPU (shapes [planes, P])."""

    def __init__(self, means, log_scales, quats, logits, sh, sh_degree):
        self.means, self.log_scales, self.quats, self.logits, self.sh = means, log_scales, quats, logits, sh
        self.sh_degree = int(sh_degree)
        P = means.shape[1]
        for name, t, planes in (("means", means, 3), ("log_scales", log_scales, 3), ("quats", quats, 4),
                                ("logits", logits, 1), ("sh", sh, 3 * (self.sh_degree + 1) ** 2)):
            if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (planes, P):
                raise ValueError(f"{name}: expected a contiguous float32 CUDA tensor of shape ({planes}, {P}), "
                                 f"got {tuple(t.shape)} {t.dtype} on {t.device}")

    @property
    def P(self):
        return int(self.means.shape[1])

    @staticmethod
    def from_numpy(scene, device="cuda"):
        def t(a):
            return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        return GaussianScene(t(scene.means), t(scene.log_scales), t(scene.quats), t(scene.logits), t(scene.sh),
                             scene.sh_degree)

    def tensors(self):
        return (self.means, self.log_scales, self.quats, self.logits, self.sh)

    def abi(self):
        return B.make_scene(self.P, self.P, self.sh_degree, *(x.data_ptr() for x in self.tensors()))


def camera_abi(cam):
    return B.make_camera(np.asarray(cam.R, np.float32), np.asarray(cam.t, np.float32),
                         np.asarray(cam.eye, np.float32), cam.fx, cam.fy, cam.cx, cam.cy, cam.near)


def options_abi(opts=None):
    if opts is None:
        return B.default_options()
    if isinstance(opts, B.FgsOptions):
        return opts
    return B.default_options(**opts)


class Renderer:
    """One fgs_context on the current CUDA (HIP) device."""

    def __init__(self, device=None):
        dev = torch.cuda.current_device() if device is None else int(device)
        self.device = dev
        self.ctx = B.Context(dev)

    def reserve(self, max_gaussians, max_pairs, max_w, max_h):
        self.ctx.check(B.lib().fgs_reserve(self.ctx.handle, int(max_gaussians), int(max_pairs), int(max_w),
                                           int(max_h)))

    def scratch_bytes(self):
        return int(B.lib().fgs_scratch_bytes(self.ctx.handle))

    def prepare(self, scene, opts=None):
        """View-independent precompute of a resident scene (renders from it are
        bit-identical to renders of the scene).  Returns a handle for
        render(..., prepared=handle); free it with release_prepared."""
        h = C.c_void_p()
        sc = scene.abi()
        op = options_abi(opts)
        stream = torch.cuda.current_stream(scene.means.device).cuda_stream
        self.ctx.check(B.lib().fgs_prepare_scene(self.ctx.handle, C.byref(sc), C.byref(op), C.byref(h), stream))
        return h

    def release_prepared(self, handle):
        if handle and self.ctx.handle:
            self.ctx.check(B.lib().fgs_prepared_release(self.ctx.handle, handle))

    def render(self, scene, cam, W, H, opts=None, out=None, want_T=False, want_last=False, save=False,
               prepared=None):
        """Render; returns dict(rgb [3,H,W], T [H,W] or None, last [H,W] or None,
        stats, frame handle or None).  prepared: a handle from prepare(scene)."""
        dev = scene.means.device
        rgb = out if out is not None else torch.empty((3, H, W), dtype=torch.float32, device=dev)
        T = torch.empty((H, W), dtype=torch.float32, device=dev) if want_T else None
        last = torch.empty((H, W), dtype=torch.int32, device=dev) if want_last else None
        sc = scene.abi()
        cm = camera_abi(cam)
        op = options_abi(opts)
        st = B.FgsStats()
        fr = C.c_void_p()
        stream = torch.cuda.current_stream(dev).cuda_stream
        outs = (rgb.data_ptr(), T.data_ptr() if T is not None else None,
                last.data_ptr() if last is not None else None, C.byref(fr) if save else None, C.byref(st), stream)
        if prepared is not None:
            status = B.lib().fgs_render_prepared(self.ctx.handle, prepared, C.byref(cm), int(W), int(H),
                                                 C.byref(op), *outs)
        else:
            status = B.lib().fgs_render(self.ctx.handle, C.byref(sc), C.byref(cm), int(W), int(H), C.byref(op),
                                        *outs)
        self.ctx.check(status)
        return dict(rgb=rgb, T=T, last=last, frame=fr if save else None,
                    stats=dict(visible=st.visible, pairs=st.pairs, tiles_x=st.tiles_x, tiles_y=st.tiles_y,
                               sort_passes=st.sort_passes, big_chunks=st.big_chunks,
                               candidates=st.candidates, entries=st.entries, cull_batches=st.cull_batches))

    def render_noalloc(self, scene, cam, W, H, opts=None, out=None, want_T=False, want_last=False):
        """render() through fgs_render_noalloc: every scratch buffer comes from
        the library's fixed per-GPU array (B.NOALLOC_SCRATCH_BYTES); no frame
        is saved.  Raises FgsError (FGS_ERR_CAPACITY) for a frame that does not
        fit."""
        dev = scene.means.device
        rgb = out if out is not None else torch.empty((3, H, W), dtype=torch.float32, device=dev)
        T = torch.empty((H, W), dtype=torch.float32, device=dev) if want_T else None
        last = torch.empty((H, W), dtype=torch.int32, device=dev) if want_last else None
        sc = scene.abi()
        cm = camera_abi(cam)
        op = options_abi(opts)
        st = B.FgsStats()
        stream = torch.cuda.current_stream(dev).cuda_stream
        self.ctx.check(B.lib().fgs_render_noalloc(self.ctx.handle, C.byref(sc), C.byref(cm), int(W), int(H),
                                                  C.byref(op), rgb.data_ptr(),
                                                  T.data_ptr() if T is not None else None,
                                                  last.data_ptr() if last is not None else None, C.byref(st),
                                                  stream))
        return dict(rgb=rgb, T=T, last=last, frame=None,
                    stats=dict(visible=st.visible, pairs=st.pairs, tiles_x=st.tiles_x, tiles_y=st.tiles_y,
                               sort_passes=st.sort_passes, big_chunks=st.big_chunks,
                               candidates=st.candidates, entries=st.entries, cull_batches=st.cull_batches))

    def render_batch(self, prepared, scene, cams, W, H, opts=None, want_T=False, want_last=False):
        """Render several cameras of a prepared scene in one call (one cull and
        one preprocess pass for the whole batch).  Returns one dict per camera
        like render(), without a frame handle."""
        dev = scene.means.device
        n = len(cams)
        rgb = [torch.empty((3, H, W), dtype=torch.float32, device=dev) for _ in range(n)]
        T = [torch.empty((H, W), dtype=torch.float32, device=dev) for _ in range(n)] if want_T else None
        last = [torch.empty((H, W), dtype=torch.int32, device=dev) for _ in range(n)] if want_last else None
        cm = (B.FgsCamera * max(n, 1))(*[camera_abi(c) for c in cams])
        ptrs = lambda ts: (C.c_void_p * max(n, 1))(*[t.data_ptr() for t in ts]) if ts is not None else None
        op = options_abi(opts)
        st = (B.FgsStats * max(n, 1))()
        stream = torch.cuda.current_stream(dev).cuda_stream
        self.ctx.check(B.lib().fgs_render_prepared_batch(self.ctx.handle, prepared, cm, n, int(W), int(H),
                                                         C.byref(op), ptrs(rgb), ptrs(T), ptrs(last), st, stream))
        return [dict(rgb=rgb[i], T=T[i] if T else None, last=last[i] if last else None, frame=None,
                     stats=dict(visible=st[i].visible, pairs=st[i].pairs, tiles_x=st[i].tiles_x,
                                tiles_y=st[i].tiles_y, sort_passes=st[i].sort_passes,
                                big_chunks=st[i].big_chunks, candidates=st[i].candidates,
                                entries=st[i].entries, cull_batches=st[i].cull_batches))
                for i in range(n)]

    def plan(self, scene, cam, W, H, opts=None):
        """Pair count and device bytes of one frame, without rendering it:
        returns dict(pairs, bytes)."""
        sc = scene.abi()
        cm = camera_abi(cam)
        op = options_abi(opts)
        n = C.c_int64()
        b = C.c_size_t()
        stream = torch.cuda.current_stream(scene.means.device).cuda_stream
        self.ctx.check(B.lib().fgs_plan(self.ctx.handle, C.byref(sc), C.byref(cm), int(W), int(H), C.byref(op),
                                        C.byref(n), C.byref(b), stream))
        return dict(pairs=int(n.value), bytes=int(b.value))

    def backward(self, frame, scene, cam, W, H, opts, dL_drgb):
        """Gradients of L with respect to the raw parameters of `scene`, given
        dL/dRGB [3, H, W] for a frame saved by render(..., save=True).
        Returns a tuple of tensors shaped like scene.tensors()."""
        dev = scene.means.device
        dL = dL_drgb.to(device=dev, dtype=torch.float32).contiguous()
        if tuple(dL.shape) != (3, H, W):
            raise ValueError(f"dL_drgb must have shape (3, {H}, {W}), got {tuple(dL.shape)}")
        grads = tuple(torch.empty_like(t) for t in scene.tensors())
        g = B.FgsSceneGrad(scene.P, *(t.data_ptr() for t in grads))
        sc = scene.abi()
        cm = camera_abi(cam)
        op = options_abi(opts)
        stream = torch.cuda.current_stream(dev).cuda_stream
        self.ctx.check(B.lib().fgs_render_backward(self.ctx.handle, frame, C.byref(sc), C.byref(cm), C.byref(op),
                                                   dL.data_ptr(), C.byref(g), stream))
        return grads

    def set_instrumentation(self, flags):
        self.ctx.check(B.lib().fgs_set_instrumentation(self.ctx.handle, int(flags)))

    def set_blend_variant(self, variant):
        """B.BLEND_LDS_BATCHES (default) or B.BLEND_PREFETCH: two blend kernels
        that render the same image bit for bit."""
        self.ctx.check(B.lib().fgs_set_blend_variant(self.ctx.handle, int(variant)))

    def measure_peaks(self):
        """Measured peak rates of the device (FMA and v_exp_f32 issue, copy
        bandwidth): dict of the fgs_peaks fields."""
        p = B.FgsPeaks()
        self.ctx.check(B.lib().fgs_measure_peaks(self.ctx.handle, C.byref(p)))
        return {k: getattr(p, k) for k, _ in B.FgsPeaks._fields_}

    def instrumentation(self):
        t = B.FgsTimings()
        self.ctx.check(B.lib().fgs_get_instrumentation(self.ctx.handle, C.byref(t)))
        return {k: getattr(t, k) for k, _ in B.FgsTimings._fields_}

    def frame_field(self, frame, field):
        n = int(B.lib().fgs_frame_field_bytes(frame, field))
        buf = np.zeros(max(n, 4) // 4, np.uint32)
        self.ctx.check(B.lib().fgs_frame_download(self.ctx.handle, frame, field,
                                                  buf.ctypes.data_as(C.c_void_p), n))
        return buf[: n // 4]

    def release(self, frame):
        # a closed context has already freed its frames
        if frame and self.ctx.handle:
            self.ctx.check(B.lib().fgs_frame_release(self.ctx.handle, frame))

    def close(self):
        self.ctx.close()


class _FrameHolder:
    """Keeps a saved frame alive for the autograd graph; releases it when the
    graph is freed."""

    def __init__(self, renderer, frame):
        self.frame = frame
        self._fin = weakref.finalize(self, renderer.release, frame)


class RenderFunction(torch.autograd.Function):
    """Differentiable render: rgb = render(means, log_scales, quats, logits, sh).

    The forward saves its frame (per-Gaussian state, sorted lists, final
    transmittance and last contributor per pixel); the backward runs the
    hand-written adjoint kernels of libfgs.so."""

    @staticmethod
    def forward(ctx, renderer, cam, W, H, opts, sh_degree, means, log_scales, quats, logits, sh):
        scene = GaussianScene(means.detach().contiguous(), log_scales.detach().contiguous(),
                              quats.detach().contiguous(), logits.detach().contiguous(), sh.detach().contiguous(),
                              sh_degree)
        out = renderer.render(scene, cam, W, H, opts, save=True)
        ctx.renderer, ctx.cam, ctx.W, ctx.H, ctx.opts = renderer, cam, W, H, opts
        ctx.scene = scene
        ctx.holder = _FrameHolder(renderer, out["frame"])
        ctx.stats = out["stats"]
        return out["rgb"]

    @staticmethod
    def backward(ctx, grad_rgb):
        grads = ctx.renderer.backward(ctx.holder.frame, ctx.scene, ctx.cam, ctx.W, ctx.H, ctx.opts, grad_rgb)
        return (None, None, None, None, None, None) + tuple(grads)


def render_differentiable(renderer, cam, W, H, opts, sh_degree, means, log_scales, quats, logits, sh):
    """rgb [3, H, W] with gradients for the five planar parameter tensors."""
    return RenderFunction.apply(renderer, cam, W, H, opts, sh_degree, means, log_scales, quats, logits, sh)
