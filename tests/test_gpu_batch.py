"""GPU parity of the multi-camera batch over a prepared scene (one union cull
and one preprocess pass for every camera, then per-camera sort and blend):
each camera's image, final transmittance and last contributor must equal, bit
for bit, those of the same camera rendered alone from the prepared scene (a
path held bit-exact against the FP32 oracle by the other GPU tests), with the
same visible and pair counts; one camera of each case is also checked against
the FP64 oracle directly.  Cases cover one camera, the largest batch, a camera
that sees nothing, ragged image sizes, and pair buffers that grow between and
inside batches, and chunk lists that overflow and are resized within a batch."""
import math

import numpy as np
import pytest

from gpu_helpers import check_image
from oracle_helpers import identity_camera, opts, random_scene, scene_from

pytestmark = pytest.mark.gpu


def _np(out):
    return dict(rgb=out["rgb"].cpu().numpy(), T=out["T"].cpu().numpy(),
                last=out["last"].cpu().numpy().view(np.uint32), stats=out["stats"])


def _cases(scenes, case):
    from paper_2408_07967_amd.scenes import look_at
    if case == "small-4":
        sc = scenes.make_scene("small")
        W, H = 256, 256
        cams = [scenes.camera_for("small"),
                look_at((0.6, 0.3, -3.5), (0.0, 0.0, 0.0), W, H, 60.0),
                look_at((-1.0, -0.5, -5.0), (0.2, 0.0, 0.0), W, H, 45.0),
                look_at((0.0, 0.0, -4.0), (0.0, 0.0, -8.0), W, H, 60.0)]  # looks away: nothing visible
    elif case == "small-1":
        sc = scenes.make_scene("small")
        W, H = 199, 131
        cams = [look_at((0.3, 0.1, -4.0), (0.0, 0.0, 0.0), W, H, 60.0)]
    elif case == "medium-orbit8":
        sc = scenes.make_scene("medium", P=100_000)
        W, H = 641, 359
        cams = [scenes.camera_for("medium", i, W=W, H=H) for i in range(8)]
    else:  # city1M-540p: three nearby viewpoints of the city scene
        sc = scenes.make_scene("city", P=1_000_000)
        W, H = 960, 540
        base = scenes.camera_for("city", W=W, H=H)
        pitch = math.radians(-30.0)
        fwd = np.array([0.0, math.sin(pitch), math.cos(pitch)])
        cams = [base]
        for dx in (-6.0, 9.0):
            eye = np.array([dx, 80.0, 2.0])
            cams.append(look_at(eye, eye + fwd, W, H, 70.0))
    return sc, cams, W, H


def _check_batch(R, gsc, h, cams, W, H, o, tag):
    ref = [_np(R.render(gsc, c, W, H, o, want_T=True, want_last=True, prepared=h)) for c in cams]
    got = [_np(x) for x in R.render_batch(h, gsc, cams, W, H, o, want_T=True, want_last=True)]
    for i, (a, b) in enumerate(zip(ref, got)):
        for k in ("rgb", "T", "last"):
            assert np.array_equal(a[k].view(np.uint32), b[k].view(np.uint32)), (tag, i, k)
        for k in ("visible", "pairs", "big_chunks", "tiles_x", "tiles_y", "sort_passes"):
            assert a["stats"][k] == b["stats"][k], (tag, i, k)
        # the batch's candidates are the union over its cameras
        assert b["stats"]["candidates"] >= a["stats"]["candidates"], (tag, i)
    cand = {b["stats"]["candidates"] for b in got}
    assert len(cand) == 1, cand
    print(f"[batch] {tag}: {len(cams)} cameras, pairs {[b['stats']['pairs'] for b in got]}, "
          f"union candidates {cand.pop()}", flush=True)
    return got


@pytest.mark.parametrize("case", ["small-4", "small-1", "medium-orbit8", "city1M-540p"])
def test_batch_is_bit_identical_to_single_renders(orc, scenes, case):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_07967_amd.render import GaussianScene, Renderer
    sc, cams, W, H = _cases(scenes, case)
    print(f"[batch] {case}: P={sc.P} {W}x{H} cameras={len(cams)}", flush=True)
    R = Renderer()
    gsc = GaussianScene.from_numpy(sc)
    o = opts()
    h = R.prepare(gsc, o)
    try:
        got = _check_batch(R, gsc, h, cams, W, H, o, case)
    finally:
        R.release_prepared(h)
        R.close()
    if case != "city1M-540p":
        check_image(got[0], orc.render(sc, cams[0], W, H, o, mode="f64"), case)
    if case == "small-4":
        assert got[3]["stats"]["visible"] == 0 and got[3]["stats"]["pairs"] == 0
        assert np.all(got[3]["rgb"] == 0.0) and np.all(got[3]["T"] == 1.0)


@pytest.mark.parametrize("seed", [600, 601, 602])
def test_batch_random_camera_poses(scenes, seed):
    """Up to eight cameras at seeded random poses around and inside one scene
    (so that each camera's cull would skip other batches): the batch's union
    cull skips only batches that every camera culls, and every camera's images
    equal its single render bit for bit."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_07967_amd.render import GaussianScene, Renderer
    rng = np.random.default_rng(seed)
    box = float(rng.uniform(3.0, 8.0))
    sc = random_scene(rng, 40000, box=box, ls_mu=-2.2, ls_sigma=0.5, sh_degree=int(rng.integers(0, 4)))
    W, H = 320, 200
    cams = []
    for _ in range(int(rng.integers(2, 9))):
        eye = rng.uniform(-1.5 * box, 1.5 * box, 3) + np.array([0.0, 0.0, 4.0])
        target = rng.uniform(-box, box, 3) + np.array([0.0, 0.0, 4.0])
        cams.append(scenes.look_at(eye, target, W, H, float(rng.uniform(40.0, 90.0))))
    print(f"[batch] random poses {seed}: P={sc.P} box {box:.1f} cameras={len(cams)}", flush=True)
    R = Renderer()
    gsc = GaussianScene.from_numpy(sc)
    o = opts()
    h = R.prepare(gsc, o)
    try:
        _check_batch(R, gsc, h, cams, W, H, o, f"poses{seed}")
    finally:
        R.release_prepared(h)
        R.close()


def test_batch_buffers_grow_between_batches(scenes):
    """A fresh context renders a small batch first (its pair buffers are sized
    by it), then a batch with many more pairs per camera, then the small one
    again: every camera still matches its single render."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_07967_amd.render import GaussianScene, Renderer
    sc = scenes.make_scene("medium", P=100_000)
    o = opts()
    R = Renderer()
    gsc = GaussianScene.from_numpy(sc)
    h = R.prepare(gsc, o)
    try:
        small = [scenes.camera_for("medium", i, W=160, H=90) for i in (0, 3)]
        big = [scenes.camera_for("medium", i, W=1920, H=1080) for i in (0, 2, 5)]
        before = R.scratch_bytes()
        _check_batch(R, gsc, h, small, 160, 90, o, "grow-1")
        mid = R.scratch_bytes()
        # the batch's per-camera buffers are counted in the context's scratch
        assert mid > before
        _check_batch(R, gsc, h, big, 1920, 1080, o, "grow-2")
        assert R.scratch_bytes() > mid
        _check_batch(R, gsc, h, small, 160, 90, o, "grow-3")
    finally:
        R.release_prepared(h)
        R.close()


def test_batch_chunk_lists_overflow_and_resize():
    """600 screen-filling Gaussians at 4K need far more large-rectangle chunk
    entries than a fresh context's lists hold, for every camera of the batch:
    the batch resizes each camera's list and renders again, and every camera
    still matches its single render."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_07967_amd.render import GaussianScene, Renderer
    from paper_2408_07967_amd.scenes import Camera
    rng = np.random.default_rng(32)
    P = 600
    means = np.c_[rng.uniform(-0.3, 0.3, P), rng.uniform(-0.2, 0.2, P), rng.uniform(5, 9, P)]
    sc = scene_from(means, np.full((P, 3), 1.2), rng.normal(size=(P, 4)), rng.normal(0, 1, P),
                    dc_rgb=rng.uniform(0, 1, (P, 3)))
    W, H = 3840, 2160
    base = identity_camera(W, H, 1500.0)
    cams = [base]
    for dx in (0.2, -0.35):
        t = np.asarray(base.t, np.float32) + np.float32([dx, 0.0, 0.0])
        cams.append(Camera(base.R, t, np.asarray(base.eye, np.float32) - np.float32([dx, 0.0, 0.0]), base.fx,
                           base.fy, base.cx, base.cy, base.near, W, H))
    o = opts()
    R = Renderer()
    gsc = GaussianScene.from_numpy(sc)
    h = R.prepare(gsc, o)
    try:
        got = _check_batch(R, gsc, h, cams, W, H, o, "overflow")
    finally:
        R.release_prepared(h)
        R.close()
    assert all(g["stats"]["big_chunks"] > P for g in got)


def test_batch_rejects_bad_camera_counts(scenes):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_07967_amd import binding as B
    from paper_2408_07967_amd.render import GaussianScene, Renderer
    sc = scenes.make_scene("small")
    cam = scenes.camera_for("small")
    R = Renderer()
    gsc = GaussianScene.from_numpy(sc)
    h = R.prepare(gsc, opts())
    try:
        with pytest.raises(B.FgsError, match="ncams"):
            R.render_batch(h, gsc, [cam] * (B.MAX_BATCH_CAMERAS + 1), 64, 64, opts())
        with pytest.raises(B.FgsError, match="ncams"):
            R.render_batch(h, gsc, [], 64, 64, opts())
    finally:
        R.release_prepared(h)
        R.close()
