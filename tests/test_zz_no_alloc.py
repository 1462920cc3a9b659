"""GPU test of fgs_render_noalloc, the render entry point whose kernels take
every scratch buffer from the library's fixed per-GPU array: two calls in a
row (the second with fewer Gaussians and a smaller image) must give the image,
final transmittance and last contributor of fgs_render bit for bit, through
the C ABI; frames that do not fit are refused with FGS_ERR_CAPACITY, and the
entry point works again after a refusal."""
import ctypes as C

import numpy as np
import pytest

from oracle_helpers import identity_camera, random_scene, opts

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2408_07967_amd.render import Renderer
    r = Renderer()
    yield r
    r.close()


def _noalloc(R, gsc, cam, W, H, o):
    """fgs_render_noalloc through the ctypes prototype of the ABI; returns
    (status, rgb, T, last, stats)."""
    import torch
    from paper_2408_07967_amd import binding as B
    from paper_2408_07967_amd.render import camera_abi, options_abi
    rgb = torch.full((3, H, W), -1.0, dtype=torch.float32, device="cuda")
    T = torch.full((H, W), -1.0, dtype=torch.float32, device="cuda")
    last = torch.full((H, W), -1, dtype=torch.int32, device="cuda")
    sc, cm, op, st = gsc.abi(), camera_abi(cam), options_abi(o), B.FgsStats()
    stream = torch.cuda.current_stream().cuda_stream
    status = B.lib().fgs_render_noalloc(R.ctx.handle, C.byref(sc), C.byref(cm), int(W), int(H), C.byref(op),
                                        rgb.data_ptr(), T.data_ptr(), last.data_ptr(), C.byref(st), stream)
    torch.cuda.synchronize()
    return status, rgb.cpu().numpy(), T.cpu().numpy(), last.cpu().numpy(), st


def _same_as_render(R, scene, cam, W, H, o, tag):
    from paper_2408_07967_amd import binding as B
    from paper_2408_07967_amd.render import GaussianScene
    import torch
    print(f"[noalloc] {tag}: P={scene.P} {W}x{H}", flush=True)
    gsc = GaussianScene.from_numpy(scene)
    status, rgb, T, last, st = _noalloc(R, gsc, cam, W, H, o)
    assert status == B.FGS_OK, (status, B.lib().fgs_last_error(R.ctx.handle))
    ref = R.render(gsc, cam, W, H, o, want_T=True, want_last=True)
    torch.cuda.synchronize()
    assert st.pairs == ref["stats"]["pairs"] and st.visible == ref["stats"]["visible"], tag
    for name, a, b in (("rgb", rgb, ref["rgb"]), ("T", T, ref["T"]), ("last", last, ref["last"])):
        b = b.cpu().numpy()
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), f"{tag} {name} differs from fgs_render"
    print(f"[noalloc] {tag}: {st.pairs} pairs, bit-identical to fgs_render", flush=True)
    return st


def test_noalloc_two_calls_match_render(R, scenes):
    # first call: 200k Gaussians of the 1M orbit scene at 1920x1080
    sc = scenes.make_scene("medium", P=200_000)
    st1 = _same_as_render(R, sc, scenes.camera_for("medium", 0), 1920, 1080, opts(), "medium200k-1080p")
    # second call, smaller: 3,000 Gaussians at a ragged 333x97; what the first
    # call left in the array must not leak into it
    rng = np.random.default_rng(12)
    sc2 = random_scene(rng, 3000, ls_mu=-2.8, sh_degree=2)
    st2 = _same_as_render(R, sc2, identity_camera(333, 97, 0.9 * 333), 333, 97, opts(), "random3000-333x97")
    assert st2.pairs < st1.pairs


def test_noalloc_refuses_what_does_not_fit(R):
    from paper_2408_07967_amd import binding as B
    from paper_2408_07967_amd.render import GaussianScene
    rng = np.random.default_rng(21)
    # per-Gaussian buffers alone beyond the array: refused before device work
    big = random_scene(rng, 600_000, ls_mu=-3.0, sh_degree=0)
    status, *_ = _noalloc(R, GaussianScene.from_numpy(big), identity_camera(64, 64, 60.0), 64, 64, opts())
    msg = B.lib().fgs_last_error(R.ctx.handle).decode()
    print(f"[noalloc] 600k Gaussians: status {status}: {msg}", flush=True)
    assert status == B.FGS_ERR_CAPACITY and "fixed scratch" in msg
    # more pairs than the pair arrays hold: refused after the frame's counters
    # (150k Gaussians of about 30 tiles each: 4.4M pairs against room for
    # about 2.7M; 7.4k large-rectangle chunks, within the chunk list)
    many = random_scene(rng, 150_000, ls_mu=-2.9, ls_sigma=0.3, sh_degree=0)
    cam = identity_camera(1024, 1024, 900.0)
    status, *_ = _noalloc(R, GaussianScene.from_numpy(many), cam, 1024, 1024, opts())
    msg = B.lib().fgs_last_error(R.ctx.handle).decode()
    print(f"[noalloc] 150k large Gaussians: status {status}: {msg}", flush=True)
    assert status == B.FGS_ERR_CAPACITY and "pairs" in msg
    # and the entry point renders correctly again afterwards
    sc = random_scene(np.random.default_rng(13), 800, ls_mu=-1.6, sh_degree=3)
    _same_as_render(R, sc, identity_camera(64, 64, 0.9 * 64), 64, 64, opts(), "random800-64x64 after refusals")
