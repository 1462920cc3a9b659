"""GPU parity at the full sizes of the benchmark workloads, compared in full
(the oracle finishes each frame in seconds): per-Gaussian state, depth order,
every sorted pair and the tile ranges bit-exact against the FP32 oracle;
image, final transmittance and last contributor against the FP64 oracle at
the stated bar (|diff| <= 2e-3 on >= 99.9 % of pixels, mean |diff| <= 1e-5).

* 10M-Gaussian city scene at 3840x2160 (the timed workload), from the
  prepared scene and from the raw parameters (which must agree bit for bit);
* the same scene at 7680x4320 (the stress case: 129,600 tiles in 2040
  super-tiles, whose ids are sorted in two passes);
* the 1M-Gaussian orbit scene at 1920x1080 through all eight orbit cameras,
  one request at a time.

At 4K the oracle's own binary32 mode misses the mean bar (about 1.4e-5): its
binary32 inverse of the dilated 2D covariance loses the narrow axis of long
thin footprints.  The renderer keeps that binary32 conic for the tile test
(so the pairs stay bit-exact) and blends with the conic evaluated in binary64
and rounded once, which meets the bar; the test logs the binary32 oracle's
mean and that of a binary64 blend over the binary32 state beside it."""
import time

import numpy as np
import pytest

from gpu_helpers import (IMG_FRAC, IMG_MAX, IMG_MEAN, check_blend_conic, check_gauss_state, check_pairs, gpu_frame,
                         image_error)
from oracle_helpers import opts

pytestmark = pytest.mark.gpu


def _log(msg):
    print(f"[fullsize] {msg}", flush=True)


def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _compare_images(orc, g, o32, o64, tag):
    """Image and T against binary64 at the stated bar; last contributor."""
    check_blend_conic(g, o64, tag)
    for key in ("rgb", "T"):
        _, _, ref_mean = image_error(o32[key], o64[key])
        mx, frac, mean = image_error(g[key], o64[key])
        _log(f"{tag} {key}: max {mx:.3g} within {IMG_MAX}: {frac:.6f} mean {mean:.3g} "
             f"(binary32 oracle mean {ref_mean:.3g})")
        assert frac >= IMG_FRAC, (tag, key, frac)
        assert mean <= IMG_MEAN, (tag, key, mean)
    agree = (g["last"] == o64["last"]).mean()
    agree32 = (g["last"] == o32["last"]).mean()
    _log(f"{tag} last contributor: {agree:.5f} equal to binary64, {agree32:.5f} to binary32")
    assert agree >= 0.995 and agree32 >= 0.995, (tag, agree, agree32)


def _city(orc, scenes, W, H, both_paths):
    from paper_2408_07967_amd.render import GaussianScene, Renderer
    t0 = time.perf_counter()
    sc = scenes.make_scene("city")
    cam = scenes.camera_for("city", W=W, H=H)
    o = opts()
    assert sc.P == 10_000_000
    _log(f"scene P={sc.P} {W}x{H} drawn in {time.perf_counter() - t0:.1f}s")
    R = Renderer()
    gsc = GaussianScene.from_numpy(sc, "cuda:0")
    h = R.prepare(gsc, o)
    try:
        g = gpu_frame(R, gsc, cam, W, H, o, prepared=h)
        graw = gpu_frame(R, gsc, cam, W, H, o) if both_paths else None  # the raw-parameter path, same frame
    finally:
        R.release_prepared(h)
        del gsc
        R.close()
    _log(f"GPU frame: visible {g['stats']['visible']} pairs {g['stats']['pairs']} "
         f"candidates {g['stats']['candidates']} sort passes {g['stats']['sort_passes']}")

    o32 = orc.render(sc, cam, W, H, o, mode="f32")
    _log(f"oracle binary32 frame done ({time.perf_counter() - t0:.1f}s)")
    for tag, gx in (("prepared", g), ("raw parameters", graw)):
        if gx is None:
            continue
        check_gauss_state(orc, gx, o32)
        check_pairs(gx, o32)
        _log(f"{tag}: state, depth order, pairs and ranges bit-exact")
    if graw is not None:
        for k in ("rgb", "T", "last"):
            assert np.array_equal(np.asarray(g[k]).view(np.uint32), np.asarray(graw[k]).view(np.uint32)), k
    o64 = orc.render(sc, cam, W, H, o, mode="f64")
    _log(f"oracle binary64 frame done ({time.perf_counter() - t0:.1f}s)")
    # information: a binary64 blend over the binary32 state and pairs
    rgb_b, _, _ = orc.blend_tiled(o64["prep"], o32["state"].astype(np.float64), o32["vals"], o32["ranges"])
    _log(f"binary64 blend over the binary32 state: mean {image_error(rgb_b, o64['rgb'])[2]:.3g}")
    del rgb_b
    _compare_images(orc, g, o32, o64, f"city {W}x{H}")
    return g


@pytest.mark.timeout(900)
def test_city_10M_4k_prepared_full_size(orc, scenes):
    _gpu()
    g = _city(orc, scenes, 3840, 2160, both_paths=True)
    assert g["stats"]["sort_passes"] == 4 + 1  # 510 super-tiles: one 9-bit pass


@pytest.mark.timeout(900)
def test_city_10M_8k_full_size(orc, scenes):
    """The 7680x4320 stress case: 129,600 tiles (> 65,536) in 2040
    super-tiles, whose ids are sorted in two passes."""
    _gpu()
    g = _city(orc, scenes, 7680, 4320, both_paths=False)
    assert g["stats"]["sort_passes"] == 4 + 2


@pytest.mark.timeout(600)
def test_medium_1M_1080p_eight_cameras_full_size(orc, scenes):
    """The 1M-Gaussian orbit scene at 1920x1080 through all eight cameras of
    the radius-10 orbit, one request at a time from the raw parameters (and
    camera 0 from the prepared scene as well)."""
    _gpu()
    from paper_2408_07967_amd.render import GaussianScene, Renderer
    sc = scenes.make_scene("medium")
    assert sc.P == 1_000_000
    o = opts()
    R = Renderer()
    gsc = GaussianScene.from_numpy(sc, "cuda:0")
    h = R.prepare(gsc, o)
    try:
        for k in range(8):
            cam = scenes.camera_for("medium", k)
            g = gpu_frame(R, gsc, cam, 1920, 1080, o)
            o32 = orc.render(sc, cam, 1920, 1080, o, mode="f32")
            check_gauss_state(orc, g, o32)
            check_pairs(g, o32)
            o64 = orc.render(sc, cam, 1920, 1080, o, mode="f64")
            _log(f"camera {k}: visible {g['stats']['visible']} pairs {g['stats']['pairs']}: state, order, pairs "
                 f"bit-exact")
            _compare_images(orc, g, o32, o64, f"medium camera {k}")
            if k == 0:
                gp = gpu_frame(R, gsc, cam, 1920, 1080, o, prepared=h)
                for key in ("rgb", "T", "last"):
                    assert np.array_equal(np.asarray(gp[key]).view(np.uint32), np.asarray(g[key]).view(np.uint32))
    finally:
        R.release_prepared(h)
        R.close()
