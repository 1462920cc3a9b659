"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Per-Gaussian state, visible set, depth order, the
sorted (tile, Gaussian) pair list and tile ranges are bit-exact against the
oracle's FP32 mode; images and final transmittance are within the stated
tolerance of the FP64 oracle."""
import numpy as np
import pytest

from gpu_helpers import gpu_frame, check_gauss_state, check_pairs, check_image, image_error
from oracle_helpers import identity_camera, random_scene, scene_from, opts

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


def _gs(scene):
    from paper_2408_07967_amd.render import GaussianScene
    return GaussianScene.from_numpy(scene)


def _full_check(orc, R, scene, cam, W, H, o, tag):
    print(f"[parity] {tag}: P={scene.P} {W}x{H}", flush=True)
    g = gpu_frame(R, _gs(scene), cam, W, H, o)
    o32 = orc.render(scene, cam, W, H, o, mode="f32")
    check_gauss_state(orc, g, o32)
    check_pairs(g, o32)
    o64 = orc.render(scene, cam, W, H, o, mode="f64")
    check_image(g, o64, tag)
    agree = (g["last"] == o32["last"]).mean()
    assert agree >= 0.995, f"{tag}: last agreement {agree}"
    return g, o32, o64


def test_small_scene_full(orc, R, scenes):
    sc = scenes.make_scene("small")
    _full_check(orc, R, sc, scenes.camera_for("small"), 256, 256, opts(), "small")


@pytest.mark.parametrize("seed,P,W,H,deg,ls_mu", [
    (11, 500, 200, 136, 1, -2.5),     # ragged tiles
    (12, 3000, 333, 97, 2, -2.8),
    (13, 800, 64, 64, 3, -1.6),       # large footprints: wave-cooperative paths, > 64 tiles
    (14, 20000, 517, 301, 3, -3.2),   # several sort / scan workgroups
])
def test_random_scenes(orc, R, seed, P, W, H, deg, ls_mu):
    rng = np.random.default_rng(seed)
    sc = random_scene(rng, P, ls_mu=ls_mu, sh_degree=deg)
    cam = identity_camera(W, H, 0.9 * max(W, H))
    _full_check(orc, R, sc, cam, W, H, opts(), f"random{seed}")


@pytest.mark.parametrize("seed,P,W,H,ls_mu", [
    (501, 60000, 2049, 1201, -1.6),   # ~10^5 chunks: Gaussians over many 64-slot windows, ragged super-tiles
    (502, 20000, 1023, 511, -1.1),    # rectangles up to the whole image, more tile rows per chunk
])
def test_dense_large_rectangles(orc, R, seed, P, W, H, ls_mu):
    """Frames whose pairs mostly come from chunked rectangles (hundreds of
    thousands of 256-tile chunks), on images that are not a whole number of
    super-tiles: state, order, pairs and ranges bit-exact against the
    binary32 oracle, the image against binary64, and the prepared scene's
    frame equal to the raw one."""
    rng = np.random.default_rng(seed)
    sc = random_scene(rng, P, box=2.0, ls_mu=ls_mu, ls_sigma=0.6, sh_degree=2)
    cam = identity_camera(W, H, 0.8 * W)
    g, _, _ = _full_check(orc, R, sc, cam, W, H, opts(), f"dense-large-{seed}")
    assert g["stats"]["big_chunks"] > 10000, g["stats"]["big_chunks"]
    gsc = _gs(sc)
    h = R.prepare(gsc, opts())
    try:
        p = gpu_frame(R, gsc, cam, W, H, opts(), prepared=h)
    finally:
        R.release_prepared(h)
    for k in ("rgb", "T", "last", "order", "tiles", "values", "ranges"):
        assert np.array_equal(np.asarray(g[k]).view(np.uint32), np.asarray(p[k]).view(np.uint32)), k


def test_medium_scene_reduced(orc, R, scenes):
    sc = scenes.make_scene("medium", P=200_000)
    _full_check(orc, R, sc, scenes.camera_for("medium", 0), 1920, 1080, opts(), "medium200k")


def test_city_scene_reduced(orc, R, scenes):
    sc = scenes.make_scene("city", P=1_000_000)
    _full_check(orc, R, sc, scenes.camera_for("city", W=960, H=540), 960, 540, opts(), "city1M-540p")


def test_wide_depth_span(orc, R):
    """Depths from 0.3 to 2e6 (the visible depth keys span more than 2^27
    binary32 values, about 16 binades, with different high key bits): raw
    frame against the binary32 oracle, state, order and pairs bit-exact; the
    prepared frame equal to it."""
    rng = np.random.default_rng(37)
    n = 4000
    z = np.exp(rng.uniform(np.log(0.3), np.log(2.0e6), n))
    means = np.stack([rng.uniform(-0.6, 0.6, n) * z, rng.uniform(-0.4, 0.4, n) * z, z], 1)
    ls = np.log(0.02 * z)[:, None] + rng.normal(0, 0.3, (n, 3))
    q = rng.normal(size=(n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    sc = scene_from(means, ls, q, rng.normal(1.0, 1.0, n), sh=rng.normal(0, 0.4, (3, n)), sh_degree=0)
    W, H = 320, 200
    cam = identity_camera(W, H, 0.8 * W)
    g, o32, _ = _full_check(orc, R, sc, cam, W, H, opts(), "wide_depth_span")
    d = g["gauss"][g["order"].astype(np.int64), 10].view(np.uint32).astype(np.int64)
    span = int(d.max()) - (int(d.min()) & ~511)
    print(f"[parity] wide_depth_span: {d.size} visible, key span 2^{np.log2(span):.2f}", flush=True)
    assert span >> 27 != 0
    gsc = _gs(sc)
    h = R.prepare(gsc, opts())
    try:
        b = gpu_frame(R, gsc, cam, W, H, opts(), prepared=h)
    finally:
        R.release_prepared(h)
    for k in ("order", "tiles", "values", "ranges", "rgb"):
        assert np.array_equal(np.asarray(g[k]).view(np.uint32), np.asarray(b[k]).view(np.uint32)), k


def test_empty_scene_is_background(orc, R):
    import torch
    from paper_2408_07967_amd.render import GaussianScene
    z = torch.zeros((3, 0), device="cuda")
    gsc = GaussianScene(z, z.clone(), torch.zeros((4, 0), device="cuda"), torch.zeros((1, 0), device="cuda"),
                        torch.zeros((3, 0), device="cuda"), 0)
    out = R.render(gsc, identity_camera(37, 21, 30), 37, 21, opts(bg=(0.25, 0.5, 0.75)), want_T=True)
    torch.cuda.synchronize()
    rgb = out["rgb"].cpu().numpy()
    assert np.allclose(rgb[0], 0.25) and np.allclose(rgb[1], 0.5) and np.allclose(rgb[2], 0.75)
    assert np.all(out["T"].cpu().numpy() == 1.0) and out["stats"]["pairs"] == 0


def test_all_culled_and_degenerate(orc, R):
    # behind the camera, zero quaternion, NaN mean, infinite scale, tiny opacity
    sc = scene_from([(0, 0, -3), (0, 0, 3), (np.nan, 0, 3), (0, 0, 3), (0, 0, 3)],
                    [(-3,) * 3, (-3,) * 3, (-3,) * 3, (np.inf, -3, -3), (-3,) * 3],
                    [(1, 0, 0, 0), (0, 0, 0, 0), (1, 0, 0, 0), (1, 0, 0, 0), (1, 0, 0, 0)],
                    [2.0, 2.0, 2.0, 2.0, -12.0], dc_rgb=(1, 1, 1))
    cam = identity_camera(48, 40, 40)
    g = gpu_frame(R, _gs(sc), cam, 48, 40, opts())
    o32 = orc.render(sc, cam, 48, 40, opts(), mode="f32")
    assert o32["ints"][:, 0].sum() == 0 and g["order"].size == 0 and g["stats"]["pairs"] == 0
    assert np.all(g["rgb"] == 0) and np.all(g["T"] == 1)


def test_one_pixel_and_one_tile_images(orc, R, scenes):
    rng = np.random.default_rng(21)
    sc = random_scene(rng, 300, ls_mu=-2.0, sh_degree=0)
    for W, H in ((1, 1), (16, 16), (17, 1), (1, 33)):
        cam = identity_camera(W, H, 20.0)
        _full_check(orc, R, sc, cam, W, H, opts(), f"{W}x{H}")


def test_wide_image_with_32bit_tile_ids(orc, R):
    """More than 65536 tiles (16384 x 1040 = 66560): tile ids need more than
    16 bits; the entries' 1152 super-tile ids (128 x 9, 11 bits) are sorted in
    two passes."""
    from oracle_helpers import scene_from
    rng = np.random.default_rng(23)
    P = 4000
    means = np.stack([rng.uniform(-30, 30, P), rng.uniform(-2.5, 2.5, P), rng.uniform(5, 7, P)], 1)
    q = rng.normal(size=(P, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    sc = scene_from(means, rng.normal(-1.5, 0.5, (P, 3)), q, rng.normal(0, 1.5, P), sh_degree=1,
                    sh=rng.normal(0, 0.3, (12, P)))
    W, H = 16384, 1040
    g, o32, _ = _full_check(orc, R, sc, identity_camera(W, H, 1000.0), W, H, opts(), f"{W}x{H}")
    assert g["stats"]["sort_passes"] == 4 + 2
    assert g["stats"]["pairs"] > 100_000


def test_bbox_binning_same_image_more_pairs(orc, R, scenes):
    sc = scenes.make_scene("small")
    cam = scenes.camera_for("small")
    a = gpu_frame(R, _gs(sc), cam, 256, 256, opts(binning=0))
    b = gpu_frame(R, _gs(sc), cam, 256, 256, opts(binning=1))
    o32 = orc.render(sc, cam, 256, 256, opts(binning=1), mode="f32")
    check_pairs(b, o32)
    assert b["stats"]["pairs"] > a["stats"]["pairs"]
    mx, frac, mean = image_error(a["rgb"], b["rgb"])
    assert mx < 1e-5, mx


@pytest.mark.parametrize("kind,P,W,H", [("small", None, 256, 256), ("medium", 150_000, 960, 540)])
def test_3sigma_square_binning_parity(orc, R, scenes, kind, P, W, H):
    """binning = 2: state, pairs and order bit-exact against the FP32 oracle
    in the same mode; the image equals the exact-binning image."""
    sc = scenes.make_scene(kind, P=P)
    cam = scenes.camera_for(kind, W=W, H=H)
    g, _, _ = _full_check(orc, R, sc, cam, W, H, opts(binning=2), f"{kind}-binning2")
    a = gpu_frame(R, _gs(sc), cam, W, H, opts(binning=0))
    assert g["stats"]["pairs"] > a["stats"]["pairs"]
    mx, frac, mean = image_error(a["rgb"], g["rgb"])
    assert mx < 1e-5, mx


@pytest.mark.parametrize("case", ["small", "random_sh3", "degenerate", "medium_binning2", "uncapped",
                                  "offscreen_big", "offscreen_big_binning2", "ties_short", "ties_long",
                                  "ties_one_run", "city1M-540p", "sh_huge", "eye_at_mean", "wide_batches", "one_gaussian",
                                  "one_behind", "all_transparent"])
def test_prepared_scene_is_bit_identical(orc, R, scenes, case):
    """A frame from the view-independent precompute equals the frame from the
    raw parameters bit for bit (state, pairs, order, image, T, last).  The
    precompute holds the Gaussians in a spatial order, so equal depths leave
    its depth sort in that order and are re-ordered by Gaussian index; the
    ties cases put many Gaussians at exactly equal depths: runs of 2 to 30
    (sorted by one thread each), runs of about 60 (sorted by a workgroup in
    LDS), and one run of 6000 (sorted in 1024-chunks and merged).

    The colour decides visibility too (a non-finite colour culls): a
    non-finite coefficient ("degenerate"), a zero view direction
    ("eye_at_mean": the camera centre given on a visible Gaussian's mean,
    0 / 0 in the basis) and coefficients near the binary32 maximum, which
    overflow the colour from some directions only ("sh_huge"), must cull the
    same Gaussians on both paths and in the binary32 oracle."""
    o = opts()
    if case.startswith("ties"):
        rng = np.random.default_rng({"ties_short": 41, "ties_long": 42, "ties_one_run": 43}[case])
        n = 6000
        sc = random_scene(rng, n, ls_mu=-3.4, ls_sigma=0.3, sh_degree=1)
        levels = {"ties_short": 600, "ties_long": 100, "ties_one_run": 1}[case]
        # identity camera: the depth is the mean's z, exactly
        sc.means[2] = (np.float32(4.0) + np.float32(0.01) * rng.integers(0, levels, n).astype(np.float32))
        W, H = 320, 240
        cam = identity_camera(W, H, 0.9 * W)
    elif case == "city1M-540p":
        sc = scenes.make_scene("city", P=1_000_000)
        W, H = 960, 540
        cam = scenes.camera_for("city", W=W, H=H)
    elif case == "small":
        sc, cam, W, H = scenes.make_scene("small"), scenes.camera_for("small"), 256, 256
    elif case == "random_sh3":
        sc = random_scene(np.random.default_rng(31), 4000, ls_mu=-2.4, sh_degree=3)
        W, H = 301, 177
        cam = identity_camera(W, H, 0.9 * W)
    elif case == "degenerate":
        rng = np.random.default_rng(32)
        sc = random_scene(rng, 600, ls_mu=-2.0, sh_degree=2)
        sc.means[0, 5] = np.nan
        sc.log_scales[1, 6] = np.inf
        sc.quats[:, 7] = 0.0
        sc.logits[0, 8] = -9.0      # below the opacity threshold
        sc.sh[4, 9] = np.nan
        sc.means[2, 10] = -1.0      # behind the camera
        W, H = 96, 80
        cam = identity_camera(W, H, 70.0)
    elif case == "sh_huge":
        rng = np.random.default_rng(34)
        sc = random_scene(rng, 3000, ls_mu=-2.6, sh_degree=2)
        # band-1 and band-2 coefficients of one colour channel near the
        # binary32 maximum, of mixed signs: the sum overflows for some view
        # directions and not for others
        idx = rng.choice(sc.P, 400, replace=False)
        for k in (1, 2, 3, 4, 6):
            sc.sh[3 * k, idx] = np.float32(3.0e38) * rng.choice([-1.0, 1.0], idx.size).astype(np.float32)
        W, H = 240, 160
        cam = identity_camera(W, H, 0.9 * W)
    elif case == "eye_at_mean":
        rng = np.random.default_rng(35)
        sc = random_scene(rng, 2000, ls_mu=-2.4, sh_degree=1)
        W, H = 160, 120
        cam = identity_camera(W, H, 0.9 * W)
        # the camera centre on the mean of a Gaussian the camera sees (its
        # view-space depth stays positive: eye and R, t are separate inputs)
        j = int(np.argmin(np.abs(sc.means[0]) + np.abs(sc.means[1])))
        cam.eye = sc.means[:, j].astype(np.float32).copy()
        sc.logits[0, j] = np.float32(4.0)
    elif case == "medium_binning2":
        sc = scenes.make_scene("medium", P=120_000)
        W, H = 960, 540
        cam = scenes.camera_for("medium", 3, W=W, H=H)
        o = opts(binning=2)
    elif case.startswith("offscreen_big"):
        # wide, elongated Gaussians centred off the image whose footprints
        # reach into it: the cull of a prepared scene must keep them
        rng = np.random.default_rng(33)
        sc = random_scene(rng, 3000, box=3.0, ls_mu=-1.2, ls_sigma=0.8, sh_degree=1)
        W, H = 200, 120
        cam = identity_camera(W, H, 60.0)
        o = opts(binning=2) if case.endswith("binning2") else opts()
    elif case in ("one_gaussian", "one_behind"):
        # one partial batch of one slot, in view or wholly behind the camera
        z = 3.0 if case == "one_gaussian" else -3.0
        sc = scene_from([(0.1, -0.05, z)], [(-1.5,) * 3], [(1, 0, 0, 0)], [2.0], dc_rgb=(0.8, 0.4, 0.2))
        W, H = 64, 48
        cam = identity_camera(W, H, 50.0)
    elif case == "all_transparent":
        # every opacity below the threshold: each batch is skipped by its
        # greatest opacity alone
        rng = np.random.default_rng(38)
        sc = random_scene(rng, 3000, ls_mu=-2.0, sh_degree=1)
        sc.logits[:] = np.float32(-7.0)
        W, H = 160, 120
        cam = identity_camera(W, H, 0.9 * W)
    elif case == "wide_batches":
        # about 200 spatial batches over a box that reaches behind the
        # camera: batches wholly behind it, across its near plane, off the
        # image, and off the image with footprints that reach into it; the
        # batch bounds may skip only batches with no candidate
        rng = np.random.default_rng(36)
        sc = random_scene(rng, 50_000, box=8.0, ls_mu=-1.3, ls_sigma=0.8, sh_degree=1)
        W, H = 200, 120
        cam = identity_camera(W, H, 60.0)
    else:
        sc, cam, W, H = scenes.make_scene("small"), scenes.camera_for("small"), 256, 256
        o = opts(cap_3sigma=0, alpha_min=0.01)
    print(f"[parity] prepared scene: {case} P={sc.P} {W}x{H}", flush=True)
    gsc = _gs(sc)
    h = R.prepare(gsc, o)
    try:
        a = gpu_frame(R, gsc, cam, W, H, o)
        b = gpu_frame(R, gsc, cam, W, H, o, prepared=h)
    finally:
        R.release_prepared(h)
    if case == "eye_at_mean":
        # the raw path culls that Gaussian through its NaN colour
        assert j not in set(a["order"].tolist())
    if case in ("sh_huge", "eye_at_mean"):
        # the raw frame against the binary32 oracle (the prepared frame
        # equals it bit for bit, below)
        o32 = orc.render(sc, cam, W, H, o, mode="f32")
        check_gauss_state(orc, a, o32)
        check_pairs(a, o32)
    if case.startswith("ties"):
        d = a["gauss"][a["order"].astype(np.int64), 10].view(np.uint32)
        runs = np.diff(np.flatnonzero(np.r_[True, d[1:] != d[:-1], True]))
        print(f"[parity] {case}: {a['stats']['visible']} visible, longest run of equal depths {runs.max()}, "
              f"runs over 32: {(runs > 32).sum()}", flush=True)
        assert runs.max() >= {"ties_short": 2, "ties_long": 33, "ties_one_run": 4000}[case]
    # the prepared scene preprocesses only the cull's candidates: never fewer
    # than the visible Gaussians, never more than the scene holds
    ca, cb = a["stats"].pop("candidates"), b["stats"].pop("candidates")
    assert ca == sc.P and a["stats"]["visible"] <= cb <= sc.P
    # the prepared scene's cull reads the batches its bounds keep
    nb = b["stats"].pop("cull_batches")
    assert a["stats"].pop("cull_batches") == 0 and nb <= (sc.P + 255) // 256
    # a batch holding a visible Gaussian is always read
    assert nb > 0 or a["stats"]["visible"] == 0
    if case in ("one_behind", "all_transparent"):
        assert nb == 0 and a["stats"]["visible"] == 0
    if case == "wide_batches":
        print(f"[parity] wide_batches: {nb} of {(sc.P + 255) // 256} batches read, {cb} candidates", flush=True)
        assert nb < (sc.P + 255) // 256
    assert a["stats"] == b["stats"]
    for k in ("rgb", "T", "last", "gauss", "rect", "count", "order", "tiles", "values", "ranges"):
        if k in ("gauss", "rect"):
            vis = a["order"].astype(np.int64)  # culled Gaussians have no state
            assert np.array_equal(a[k][vis].view(np.uint32), b[k][vis].view(np.uint32)), k
        else:
            assert np.array_equal(np.asarray(a[k]).view(np.uint32), np.asarray(b[k]).view(np.uint32)), k


def test_prepared_random_camera_poses(orc, R, scenes):
    """Sixteen seeded random camera poses, eyes inside and outside scene
    boxes of 2 to 10 units, fields of view of 30-100 degrees: the raw frame
    against the binary32 oracle (state, order, pairs bit-exact) and the
    prepared frame, whose cull skips 256-slot batches by their bounds, equal
    to it.  Some batches must be skipped over the set."""
    skipped = 0
    for seed in range(500, 516):
        rng = np.random.default_rng(seed)
        W = int(rng.choice([97, 256, 320, 640, 1000]))
        H = int(rng.choice([64, 180, 240, 480]))
        P = int(rng.choice([3000, 20000, 60000]))
        deg = int(rng.integers(0, 4))
        box = float(rng.uniform(2.0, 10.0))
        sc = random_scene(rng, P, box=box, ls_mu=float(rng.uniform(-3.0, -0.8)),
                          ls_sigma=float(rng.uniform(0.2, 0.9)), sh_degree=deg)
        eye = rng.uniform(-1.5 * box, 1.5 * box, 3) + np.array([0.0, 0.0, 4.0])
        target = rng.uniform(-box, box, 3) + np.array([0.0, 0.0, 4.0])
        cam = scenes.look_at(eye, target, W, H, float(rng.uniform(30.0, 100.0)))
        o = opts(binning=int(rng.choice([0, 0, 0, 2])))
        tag = f"pose{seed}"
        print(f"[parity] {tag}: P={P} {W}x{H} deg {deg} box {box:.1f}", flush=True)
        gsc = _gs(sc)
        g = gpu_frame(R, gsc, cam, W, H, o)
        o32 = orc.render(sc, cam, W, H, o, mode="f32")
        check_gauss_state(orc, g, o32)
        check_pairs(g, o32)
        h = R.prepare(gsc, o)
        try:
            p = gpu_frame(R, gsc, cam, W, H, o, prepared=h)
        finally:
            R.release_prepared(h)
        for k in ("rgb", "T", "last", "order", "tiles", "values", "ranges"):
            assert np.array_equal(np.asarray(g[k]).view(np.uint32), np.asarray(p[k]).view(np.uint32)), (tag, k)
        skipped += (P + 255) // 256 - p["stats"]["cull_batches"]
    print(f"[parity] random poses: {skipped} batches skipped", flush=True)
    assert skipped > 0


def test_backward_of_prepared_frame_not_supported(R, scenes):
    """A prepared scene's frame holds its state by candidate position: the
    adjoint is for frames rendered from the parameters, and says so."""
    import torch
    from paper_2408_07967_amd import binding as B
    sc = scenes.make_scene("small")
    cam = scenes.camera_for("small")
    gsc = _gs(sc)
    h = R.prepare(gsc, opts())
    try:
        out = R.render(gsc, cam, 256, 256, opts(), save=True, prepared=h)
        with pytest.raises(B.FgsError, match="not supported"):
            R.backward(out["frame"], gsc, cam, 256, 256, opts(), torch.ones((3, 256, 256), device="cuda"))
        R.release(out["frame"])
    finally:
        R.release_prepared(h)


@pytest.mark.parametrize("case", ["small", "random14", "city1M-540p"])
def test_prefetch_blend_variant_is_bit_identical(orc, R, scenes, case):
    """The prefetch-pipeline blend (no LDS staging, no half masks) renders the
    image, T_final and last contributor of the default blend bit for bit, and
    both meet the oracle's bar."""
    from paper_2408_07967_amd import binding as B
    if case == "small":
        sc, cam, W, H = scenes.make_scene("small"), scenes.camera_for("small"), 256, 256
    elif case == "random14":
        rng = np.random.default_rng(14)
        sc = random_scene(rng, 20000, ls_mu=-3.2, sh_degree=3)
        W, H = 517, 301
        cam = identity_camera(W, H, 0.9 * max(W, H))
    else:
        sc = scenes.make_scene("city", P=1_000_000)
        W, H = 960, 540
        cam = scenes.camera_for("city", W=W, H=H)
    print(f"[parity] blend variants: {case} P={sc.P} {W}x{H}", flush=True)
    gsc = _gs(sc)
    a = gpu_frame(R, gsc, cam, W, H, opts())
    R.set_blend_variant(B.BLEND_PREFETCH)
    try:
        b = gpu_frame(R, gsc, cam, W, H, opts())
    finally:
        R.set_blend_variant(B.BLEND_LDS_BATCHES)
    for k in ("rgb", "T", "last", "tiles", "values", "ranges"):
        assert np.array_equal(np.asarray(a[k]).view(np.uint32), np.asarray(b[k]).view(np.uint32)), k
    if case != "city1M-540p":
        check_image(b, orc.render(sc, cam, W, H, opts(), mode="f64"), case)


def test_deterministic_repeat(orc, R, scenes):
    sc = scenes.make_scene("medium", P=100_000)
    cam = scenes.camera_for("medium", 2)
    gsc = _gs(sc)
    a = gpu_frame(R, gsc, cam, 1920, 1080, opts())
    b = gpu_frame(R, gsc, cam, 1920, 1080, opts())
    for k in ("rgb", "T", "last", "order", "tiles", "values", "ranges"):
        assert np.array_equal(a[k], b[k]), k


def test_pair_buffers_grow_inside_a_frame(orc, scenes):
    """A fresh context renders a small frame, then one with far more pairs
    than its buffers hold: the second half, enqueued with the small buffers,
    runs again after they grow (every sort pass's group sums cleared again).
    The grown frame and a repeat of it are bit-exact against the oracle."""
    import torch
    from paper_2408_07967_amd.render import Renderer
    Rf = Renderer()
    try:
        small = scenes.make_scene("small")
        gpu_frame(Rf, _gs(small), scenes.camera_for("small"), 64, 64, opts())
        sc = scenes.make_scene("medium", P=200_000)
        cam = scenes.camera_for("medium", 3, W=1280, H=720)
        print("[parity] regrow: small 64x64, then medium P=200000 1280x720 twice", flush=True)
        gsc = _gs(sc)
        g1 = gpu_frame(Rf, gsc, cam, 1280, 720, opts())
        o32 = orc.render(sc, cam, 1280, 720, opts(), mode="f32")
        check_gauss_state(orc, g1, o32)
        check_pairs(g1, o32)
        g2 = gpu_frame(Rf, gsc, cam, 1280, 720, opts())
        for k in ("rgb", "T", "last", "order", "tiles", "values", "ranges"):
            assert np.array_equal(g1[k], g2[k]), k
        torch.cuda.synchronize()
    finally:
        Rf.close()


def test_plan_reports_the_pairs_of_the_render(orc, R, scenes):
    """fgs_plan runs only the first half: its pair count equals the FP32
    oracle's and the render's, and a render within its byte figure does not
    grow the context's scratch beyond it."""
    sc = scenes.make_scene("medium", P=200_000)
    cam = scenes.camera_for("medium", 1, W=1280, H=720)
    gsc = _gs(sc)
    o = opts()
    print("[parity] plan: medium P=200000 1280x720", flush=True)
    pl = R.plan(gsc, cam, 1280, 720, o)
    o32 = orc.render(sc, cam, 1280, 720, o, mode="f32")
    assert pl["pairs"] == o32["npairs"]
    out = R.render(gsc, cam, 1280, 720, o)
    assert out["stats"]["pairs"] == pl["pairs"]
    assert pl["bytes"] > 16 * pl["pairs"]


def test_large_rectangles_chunked(orc, R):
    """Gaussians whose rectangles span hundreds of tiles (chunked tile test
    and emission across workgroups)."""
    rng = np.random.default_rng(31)
    P = 400
    means = np.c_[rng.uniform(-2, 2, P), rng.uniform(-1.2, 1.2, P), rng.uniform(3, 12, P)]
    ls = rng.normal(-1.2, 0.6, (P, 3))
    sc = scene_from(means, ls, rng.normal(size=(P, 4)), rng.normal(-1, 1.5, P), sh=rng.normal(0, 0.3, (12, P)),
                    sh_degree=1)
    cam = identity_camera(1024, 768, 700.0)
    g, o32, _ = _full_check(orc, R, sc, cam, 1024, 768, opts(), "chunked")
    nt = (o32["ints"][:, orc.I_TX1] - o32["ints"][:, orc.I_TX0] + 1) * (o32["ints"][:, orc.I_TY1] - o32["ints"][:, orc.I_TY0] + 1)
    assert (nt[o32["ints"][:, 0] == 1] > 256).sum() > 20


def test_chunk_list_overflow_falls_back(orc, R):
    """More chunk entries than the list holds (600 screen-filling Gaussians at
    4K need about 76,000): the overflow Gaussians are counted in-wave and the
    result is unchanged."""
    rng = np.random.default_rng(32)
    P = 600
    means = np.c_[rng.uniform(-0.3, 0.3, P), rng.uniform(-0.2, 0.2, P), rng.uniform(5, 9, P)]
    sc = scene_from(means, np.full((P, 3), 1.2), rng.normal(size=(P, 4)), rng.normal(0, 1, P),
                    dc_rgb=rng.uniform(0, 1, (P, 3)))
    cam = identity_camera(3840, 2160, 1500.0)
    g, o32, _ = _full_check(orc, R, sc, cam, 3840, 2160, opts(), "overflow")
    assert o32["npairs"] > 65536 * 256
