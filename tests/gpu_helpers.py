"""Shared helpers for the GPU parity tests: run the HIP path through the C ABI
and compare it with the CPU oracle on the same seeded inputs."""
import numpy as np

from paper_2408_07967_amd import binding as B

# image tolerance (per channel): |diff| <= 2e-3 on >= 99.9 % of pixels and
# mean |diff| <= 1e-5 against the binary64 oracle
IMG_MAX = 2e-3
IMG_FRAC = 0.999
IMG_MEAN = 1e-5


def gpu_frame(R, gscene, cam, W, H, opts, prepared=None):
    """Render on the GPU (from the raw parameters, or from a prepared scene)
    and download the saved frame's fields."""
    import torch
    out = R.render(gscene, cam, W, H, opts, want_T=True, want_last=True, save=True, prepared=prepared)
    torch.cuda.synchronize()
    fr = out["frame"]
    P = gscene.P
    res = dict(rgb=out["rgb"].cpu().numpy(), T=out["T"].cpu().numpy(),
               last=out["last"].cpu().numpy().view(np.uint32), stats=out["stats"])
    res["gauss"] = R.frame_field(fr, B.FIELD_GAUSS).view(np.float32).reshape(P, 16) if P else np.zeros((0, 16))
    res["rect"] = R.frame_field(fr, B.FIELD_RECT).reshape(P, 4) if P else np.zeros((0, 4), np.uint32)
    res["count"] = R.frame_field(fr, B.FIELD_COUNT)
    res["order"] = R.frame_field(fr, B.FIELD_ORDER)
    res["tiles"] = R.frame_field(fr, B.FIELD_TILES)
    res["values"] = R.frame_field(fr, B.FIELD_VALUES)
    res["ranges"] = R.frame_field(fr, B.FIELD_RANGES).reshape(-1, 2)
    R.release(fr)
    return res


def check_gauss_state(orc, g, o32):
    """Per-Gaussian state of the GPU vs the FP32 oracle: bit-exact for every
    quantity that decides pairs or order; colour and opacity to 1e-5."""
    st, iv = o32["state"], o32["ints"]
    valid = iv[:, orc.I_VALID] == 1
    vidx = np.nonzero(valid)[0]
    # visible set and depth order: (depth bits, index) ascending
    dbits = st[:, orc.S_DEPTH].astype(np.float32).view(np.uint32)
    expect_order = vidx[np.lexsort((vidx, dbits[vidx]))]
    assert np.array_equal(g["order"], expect_order.astype(np.uint32)), "visible set / depth order differs"
    gg = g["gauss"][vidx]
    for col, s in ((0, orc.S_U), (1, orc.S_V), (2, orc.S_A), (3, orc.S_B), (4, orc.S_C), (5, orc.S_K2),
                   (10, orc.S_DEPTH)):
        a = gg[:, col].view(np.uint32)
        b = st[vidx, s].astype(np.float32).view(np.uint32)
        bad = np.nonzero(a != b)[0]
        assert bad.size == 0, f"state column {col}: {bad.size} mismatches, first g={vidx[bad[:5]]}"
    rect = g["rect"][vidx].astype(np.int64)
    assert np.array_equal(rect[:, 0], iv[vidx, orc.I_TX0]) and np.array_equal(rect[:, 1], iv[vidx, orc.I_TX1])
    assert np.array_equal(rect[:, 2], iv[vidx, orc.I_TY0]) and np.array_equal(rect[:, 3], iv[vidx, orc.I_TY1])
    assert np.array_equal(g["count"].astype(np.int64), np.where(valid, iv[:, orc.I_COUNT], 0))
    np.testing.assert_allclose(gg[:, 11], st[vidx, orc.S_O], rtol=1e-6)
    for col, s in ((7, orc.S_R), (8, orc.S_G), (9, orc.S_BL)):
        np.testing.assert_allclose(gg[:, col], st[vidx, s], rtol=1e-4, atol=1e-5)


def check_pairs(g, o32):
    """Sorted pair list and tile ranges: bit-exact vs the FP32 oracle."""
    n = o32["npairs"]
    assert g["stats"]["pairs"] == n, (g["stats"]["pairs"], n)
    assert np.array_equal(g["tiles"], o32["tiles"]), "sorted tile ids differ"
    assert np.array_equal(g["values"], o32["vals"]), "sorted Gaussian ids differ"
    gr = g["ranges"].astype(np.int64)
    orr = o32["ranges"]
    empty = orr[:, 0] == orr[:, 1]
    assert np.all(gr[empty, 0] == gr[empty, 1]), "an empty tile has a non-empty range"
    assert np.array_equal(gr[~empty], orr[~empty]), "tile ranges differ"


def image_error(a, b):
    d = np.abs(a.astype(np.float64) - b.astype(np.float64))
    return d.max(), (d <= IMG_MAX).mean(), d.mean()


# columns of the downloaded per-Gaussian record (fgs.h, FGS_FIELD_GAUSS)
COL_A, COL_B, COL_C, COL_AB, COL_BB, COL_CB = 2, 3, 4, 12, 13, 14
# the blend's conic is the binary64 conic rounded once: against the binary64
# oracle's conic, relative to the larger diagonal entry
BLEND_CONIC_REL = 1e-4


def check_blend_conic(g, o64, tag=""):
    """The conic the blend evaluates pixels with against the binary64 oracle's
    (the binary32 canonical conic, which decides the pairs, may be several
    per cent off for long thin footprints)."""
    st = o64["state"]
    vis = np.zeros(st.shape[0], bool)
    vis[g["order"]] = True  # the GPU's visible set
    vidx = np.nonzero((o64["ints"][:, 0] == 1) & vis)[0]
    if vidx.size == 0:
        return
    gg = g["gauss"][vidx].astype(np.float64)
    ref = st[vidx][:, [2, 3, 4]]
    got = gg[:, [COL_AB, COL_BB, COL_CB]]
    scale = np.maximum(np.abs(ref[:, 0]), np.abs(ref[:, 2]))
    rel = np.abs(got - ref).max(axis=1) / scale
    assert rel.max() <= BLEND_CONIC_REL, f"{tag} blend conic: max relative error {rel.max():.3g}"


def check_image(g, o64, tag=""):
    if "gauss" in g:  # a saved frame's state (batched frames keep none)
        check_blend_conic(g, o64, tag)
    mx, frac, mean = image_error(g["rgb"], o64["rgb"])
    assert frac >= IMG_FRAC and mean <= IMG_MEAN, f"{tag} image: max {mx:.3g} frac {frac:.6f} mean {mean:.3g}"
    mx, frac, mean = image_error(g["T"], o64["T"])
    assert frac >= IMG_FRAC and mean <= IMG_MEAN, f"{tag} T_final: max {mx:.3g} frac {frac:.6f} mean {mean:.3g}"
    agree = (g["last"] == o64["last"]).mean()
    assert agree >= 0.995, f"{tag} last-contributor agreement {agree:.5f}"
