"""Pins of the oracle's binary64 adjoint against central finite differences of
the oracle's binary64 forward render (CPU only).

The adjoint (oracle/orc_grad.c) and the forward (oracle/orc_core.c) are
separate code: the forward composites front to back and never forms a
derivative; the adjoint uses the back-to-front "over" recursion and the chain
rule through every preprocessing step.  A dropped term, a wrong sign or a
transposed factor anywhere in the adjoint moves some parameter's gradient far
outside the tolerance below.

Finite differences are only meaningful where the discrete structure of the
image (contributors, clamps, stopping points) does not change within the
step.  A parameter is used when the central differences at h and h/2 agree
(Richardson check); the test requires that almost all parameters pass it.
"""
import numpy as np
import pytest

from oracle import oracle as orc
from oracle_helpers import identity_camera, logit, opts, scene_from

from paper_2408_07967_amd.scenes import Scene

W = H = 32
F = 27.712812921102035  # (H/2) / tan(30 deg)
GROUPS = ("means", "log_scales", "quats", "logits", "sh")


def feature_scene(seed):
    """Random Gaussians (SH degree 3) plus the cases whose derivative rules
    differ: opaque Gaussians centred on a pixel sample (alpha clamped at 0.99,
    and a stack of them makes pixels stop early), a Gaussian whose red channel
    is clamped at 0, and a wide Gaussian whose centre lies beyond the Jacobian
    clamp but still covers the right edge of the image."""
    rng = np.random.default_rng(seed)
    n_rand = 22
    means = np.concatenate([rng.uniform(-0.6, 0.6, (n_rand, 2)), rng.uniform(3.5, 4.5, (n_rand, 1))], axis=1)
    ls = rng.normal(-2.2, 0.4, (n_rand, 3))
    q = rng.normal(size=(n_rand, 4))
    lg = rng.normal(0.5, 1.5, n_rand)
    # pixel sample (16.5, 12.5) and (16.5, 20.5) at depth 4: x = (u - 16) z / f
    opaque = []
    for k, (u, v) in enumerate([(16.5, 12.5), (16.5, 12.5), (16.5, 12.5), (16.5, 20.5)]):
        z = 3.0 + 0.1 * k
        opaque.append([(u - 16.0) * z / F, (v - 16.0) * z / F, z])
    means = np.concatenate([means, np.array(opaque)], axis=0)
    ls = np.concatenate([ls, np.full((4, 3), -1.9) + rng.normal(0, 0.05, (4, 3))], axis=0)
    q = np.concatenate([q, rng.normal(size=(4, 4))], axis=0)
    lg = np.concatenate([lg, [6.0, 5.5, 7.0, 6.5]])
    # clamped red channel
    means = np.concatenate([means, [[0.3, -0.2, 3.8]]], axis=0)
    ls = np.concatenate([ls, [[-1.8, -2.0, -1.9]]], axis=0)
    q = np.concatenate([q, [[1.0, 0.2, -0.1, 0.3]]], axis=0)
    lg = np.concatenate([lg, [1.0]])
    # beyond the Jacobian clamp: x~ = 1.0 > 1.3 * 16 / F = 0.75, footprint reaching x < 32 px
    means = np.concatenate([means, [[4.0, 0.3, 4.0]]], axis=0)
    ls = np.concatenate([ls, [[-0.6, -0.8, -0.7]]], axis=0)
    q = np.concatenate([q, [[0.9, 0.1, 0.3, -0.2]]], axis=0)
    lg = np.concatenate([lg, [0.5]])
    P = means.shape[0]
    sh = rng.normal(0, 0.1, (48, P))
    sh[0:3] = rng.normal(0, 0.5, (3, P))
    sh[0, n_rand + 4] = -3.0  # red: Y00 * (-3) + 0.5 < 0
    return scene_from(means, ls, q, lg, sh=sh, sh_degree=3, dtype=np.float64), n_rand


def render(sc, o, cam):
    return orc.render(sc, cam, W, H, o, "f64")


def check_features(sc, n_rand, o, cam):
    out = render(sc, o, cam)
    st, iv = out["state"], out["ints"]
    # alpha clamp: an opaque Gaussian centred on a pixel sample with o > 0.99
    assert iv[n_rand, 0] and st[n_rand, orc.S_O] > 0.99
    # early termination changes the image
    nostop = render(sc, dict(o, T_stop=0.0), cam)
    assert np.abs(nostop["rgb"] - out["rgb"]).max() > 1e-6
    # colour clamp
    g = n_rand + 4
    assert iv[g, 0] and st[g, orc.S_R] == 0.0
    # Jacobian clamp on a visible Gaussian
    g = n_rand + 5
    assert iv[g, 0] and sc.means[0, g] / sc.means[2, g] > 1.3 * (W / 2) / F
    return out


def fd_check(sc, o, cam, seed):
    rng = np.random.default_rng(seed)
    w = rng.uniform(-1.0, 1.0, (3, H, W))  # L = sum(w * rgb): smooth in the image

    def loss(s):
        return float((w * render(s, o, cam)["rgb"]).sum())

    out = render(sc, o, cam)
    g = orc.backward(out, w)
    arrays = [a.copy() for a in sc.arrays()]
    used = total = 0
    for gi, name in enumerate(GROUPS):
        errs, fds = [], []
        for r in range(arrays[gi].shape[0]):
            for c in range(sc.P):
                def cd(h):
                    a = [x.copy() for x in arrays]
                    a[gi][r, c] += h
                    lp = loss(Scene(*a, sc.sh_degree))
                    a[gi][r, c] -= 2 * h
                    lm = loss(Scene(*a, sc.sh_degree))
                    return (lp - lm) / (2 * h)
                f1, f2 = cd(1e-6), cd(5e-7)
                total += 1
                if abs(f1 - f2) > 1e-6 * abs(f1) + 1e-8:
                    continue  # the structure changes within the step
                used += 1
                errs.append(abs(g[name][r, c] - f1))
                fds.append(f1)
        errs, fds = np.array(errs), np.array(fds)
        rms = float(np.sqrt((fds ** 2).mean()))
        assert rms > 0, name
        bound = 1e-5 * np.maximum(np.abs(fds), rms)
        bad = np.nonzero(errs > bound)[0]
        assert bad.size == 0, (name, errs[bad][:5], fds[bad][:5])
    assert used >= 0.97 * total, (used, total)


@pytest.mark.parametrize("bg", [(0.0, 0.0, 0.0), (0.2, 0.7, 0.4)])
def test_adjoint_matches_central_differences(bg):
    sc, n_rand = feature_scene(3)
    cam = identity_camera(W, H, F)
    o = opts(bg=list(bg))
    check_features(sc, n_rand, o, cam)
    fd_check(sc, o, cam, seed=17)


def test_adjoint_uncapped_extent_and_box_binning():
    """The gradient does not depend on how pairs were binned, and holds with
    the uncapped extent (k^2 = 2 ln(o / tau))."""
    sc, _ = feature_scene(4)
    cam = identity_camera(W, H, F)
    w = np.random.default_rng(2).uniform(-1, 1, (3, H, W))
    g_exact = orc.backward(render(sc, opts(), cam), w)
    g_box = orc.backward(render(sc, opts(binning=1), cam), w)
    for name in GROUPS:
        np.testing.assert_array_equal(g_exact[name], g_box[name])
    fd_check(sc, opts(cap_3sigma=0), cam, seed=5)


def test_adjoint_of_culled_gaussians_is_zero():
    cam = identity_camera(W, H, F)
    sc = scene_from([[0, 0, 4.0], [0, 0, 0.1], [0.1, 0, 4.0]], [[-2, -2, -2]] * 3, [[1, 0, 0, 0]] * 3,
                    [1.0, 1.0, logit(1.0 / 255 * 0.5)], dc_rgb=[0.6, 0.4, 0.2], dtype=np.float64)
    out = render(sc, opts(), cam)
    g = orc.backward(out, np.ones((3, H, W)))
    assert out["ints"][:, 0].tolist() == [1, 0, 0]
    for name in GROUPS:
        assert np.all(g[name][:, 1:] == 0.0)
        assert np.any(g[name][:, 0] != 0.0) or name == "quats"


def test_opacity_gradient_closed_form():
    """One isotropic Gaussian, head-on: C = c a at every contributing pixel with
    a = o exp(-q/2) unclamped, so dL/dlogit = sum_p w_p c exp(-q_p/2) o (1 - o)
    over the contributing pixels (closed form, independent of the adjoint's
    recursion)."""
    cam = identity_camera(W, H, F)
    o_ = 0.6
    sc = scene_from([[0.01, -0.02, 4.0]], [[-1.5, -1.5, -1.5]], [[1, 0, 0, 0]], [logit(o_)],
                    dc_rgb=[0.7, 0.3, 0.5], dtype=np.float64)
    out = render(sc, opts(), cam)
    st = out["state"][0]
    w = np.random.default_rng(1).uniform(-1, 1, (3, H, W))
    g = orc.backward(out, w)
    jj, ii = np.mgrid[0:H, 0:W]
    dx, dy = ii + 0.5 - st[orc.S_U], jj + 0.5 - st[orc.S_V]
    q = st[orc.S_A] * dx * dx + 2 * st[orc.S_B] * dx * dy + st[orc.S_C] * dy * dy
    inside = q <= st[orc.S_K2]
    G = np.exp(-0.5 * q) * inside
    col = st[orc.S_R:orc.S_BL + 1]
    expect = sum((w[ch] * col[ch] * G).sum() for ch in range(3)) * o_ * (1 - o_)
    assert g["logits"][0, 0] == pytest.approx(expect, rel=1e-12)
