"""Small hand-made scenes and cameras for the oracle's pin tests."""
import numpy as np

from paper_2408_07967_amd.scenes import Camera, Scene, DEFAULT_OPTIONS

Y00 = 0.28209479177387814  # 1 / (2 sqrt(pi))


def identity_camera(W, H, f, near=0.2):
    """Camera frame == world frame: x right, y down, z forward."""
    return Camera(np.eye(3, dtype=np.float32), np.zeros(3, np.float32), np.zeros(3, np.float32),
                  float(f), float(f), W / 2.0, H / 2.0, near, W, H)


def scene_from(means, log_scales, quats, logits, dc_rgb=None, sh_degree=0, sh=None, dtype=np.float32):
    means = np.asarray(means, np.float64).reshape(-1, 3).T
    P = means.shape[1]
    ls = np.broadcast_to(np.asarray(log_scales, np.float64).reshape(-1, 3).T, (3, P))
    q = np.broadcast_to(np.asarray(quats, np.float64).reshape(-1, 4).T, (4, P))
    lg = np.broadcast_to(np.asarray(logits, np.float64).reshape(1, -1), (1, P))
    if sh is None:
        nk = (sh_degree + 1) ** 2
        sh = np.zeros((3 * nk, P))
        if dc_rgb is not None:
            # colour c = Y00 * sh_dc + 0.5
            dc = (np.broadcast_to(np.asarray(dc_rgb, np.float64).reshape(-1, 3), (P, 3)) - 0.5) / Y00
            sh[0:3] = dc.T
    return Scene(*(np.ascontiguousarray(a, dtype=dtype) for a in (means, ls, q, lg, sh)), sh_degree)


def opts(**kw):
    o = dict(DEFAULT_OPTIONS)
    o.update(kw)
    return o


def logit(o):
    return float(np.log(o / (1.0 - o)))


def random_scene(rng, P, box=1.0, ls_mu=-3.0, ls_sigma=0.6, sh_degree=1, z0=4.0, dtype=np.float32):
    means = rng.uniform(-box, box, (P, 3))
    means[:, 2] += z0
    ls = rng.normal(ls_mu, ls_sigma, (P, 3))
    q = rng.normal(size=(P, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    lg = rng.normal(0, 1.5, P)
    nk = (sh_degree + 1) ** 2
    sh = rng.normal(0, 0.3, (3 * nk, P))
    sh[:3] = rng.normal(0, 0.5, (3, P))
    return scene_from(means, ls, q, lg, sh=sh, sh_degree=sh_degree, dtype=dtype)
