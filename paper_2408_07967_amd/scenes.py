"""Seeded synthetic scenes and cameras (input generation only).

This module draws the inputs that both the GPU path and the CPU oracle
consume.  It holds none of the rasterizer's arithmetic: it only samples
Gaussian parameters and builds pinhole cameras.

Scene layout (planar, float32, numpy): every attribute is an array of shape
[planes, P] so plane c of Gaussian g is attr[c, g]:
  means [3, P] (world x, y, z), log_scales [3, P], quats [4, P] (w, x, y, z,
  unit norm), logits [1, P] (opacity = sigmoid(logit)), sh [3 (D+1)^2, P]
  (plane 3 k + channel, k = l^2 + l + m).

Camera: R (3x3, world -> camera, rows = camera right, down, forward axes),
t (x_cam = R x + t), eye (camera centre), fx, fy, cx, cy (pixels), near.

Workloads (the paper measures trained MatrixCity / Mill19 / Tanks&Temples /
Deep Blending scenes, which are not available; these synthetic scenes stand
in for them, the 10M-Gaussian ground-plane scene playing the large-scale
aerial 4K case):
  small   - 10,000 Gaussians in [-1, 1]^3, SH degree 0, 256x256, fov 60.
  medium  - 1,000,000 Gaussians in [-5, 5]^3, SH degree 3, 1920x1080,
            8 cameras on a radius-10 orbit.
  city    - 10,000,000 Gaussians over a 1000 m x 1000 m ground plane,
            heights exponential (mean 15 m), log-scales N(-1, 1.2), SH
            degree 3; camera at 80 m altitude pitched 30 deg down, fov 70,
            3840x2160 (and 7680x4320).
  serve   - 6,000,000 Gaussians with the city distributions; request poses on
            a 200 m orbit at 50-150 m altitude.
"""
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass
import math
import os

import numpy as np


@dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    logits: np.ndarray
    sh: np.ndarray
    sh_degree: int

    @property
    def P(self):
        return int(self.means.shape[1])

    def subset(self, idx):
        idx = np.asarray(idx)
        return Scene(*(np.ascontiguousarray(a[:, idx]) for a in
                       (self.means, self.log_scales, self.quats, self.logits, self.sh)),
                     self.sh_degree)

    def astype(self, dtype):
        return Scene(*(np.ascontiguousarray(a, dtype=dtype) for a in
                       (self.means, self.log_scales, self.quats, self.logits, self.sh)),
                     self.sh_degree)

    def arrays(self):
        return (self.means, self.log_scales, self.quats, self.logits, self.sh)


@dataclass
class Camera:
    R: np.ndarray          # [3, 3] float32
    t: np.ndarray          # [3]
    eye: np.ndarray        # [3]
    fx: float
    fy: float
    cx: float
    cy: float
    near: float = 0.2
    W: int = 0
    H: int = 0


def _plane_rngs(seed, n):
    """Independent PCG64 streams, one per plane (SeedSequence.spawn), so that
    planes can be drawn in parallel threads with a fixed result."""
    return [np.random.Generator(np.random.PCG64(c)) for c in np.random.SeedSequence(seed).spawn(n)]


def _draw(jobs, P):
    """jobs: list of (rng, kind, a, b); kind in normal/uniform/exponential.
    Returns a [len(jobs), P] float32 array."""
    out = np.empty((len(jobs), P), np.float32)

    def one(i):
        rng, kind, a, b = jobs[i]
        if kind == "normal":
            x = rng.standard_normal(P, dtype=np.float32)
            x *= np.float32(b)
            x += np.float32(a)
        elif kind == "uniform":
            x = rng.random(P, dtype=np.float32)
            x *= np.float32(b - a)
            x += np.float32(a)
        else:  # exponential with mean a
            x = rng.standard_exponential(P, dtype=np.float32)
            x *= np.float32(a)
        out[i] = x

    workers = min(16, os.cpu_count() or 1, len(jobs))
    if P * len(jobs) < 2_000_000 or workers <= 1:
        for i in range(len(jobs)):
            one(i)
    else:
        with ThreadPoolExecutor(max_workers=workers) as ex:
            list(ex.map(one, range(len(jobs))))
    return out


def make_scene(kind, seed=None, P=None):
    """Draw a scene.  Each plane has its own PCG64 stream spawned from the
    seed, in the order: means (3), log-scales (3), quaternion components (4,
    N(0, 1) then normalised), opacity logits (1), SH DC (3), SH rest."""
    if kind == "small":
        seed, P, degree = (1 if seed is None else seed), (10_000 if P is None else P), 0
        mean_jobs = [("uniform", -1.0, 1.0)] * 3
        ls_mu, ls_sigma = -3.5, 0.5
    elif kind == "medium":
        seed, P, degree = (2 if seed is None else seed), (1_000_000 if P is None else P), 3
        mean_jobs = [("uniform", -5.0, 5.0)] * 3
        ls_mu, ls_sigma = -3.5, 0.5
    elif kind in ("city", "serve"):
        seed = (3 if kind == "city" else 5) if seed is None else seed
        P = (10_000_000 if kind == "city" else 6_000_000) if P is None else P
        degree = 3
        mean_jobs = [("uniform", -500.0, 500.0), ("exponential", 15.0, 0.0), ("uniform", -500.0, 500.0)]
        ls_mu, ls_sigma = -1.0, 1.2
    else:
        raise ValueError(f"unknown scene kind {kind!r}")
    nk = (degree + 1) ** 2
    specs = (mean_jobs + [("normal", ls_mu, ls_sigma)] * 3 + [("normal", 0.0, 1.0)] * 4 +
             [("normal", 0.0, 1.5)] + [("normal", 0.0, 0.5)] * 3 + [("normal", 0.0, 0.1)] * (3 * nk - 3))
    rngs = _plane_rngs(seed, len(specs))
    planes = _draw([(r, *sp) for r, sp in zip(rngs, specs)], P)
    means, ls, q, logits, sh = planes[0:3], planes[3:6], planes[6:10], planes[10:11], planes[11:]
    nrm = np.sqrt((q.astype(np.float64) ** 2).sum(0))
    nrm[nrm == 0] = 1.0
    quats = (q / nrm).astype(np.float32)
    return Scene(np.ascontiguousarray(means), np.ascontiguousarray(ls), quats, np.ascontiguousarray(logits),
                 np.ascontiguousarray(sh), degree)


def look_at(eye, target, W, H, fov_deg, up=(0.0, 1.0, 0.0), near=0.2):
    """Pinhole camera at eye looking at target; vertical field of view
    fov_deg; camera axes x right, y down, z forward; world up +y."""
    eye = np.asarray(eye, np.float64)
    f = np.asarray(target, np.float64) - eye
    f /= np.linalg.norm(f)
    upv = np.asarray(up, np.float64)
    d = -upv + np.dot(upv, f) * f
    d /= np.linalg.norm(d)
    r = np.cross(d, f)
    R = np.stack([r, d, f])
    t = -R @ eye
    focal = (H / 2.0) / math.tan(math.radians(fov_deg) / 2.0)
    return Camera(R.astype(np.float32), t.astype(np.float32), eye.astype(np.float32),
                  float(np.float32(focal)), float(np.float32(focal)),
                  float(W) / 2.0, float(H) / 2.0, near, W, H)


def camera_for(kind, index=0, W=None, H=None):
    if kind == "small":
        return look_at((0.0, 0.0, -4.0), (0.0, 0.0, 0.0), W or 256, H or 256, 60.0)
    if kind == "medium":
        th = 2.0 * math.pi * index / 8.0
        return look_at((10.0 * math.sin(th), 0.0, -10.0 * math.cos(th)), (0.0, 0.0, 0.0),
                       W or 1920, H or 1080, 60.0)
    if kind == "city":
        pitch = math.radians(-30.0)
        eye = np.array([0.0, 80.0, 0.0])
        fwd = np.array([0.0, math.sin(pitch), math.cos(pitch)])
        return look_at(eye, eye + fwd, W or 3840, H or 2160, 70.0)
    raise ValueError(kind)


def serve_pose(rng):
    """One serving request: pose on a 200 m orbit, altitude U[50, 150] m,
    looking at the origin, fov 70, resolution uniform over four sizes."""
    th = rng.uniform(0.0, 2.0 * math.pi)
    h = rng.uniform(50.0, 150.0)
    W, H = [(1280, 720), (1920, 1080), (2560, 1440), (3840, 2160)][int(rng.integers(0, 4))]
    return look_at((200.0 * math.cos(th), h, 200.0 * math.sin(th)), (0.0, 0.0, 0.0), W, H, 70.0)


def perturb_means(scene, seed=4, sigma=0.01):
    """Target scene for the differentiation workload: means + N(0, sigma)."""
    m = scene.means + _draw([(r, "normal", 0.0, sigma) for r in _plane_rngs(seed, 3)], scene.P)
    return Scene(m.astype(np.float32), scene.log_scales, scene.quats, scene.logits, scene.sh, scene.sh_degree)


DEFAULT_OPTIONS = dict(alpha_min=1.0 / 255.0, T_stop=1e-4, alpha_max=0.99, dilation=0.3, jac_clip=1.3,
                       bg=(0.0, 0.0, 0.0), cap_3sigma=1, binning=0)
