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
from dataclasses import dataclass, field
import math

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


def _normal(rng, mu, sigma, n):
    return (rng.standard_normal(n, dtype=np.float32) * np.float32(sigma) + np.float32(mu)).astype(np.float32)


def _unit_quats(rng, n):
    q = np.empty((4, n), np.float32)
    for c in range(4):
        q[c] = rng.standard_normal(n, dtype=np.float32)
    nrm = np.sqrt((q.astype(np.float64) ** 2).sum(0))
    nrm[nrm == 0] = 1.0
    return (q / nrm).astype(np.float32)


def _sh(rng, degree, n, dc_sigma=0.5, rest_sigma=0.1):
    nk = (degree + 1) ** 2
    sh = np.empty((3 * nk, n), np.float32)
    for p in range(3 * nk):
        sh[p] = _normal(rng, 0.0, dc_sigma if p < 3 else rest_sigma, n)
    return sh


def make_scene(kind, seed=None, P=None):
    """Draw a scene.  Draw order: means, log-scales, quaternions, logits,
    SH DC, SH rest; every draw float32 from numpy's PCG64 default_rng."""
    if kind == "small":
        seed = 1 if seed is None else seed
        P = 10_000 if P is None else P
        rng = np.random.default_rng(seed)
        means = np.stack([rng.uniform(-1, 1, P).astype(np.float32) for _ in range(3)])
        ls = np.stack([_normal(rng, -3.5, 0.5, P) for _ in range(3)])
        degree = 0
    elif kind == "medium":
        seed = 2 if seed is None else seed
        P = 1_000_000 if P is None else P
        rng = np.random.default_rng(seed)
        means = np.stack([rng.uniform(-5, 5, P).astype(np.float32) for _ in range(3)])
        ls = np.stack([_normal(rng, -3.5, 0.5, P) for _ in range(3)])
        degree = 3
    elif kind in ("city", "serve"):
        seed = (3 if kind == "city" else 5) if seed is None else seed
        P = (10_000_000 if kind == "city" else 6_000_000) if P is None else P
        rng = np.random.default_rng(seed)
        x = rng.uniform(-500, 500, P).astype(np.float32)
        y = (rng.standard_exponential(P, dtype=np.float32) * np.float32(15.0)).astype(np.float32)
        z = rng.uniform(-500, 500, P).astype(np.float32)
        means = np.stack([x, y, z])
        ls = np.stack([_normal(rng, -1.0, 1.2, P) for _ in range(3)])
        degree = 3
    else:
        raise ValueError(f"unknown scene kind {kind!r}")
    quats = _unit_quats(rng, P)
    logits = _normal(rng, 0.0, 1.5, P)[None, :]
    sh = _sh(rng, degree, P)
    return Scene(np.ascontiguousarray(means), np.ascontiguousarray(ls), quats,
                 np.ascontiguousarray(logits), sh, degree)


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
    rng = np.random.default_rng(seed)
    m = scene.means + np.stack([_normal(rng, 0.0, sigma, scene.P) for _ in range(3)])
    return Scene(m.astype(np.float32), scene.log_scales, scene.quats, scene.logits, scene.sh, scene.sh_degree)


DEFAULT_OPTIONS = dict(alpha_min=1.0 / 255.0, T_stop=1e-4, alpha_max=0.99, dilation=0.3, jac_clip=1.3,
                       bg=(0.0, 0.0, 0.0), cap_3sigma=1, binning=0)
