"""ctypes wrapper around the CPU oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this
module.  It never touches the GPU path.

Modes: "f64" (plain definition, binary64, libm) and "f32" (canonical binary32
operation sequence, used for the bit-exact comparisons of per-Gaussian state,
pairs and sorted order).
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

S_U, S_V, S_A, S_B, S_C, S_K2, S_O, S_DEPTH, S_R, S_G, S_BL, S_COVA, S_COVB, S_COVC, S_HX, S_HY = range(16)
S_N = 16
I_VALID, I_COUNT, I_I0, I_I1, I_J0, I_J1, I_TX0, I_TX1, I_TY0, I_TY1 = range(10)
I_N = 10
TILE = 16


def _lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(HERE, "liboracle.so")
        if not os.path.exists(path):
            import importlib.util
            spec = importlib.util.spec_from_file_location("_orc_build", os.path.join(HERE, "build.py"))
            mod = importlib.util.module_from_spec(spec)
            spec.loader.exec_module(mod)
            mod.build()
        _LIB = C.CDLL(path)
    return _LIB


def _types(mode):
    R = C.c_double if mode == "f64" else C.c_float

    class Scene(C.Structure):
        _fields_ = [("P", C.c_int64), ("stride", C.c_int64), ("D", C.c_int32), ("pad_", C.c_int32),
                    ("means", C.c_void_p), ("log_scales", C.c_void_p), ("quats", C.c_void_p),
                    ("logits", C.c_void_p), ("sh", C.c_void_p)]

    class Camera(C.Structure):
        _fields_ = [("R", R * 9), ("t", R * 3), ("eye", R * 3), ("fx", R), ("fy", R), ("cx", R), ("cy", R),
                    ("near_z", R)]

    class Options(C.Structure):
        _fields_ = [("alpha_min", R), ("T_stop", R), ("alpha_max", R), ("dilation", R), ("jac_clip", R),
                    ("bg", R * 3), ("cap_3sigma", C.c_int32), ("binning", C.c_int32)]

    return Scene, Camera, Options


_TYPES = {m: _types(m) for m in ("f32", "f64")}


def _np(mode):
    return np.float64 if mode == "f64" else np.float32


def _f32(x):
    """Round a Python number to binary32 (the GPU receives binary32 inputs)."""
    return float(np.float32(x))


class Prepared:
    """Inputs marshalled for one oracle mode; keeps the arrays alive."""

    def __init__(self, scene, cam, W, H, opts, mode):
        self.mode = mode
        dt = _np(mode)
        Scene, Camera, Options = _TYPES[mode]
        self.arrays = [np.ascontiguousarray(a, dtype=dt) for a in scene.arrays()]
        P = self.arrays[0].shape[1]
        self.P = P
        self.sc = Scene(P, P, scene.sh_degree, 0, *(a.ctypes.data for a in self.arrays))
        c = Camera()
        # camera values are binary32 inputs; binary64 mode promotes them exactly
        for i in range(9):
            c.R[i] = _f32(cam.R.reshape(-1)[i])
        for i in range(3):
            c.t[i] = _f32(cam.t[i])
            c.eye[i] = _f32(cam.eye[i])
        c.fx, c.fy, c.cx, c.cy, c.near_z = (_f32(v) for v in (cam.fx, cam.fy, cam.cx, cam.cy, cam.near))
        self.cam = c
        o = Options()
        o.alpha_min = _f32(opts["alpha_min"])
        o.T_stop = _f32(opts["T_stop"])
        o.alpha_max = _f32(opts["alpha_max"])
        o.dilation = _f32(opts["dilation"])
        o.jac_clip = _f32(opts["jac_clip"])
        for i in range(3):
            o.bg[i] = _f32(opts["bg"][i])
        o.cap_3sigma = int(opts["cap_3sigma"])
        o.binning = int(opts["binning"])
        self.opts = o
        self.W, self.H = int(W), int(H)


def _fn(name, mode):
    return getattr(_lib(), f"{name}_{mode}")


def preprocess(prep):
    """Per-Gaussian state [P, 16] and ints [P, 10]; returns (state, ints, npairs)."""
    dt = _np(prep.mode)
    state = np.zeros((prep.P, S_N), dt)
    ints = np.zeros((prep.P, I_N), np.int32)
    f = _fn("orc_preprocess", prep.mode)
    f.restype = C.c_int64
    n = f(C.byref(prep.sc), C.byref(prep.cam), prep.W, prep.H, C.byref(prep.opts),
          state.ctypes.data_as(C.c_void_p), ints.ctypes.data_as(C.c_void_p))
    return state, ints, int(n)


def pairs(prep, state, ints, npairs):
    """Sorted (tile, value) pairs and per-tile ranges [ntiles, 2]."""
    tiles_x = (prep.W + TILE - 1) // TILE
    tiles_y = (prep.H + TILE - 1) // TILE
    tiles = np.zeros(max(npairs, 1), np.uint32)
    vals = np.zeros(max(npairs, 1), np.uint32)
    rng = np.zeros((tiles_x * tiles_y, 2), np.int64)
    f = _fn("orc_pairs", prep.mode)
    f.restype = None
    f(C.byref(prep.sc), prep.W, prep.H, C.byref(prep.opts), state.ctypes.data_as(C.c_void_p),
      ints.ctypes.data_as(C.c_void_p), C.c_int64(npairs), tiles.ctypes.data_as(C.c_void_p),
      vals.ctypes.data_as(C.c_void_p), rng.ctypes.data_as(C.c_void_p))
    return tiles[:npairs], vals[:npairs], rng


def blend_tiled(prep, state, vals, rng):
    dt = _np(prep.mode)
    H, W = prep.H, prep.W
    rgb = np.zeros((3, H, W), dt)
    T = np.zeros((H, W), dt)
    last = np.zeros((H, W), np.uint32)
    f = _fn("orc_blend_tiled", prep.mode)
    f.restype = None
    vals = np.ascontiguousarray(vals, np.uint32)
    if vals.size == 0:
        vals = np.zeros(1, np.uint32)
    f(state.ctypes.data_as(C.c_void_p), W, H, C.byref(prep.opts), vals.ctypes.data_as(C.c_void_p),
      np.ascontiguousarray(rng).ctypes.data_as(C.c_void_p), rgb.ctypes.data_as(C.c_void_p),
      T.ctypes.data_as(C.c_void_p), last.ctypes.data_as(C.c_void_p))
    return rgb, T, last


def blend_brute(prep, state, ints):
    dt = _np(prep.mode)
    H, W = prep.H, prep.W
    rgb = np.zeros((3, H, W), dt)
    T = np.zeros((H, W), dt)
    last = np.zeros((H, W), np.uint32)
    f = _fn("orc_blend_brute", prep.mode)
    f.restype = None
    f(state.ctypes.data_as(C.c_void_p), ints.ctypes.data_as(C.c_void_p), C.c_int64(prep.P), W, H,
      C.byref(prep.opts), rgb.ctypes.data_as(C.c_void_p), T.ctypes.data_as(C.c_void_p),
      last.ctypes.data_as(C.c_void_p))
    return rgb, T, last


def render(scene, cam, W, H, opts, mode="f64", brute=False):
    """Full oracle render.  Returns a dict with the image [3, H, W], T_final,
    last, per-Gaussian state/ints, and the sorted pairs."""
    prep = Prepared(scene, cam, W, H, opts, mode)
    state, ints, n = preprocess(prep)
    out = dict(state=state, ints=ints, npairs=n, prep=prep)
    if brute:
        rgb, T, last = blend_brute(prep, state, ints)
    else:
        tiles, vals, rng = pairs(prep, state, ints, n)
        out.update(tiles=tiles, vals=vals, ranges=rng)
        rgb, T, last = blend_tiled(prep, state, vals, rng)
    out.update(rgb=rgb, T=T, last=last)
    return out


def tile_hit(state_row, tx, ty, W, H, mode="f64"):
    dt = _np(mode)
    s = np.ascontiguousarray(state_row, dt)
    f = _fn("orc_tile_hit_api", mode)
    f.restype = C.c_int
    return bool(f(s.ctypes.data_as(C.c_void_p), int(tx), int(ty), int(W), int(H)))


def sh_basis(x, y, z, mode="f64"):
    dt = _np(mode)
    Y = np.zeros(16, dt)
    R = C.c_double if mode == "f64" else C.c_float
    f = _fn("orc_sh_eval", mode)
    f.restype = None
    f.argtypes = [R, R, R, C.c_void_p]
    f(x, y, z, Y.ctypes.data_as(C.c_void_p))
    return Y


def exp_d(x):
    f = _lib().orc_exp_d
    f.restype = C.c_double
    f.argtypes = [C.c_double]
    return f(x)


def log_d(x):
    f = _lib().orc_log_d
    f.restype = C.c_double
    f.argtypes = [C.c_double]
    return f(x)


def backward(out, dL_drgb):
    """Binary64 adjoint of a binary64 render (`out` from render(..., mode="f64")).

    dL_drgb: [3, H, W].  Returns gradients shaped like the scene's arrays
    (means [3, P], log_scales [3, P], quats [4, P], logits [1, P],
    sh [3 (D+1)^2, P]) and the per-Gaussian state gradient [P, 9]
    (u, v, A, B, C, o, r, g, b)."""
    prep = out["prep"]
    assert prep.mode == "f64", "the adjoint is defined on the binary64 render"
    P = prep.P
    nsh = prep.arrays[4].shape[0]
    g = dict(means=np.zeros((3, P)), log_scales=np.zeros((3, P)), quats=np.zeros((4, P)),
             logits=np.zeros((1, P)), sh=np.zeros((nsh, P)), state=np.zeros((P, 9)))
    dL = np.ascontiguousarray(dL_drgb, np.float64)
    assert dL.shape == (3, prep.H, prep.W)
    vals = np.ascontiguousarray(out["vals"], np.uint32)
    if vals.size == 0:
        vals = np.zeros(1, np.uint32)
    f = _lib().orc_backward_f64
    f.restype = None
    ptr = lambda a: a.ctypes.data_as(C.c_void_p)
    f(C.byref(prep.sc), C.byref(prep.cam), prep.W, prep.H, C.byref(prep.opts), ptr(out["state"]), ptr(out["ints"]),
      ptr(vals), ptr(np.ascontiguousarray(out["ranges"])), ptr(dL), ptr(g["means"]), ptr(g["log_scales"]),
      ptr(g["quats"]), ptr(g["logits"]), ptr(g["sh"]), ptr(g["state"]))
    return g
