"""Host-side checks of the C-ABI library: it loads, exports every entry point
declared in include/fgs.h, and rejects bad arguments before any HIP call."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

from paper_2408_07967_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "fgs.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fgs_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = B.lib()
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
        assert n in B.PROTOTYPES, f"{n} has no binding prototype"


def test_default_options():
    o = B.default_options()
    assert o.alpha_min == pytest.approx(1 / 255) and o.T_stop == pytest.approx(1e-4)
    assert o.alpha_max == pytest.approx(0.99) and o.dilation == pytest.approx(0.3)
    assert o.jac_clip == pytest.approx(1.3) and o.cap_3sigma == 1 and o.binning == 0
    assert list(o.bg) == [0.0, 0.0, 0.0]


def _good():
    P = 10
    sc = B.make_scene(P, P, 0, 1, 2, 3, 4, 5)  # non-null fake pointers: never dereferenced
    cam = B.make_camera(np.eye(3), [0, 0, 0], [0, 0, 0], 100, 100, 32, 32)
    return sc, cam, B.default_options()


def _validate(sc, cam, W, H, op):
    return B.lib().fgs_validate(C.byref(sc) if sc is not None else None,
                                C.byref(cam) if cam is not None else None, W, H,
                                C.byref(op) if op is not None else None)


def test_validate_accepts_good_arguments():
    sc, cam, op = _good()
    assert _validate(sc, cam, 64, 64, op) == B.FGS_OK
    assert _validate(sc, cam, 64, 64, None) == B.FGS_OK
    empty = B.make_scene(0, 0, 0, None, None, None, None, None)
    assert _validate(empty, cam, 1, 1, op) == B.FGS_OK


@pytest.mark.parametrize("mutate, W, H", [
    (lambda sc, cam, op: setattr(sc, "num_gaussians", -1), 64, 64),
    (lambda sc, cam, op: setattr(sc, "plane_stride", 5), 64, 64),
    (lambda sc, cam, op: setattr(sc, "sh_degree", 4), 64, 64),
    (lambda sc, cam, op: setattr(sc, "sh_degree", -1), 64, 64),
    (lambda sc, cam, op: setattr(sc, "means", None), 64, 64),
    (lambda sc, cam, op: setattr(sc, "reserved", 7), 64, 64),
    (lambda sc, cam, op: None, 0, 64),
    (lambda sc, cam, op: None, 64, 16385),
    (lambda sc, cam, op: setattr(cam, "fx", 0.0), 64, 64),
    (lambda sc, cam, op: setattr(cam, "near_z", 0.0), 64, 64),
    (lambda sc, cam, op: cam.R.__setitem__(4, math.nan), 64, 64),
    (lambda sc, cam, op: cam.t.__setitem__(0, math.inf), 64, 64),
    (lambda sc, cam, op: setattr(op, "alpha_min", 0.0), 64, 64),
    (lambda sc, cam, op: setattr(op, "alpha_max", 1.0), 64, 64),
    (lambda sc, cam, op: setattr(op, "T_stop", -1.0), 64, 64),
    (lambda sc, cam, op: setattr(op, "binning", 3), 64, 64),
    (lambda sc, cam, op: op.bg.__setitem__(1, math.nan), 64, 64),
])
def test_validate_rejects(mutate, W, H):
    sc, cam, op = _good()
    mutate(sc, cam, op)
    assert _validate(sc, cam, W, H, op) == B.FGS_ERR_INVALID_ARGUMENT
    assert len(B.lib().fgs_last_error(None)) > 0


def test_null_arguments_rejected_without_device():
    sc, cam, op = _good()
    assert _validate(None, cam, 8, 8, op) == B.FGS_ERR_INVALID_ARGUMENT
    assert _validate(sc, None, 8, 8, op) == B.FGS_ERR_INVALID_ARGUMENT
    # render with a NULL context is rejected on the host
    st = B.lib().fgs_render(None, C.byref(sc), C.byref(cam), 8, 8, C.byref(op), 1, None, None, None, None, None)
    assert st == B.FGS_ERR_INVALID_ARGUMENT
    n = C.c_int64(5)
    assert B.lib().fgs_plan(None, C.byref(sc), C.byref(cam), 8, 8, C.byref(op), C.byref(n), None, None) == \
        B.FGS_ERR_INVALID_ARGUMENT
    assert n.value == 0
    g = B.FgsSceneGrad(0, None, None, None, None, None)
    st = B.lib().fgs_render_backward(None, None, C.byref(sc), C.byref(cam), C.byref(op), None, C.byref(g), None)
    assert st == B.FGS_ERR_INVALID_ARGUMENT
    cfg = B.FgsServerConfig(1 << 30, 4, 64, 64, 2, 1, 0)
    h = C.c_void_p()
    assert B.lib().fgs_server_create(0, C.byref(sc), C.byref(op), None, C.byref(h)) == B.FGS_ERR_INVALID_ARGUMENT
    bad = B.FgsServerConfig(1 << 30, 0, 64, 64, 2, 1, 0)  # no slots
    assert B.lib().fgs_server_create(0, C.byref(sc), C.byref(op), C.byref(bad), C.byref(h)) == \
        B.FGS_ERR_INVALID_ARGUMENT
    bad = B.FgsServerConfig(1 << 30, 4, 64, 64, 2, 1, -1)  # negative sharing threshold
    assert B.lib().fgs_server_create(0, C.byref(sc), C.byref(op), C.byref(bad), C.byref(h)) == \
        B.FGS_ERR_INVALID_ARGUMENT
    assert B.lib().fgs_server_create(0, None, C.byref(op), C.byref(cfg), C.byref(h)) == B.FGS_ERR_INVALID_ARGUMENT
    assert not h.value
    assert B.lib().fgs_server_submit(None, 1, C.byref(cam), 8, 8, 0, None) == B.FGS_ERR_INVALID_ARGUMENT
    assert B.lib().fgs_server_poll(None, None, 0, 0) < 0
    assert B.lib().fgs_server_release(None, 1) == B.FGS_ERR_INVALID_ARGUMENT
    B.lib().fgs_server_destroy(None)
    assert B.lib().fgs_clock_ns() > 0
    assert B.lib().fgs_frame_release(None, None) == B.FGS_OK
    assert B.lib().fgs_frame_field_bytes(None, 0) == 0
    assert B.lib().fgs_scratch_bytes(None) == 0
    assert B.lib().fgs_set_blend_variant(None, B.BLEND_PREFETCH) == B.FGS_ERR_INVALID_ARGUMENT
    cams = (B.FgsCamera * 2)(cam, cam)
    assert B.lib().fgs_render_prepared_batch(None, None, cams, 2, 8, 8, C.byref(op), None, None, None, None,
                                             None) == B.FGS_ERR_INVALID_ARGUMENT


def test_status_strings():
    for s in range(7):
        assert len(B.lib().fgs_status_string(s)) > 0


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert B.lib().fgs_create(0, C.byref(h)) == B.FGS_ERR_DEVICE
    assert not h.value
