"""ctypes binding of the C ABI in include/fgs.h (argument marshalling only).

Every stage of the rasterizer runs in the HIP kernels of libfgs.so; this
module only mirrors the ABI's structs and function prototypes.  There is no
CPU fallback: if the library is missing, loading fails with an error.
"""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfgs.so")

FGS_OK = 0
FGS_ERR_INVALID_ARGUMENT = 1
FGS_ERR_OUT_OF_MEMORY = 2
FGS_ERR_CAPACITY = 3
FGS_ERR_DEVICE = 4
FGS_ERR_NOT_SUPPORTED = 5
FGS_ERR_INTERNAL = 6

FIELD_GAUSS, FIELD_RECT, FIELD_COUNT, FIELD_ORDER, FIELD_TILES, FIELD_VALUES, FIELD_RANGES = range(7)


class FgsScene(C.Structure):
    _fields_ = [("num_gaussians", C.c_int64), ("plane_stride", C.c_int64), ("sh_degree", C.c_int32),
                ("reserved", C.c_int32), ("means", C.c_void_p), ("log_scales", C.c_void_p),
                ("quats", C.c_void_p), ("opacity_logits", C.c_void_p), ("sh", C.c_void_p)]


class FgsSceneGrad(C.Structure):
    _fields_ = [("plane_stride", C.c_int64), ("means", C.c_void_p), ("log_scales", C.c_void_p),
                ("quats", C.c_void_p), ("opacity_logits", C.c_void_p), ("sh", C.c_void_p)]


class FgsCamera(C.Structure):
    _fields_ = [("R", C.c_float * 9), ("t", C.c_float * 3), ("eye", C.c_float * 3), ("fx", C.c_float),
                ("fy", C.c_float), ("cx", C.c_float), ("cy", C.c_float), ("near_z", C.c_float)]


class FgsOptions(C.Structure):
    _fields_ = [("alpha_min", C.c_float), ("T_stop", C.c_float), ("alpha_max", C.c_float),
                ("dilation", C.c_float), ("jac_clip", C.c_float), ("bg", C.c_float * 3),
                ("cap_3sigma", C.c_int32), ("binning", C.c_int32)]


class FgsStats(C.Structure):
    _fields_ = [("visible", C.c_int64), ("pairs", C.c_int64), ("tiles_x", C.c_int32), ("tiles_y", C.c_int32),
                ("sort_passes", C.c_int32), ("big_chunks", C.c_int32),
                ("candidates", C.c_int64), ("entries", C.c_int64), ("cull_batches", C.c_int64)]


class FgsTimings(C.Structure):
    _fields_ = [("frames", C.c_int64), ("ms_preprocess", C.c_double), ("ms_depth_sort", C.c_double),
                ("ms_scan", C.c_double), ("ms_emit", C.c_double), ("ms_super_sort", C.c_double),
                ("ms_tile_lists", C.c_double), ("ms_blend", C.c_double), ("blend_evaluations", C.c_int64),
                ("ms_cull", C.c_double), ("blend_wave_steps", C.c_int64)]


class FgsPeaks(C.Structure):
    _fields_ = [("fma_lane_ops_per_s", C.c_double), ("valu_wave_instr_per_s", C.c_double),
                ("exp_lane_ops_per_s", C.c_double), ("copy_bytes_per_s", C.c_double),
                ("compute_units", C.c_int32), ("clock_mhz", C.c_int32)]


INSTR_STAGE_TIMES = 1
INSTR_WORK = 2
BLEND_LDS_BATCHES = 0
BLEND_PREFETCH = 1
MAX_BATCH_CAMERAS = 8
NOALLOC_SCRATCH_BYTES = 64 << 20   # FGS_NOALLOC_SCRATCH_BYTES


class FgsServerConfig(C.Structure):
    _fields_ = [("budget_bytes", C.c_int64), ("max_inflight", C.c_int32), ("max_width", C.c_int32),
                ("max_height", C.c_int32), ("max_bypass", C.c_int32), ("use_graphs", C.c_int32),
                ("share_queue", C.c_int32), ("batch_fronts", C.c_int32)]


class FgsServerResult(C.Structure):
    _fields_ = [("id", C.c_uint64), ("status", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("slot", C.c_int32), ("rgb", C.c_void_p), ("arrival_ns", C.c_int64), ("start_ns", C.c_int64),
                ("admit_ns", C.c_int64), ("done_ns", C.c_int64), ("visible", C.c_int64), ("pairs", C.c_int64)]


class FgsServerStats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("graphs_captured", C.c_int64), ("graph_launches", C.c_int64), ("region_allocs", C.c_int64),
                ("region_evictions", C.c_int64), ("bypasses", C.c_int64), ("peak_bytes_in_use", C.c_int64),
                ("budget_bytes", C.c_int64), ("slot_bytes", C.c_int64), ("batched_fronts", C.c_int64),
                ("batched_requests", C.c_int64), ("spec_launches", C.c_int64), ("spec_misses", C.c_int64)]


class FgsTraceRequest(C.Structure):
    _fields_ = [("id", C.c_uint64), ("cam", FgsCamera), ("width", C.c_int32), ("height", C.c_int32),
                ("arrival_offset_ns", C.c_int64)]

# name -> (restype, argtypes); the exported symbols of include/fgs.h
PROTOTYPES = {
    "fgs_create": (C.c_int, [C.c_int, C.POINTER(C.c_void_p)]),
    "fgs_destroy": (None, [C.c_void_p]),
    "fgs_status_string": (C.c_char_p, [C.c_int]),
    "fgs_last_error": (C.c_char_p, [C.c_void_p]),
    "fgs_default_options": (None, [C.POINTER(FgsOptions)]),
    "fgs_validate": (C.c_int, [C.POINTER(FgsScene), C.POINTER(FgsCamera), C.c_int32, C.c_int32,
                               C.POINTER(FgsOptions)]),
    "fgs_reserve": (C.c_int, [C.c_void_p, C.c_int64, C.c_int64, C.c_int32, C.c_int32]),
    "fgs_scratch_bytes": (C.c_size_t, [C.c_void_p]),
    "fgs_render": (C.c_int, [C.c_void_p, C.POINTER(FgsScene), C.POINTER(FgsCamera), C.c_int32, C.c_int32,
                             C.POINTER(FgsOptions), C.c_void_p, C.c_void_p, C.c_void_p,
                             C.POINTER(C.c_void_p), C.POINTER(FgsStats), C.c_void_p]),
    "fgs_render_noalloc": (C.c_int, [C.c_void_p, C.POINTER(FgsScene), C.POINTER(FgsCamera), C.c_int32, C.c_int32,
                                     C.POINTER(FgsOptions), C.c_void_p, C.c_void_p, C.c_void_p,
                                     C.POINTER(FgsStats), C.c_void_p]),
    "fgs_render_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(FgsScene), C.POINTER(FgsCamera),
                                      C.POINTER(FgsOptions), C.c_void_p, C.POINTER(FgsSceneGrad), C.c_void_p]),
    "fgs_frame_release": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fgs_frame_field_bytes": (C.c_size_t, [C.c_void_p, C.c_int]),
    "fgs_frame_download": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int, C.c_void_p, C.c_size_t]),
    "fgs_frame_stats": (C.c_int, [C.c_void_p, C.POINTER(FgsStats)]),
    "fgs_set_instrumentation": (C.c_int, [C.c_void_p, C.c_int]),
    "fgs_set_blend_variant": (C.c_int, [C.c_void_p, C.c_int32]),
    "fgs_get_instrumentation": (C.c_int, [C.c_void_p, C.POINTER(FgsTimings)]),
    "fgs_measure_peaks": (C.c_int, [C.c_void_p, C.POINTER(FgsPeaks)]),
    "fgs_plan": (C.c_int, [C.c_void_p, C.POINTER(FgsScene), C.POINTER(FgsCamera), C.c_int32, C.c_int32,
                           C.POINTER(FgsOptions), C.POINTER(C.c_int64), C.POINTER(C.c_size_t), C.c_void_p]),
    "fgs_prepare_scene": (C.c_int, [C.c_void_p, C.POINTER(FgsScene), C.POINTER(FgsOptions),
                                    C.POINTER(C.c_void_p), C.c_void_p]),
    "fgs_prepared_release": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fgs_render_prepared": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(FgsCamera), C.c_int32, C.c_int32,
                                      C.POINTER(FgsOptions), C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.POINTER(C.c_void_p), C.POINTER(FgsStats), C.c_void_p]),
    "fgs_render_prepared_batch": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(FgsCamera), C.c_int32, C.c_int32,
                                            C.c_int32, C.POINTER(FgsOptions), C.POINTER(C.c_void_p),
                                            C.POINTER(C.c_void_p), C.POINTER(C.c_void_p), C.POINTER(FgsStats),
                                            C.c_void_p]),
    "fgs_clock_ns": (C.c_int64, []),
    "fgs_server_create": (C.c_int, [C.c_int, C.POINTER(FgsScene), C.POINTER(FgsOptions),
                                    C.POINTER(FgsServerConfig), C.POINTER(C.c_void_p)]),
    "fgs_server_destroy": (None, [C.c_void_p]),
    "fgs_server_last_error": (C.c_char_p, [C.c_void_p]),
    "fgs_server_submit": (C.c_int, [C.c_void_p, C.c_uint64, C.POINTER(FgsCamera), C.c_int32, C.c_int32,
                                    C.c_int64, C.c_void_p]),
    "fgs_server_poll": (C.c_int32, [C.c_void_p, C.POINTER(FgsServerResult), C.c_int32, C.c_int64]),
    "fgs_server_release": (C.c_int, [C.c_void_p, C.c_uint64]),
    "fgs_server_get_stats": (C.c_int, [C.c_void_p, C.POINTER(FgsServerStats)]),
    "fgs_server_replay": (C.c_int, [C.c_void_p, C.POINTER(FgsTraceRequest), C.c_int64,
                                    C.POINTER(FgsServerResult)]),
    "fgs_replay_plain": (C.c_int, [C.c_void_p, C.POINTER(FgsScene), C.POINTER(FgsOptions),
                                   C.POINTER(FgsTraceRequest), C.c_int64, C.c_void_p, C.POINTER(FgsServerResult),
                                   C.c_void_p]),
    "fgs_replay_plain_prepared": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(FgsOptions),
                                            C.POINTER(FgsTraceRequest), C.c_int64, C.c_void_p,
                                            C.POINTER(FgsServerResult), C.c_void_p]),
}

_lib = None


def lib():
    """Load libfgs.so (built by paper_2408_07967_amd/build.py); raises if missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run paper_2408_07967_amd/build.py "
                               "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in PROTOTYPES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class FgsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{lib().fgs_status_string(status).decode()}: {msg}")
        self.status = status


def check(status, ctx=None):
    if status != FGS_OK:
        raise FgsError(status, lib().fgs_last_error(ctx).decode())


def default_options(**overrides):
    o = FgsOptions()
    lib().fgs_default_options(C.byref(o))
    for k, v in overrides.items():
        if k == "bg":
            for i in range(3):
                o.bg[i] = float(v[i])
        else:
            setattr(o, k, v)
    return o


def make_camera(R, t, eye, fx, fy, cx, cy, near=0.2):
    c = FgsCamera()
    Rf = [float(x) for x in list(R.reshape(-1))] if hasattr(R, "reshape") else [float(x) for x in R]
    for i in range(9):
        c.R[i] = Rf[i]
    for i in range(3):
        c.t[i] = float(t[i])
        c.eye[i] = float(eye[i])
    c.fx, c.fy, c.cx, c.cy, c.near_z = float(fx), float(fy), float(cx), float(cy), float(near)
    return c


def make_scene(P, stride, sh_degree, means, log_scales, quats, logits, sh):
    """Pointers are integer device addresses (e.g. torch tensor data_ptr())."""
    return FgsScene(int(P), int(stride), int(sh_degree), 0, means, log_scales, quats, logits, sh)


class Context:
    """Owns an fgs_context on one device."""

    def __init__(self, device=0):
        h = C.c_void_p()
        check(lib().fgs_create(int(device), C.byref(h)))
        self.handle = h

    def close(self):
        if self.handle:
            lib().fgs_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, status):
        check(status, self.handle)
