"""ctypes declarations of libm3s (include/m3s.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libm3s.so")

M3S_OK = 0
STATUS_NAMES = {0: "M3S_OK", 1: "M3S_ERR_NULL", 2: "M3S_ERR_SHAPE", 3: "M3S_ERR_PARAM",
                4: "M3S_ERR_WORKSPACE", 5: "M3S_ERR_HIP", 6: "M3S_ERR_UNSUPPORTED"}
M3S_BATCH_GRAPH = 0x1
M3S_BATCH_AUTOTUNE = 0x2
M3S_BWD_ACCUMULATE = 0x4

c_fp = ctypes.POINTER(ctypes.c_float)


class Params(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("lambda_init", ctypes.c_float),
                ("refine_radius", ctypes.c_int32), ("refine_levels", ctypes.c_int32), ("conf_min", ctypes.c_float),
                ("max_theta", ctypes.c_float), ("max_dist", ctypes.c_float)]


class Pair(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("D", ctypes.c_int32),
                ("Xii", ctypes.c_void_p), ("Xji", ctypes.c_void_p), ("Dii", ctypes.c_void_p),
                ("Dji", ctypes.c_void_p), ("Qii", ctypes.c_void_p), ("Qji", ctypes.c_void_p),
                ("p_init", ctypes.c_void_p)]


class Outputs(ctypes.Structure):
    _fields_ = [("p", ctypes.c_void_p), ("idx", ctypes.c_void_p), ("valid", ctypes.c_void_p),
                ("theta", ctypes.c_void_p), ("xhat", ctypes.c_void_p)]


class Edge(ctypes.Structure):
    _fields_ = [("in_", Pair), ("out", Outputs), ("max_iter", ctypes.c_int32),
                ("refine_radius", ctypes.c_int32)]


class BwdEdge(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("Xii", ctypes.c_void_p), ("Xji", ctypes.c_void_p),
                ("p", ctypes.c_void_p), ("valid", ctypes.c_void_p), ("grad_p", ctypes.c_void_p),
                ("grad_xhat", ctypes.c_void_p), ("grad_Xii", ctypes.c_void_p), ("grad_Xji", ctypes.c_void_p)]


class TrackParams(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("q_min", ctypes.c_float), ("sigma_ray", ctypes.c_float),
                ("sigma_dist", ctypes.c_float), ("huber", ctypes.c_float)]


class TrackProblem(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("Xk", ctypes.c_void_p), ("Xf", ctypes.c_void_p),
                ("idx", ctypes.c_void_p), ("valid", ctypes.c_void_p), ("Qf", ctypes.c_void_p),
                ("Qk", ctypes.c_void_p)]


class FuseProblem(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int32), ("W", ctypes.c_int32), ("Xc", ctypes.c_void_p), ("Cc", ctypes.c_void_p),
                ("X", ctypes.c_void_p), ("C", ctypes.c_void_p)]


class BackendParams(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("q_min", ctypes.c_float), ("sigma_ray", ctypes.c_float),
                ("sigma_dist", ctypes.c_float), ("huber", ctypes.c_float), ("step_tol", ctypes.c_double)]


class BackendProblem(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("H", ctypes.c_int32), ("W", ctypes.c_int32), ("E", ctypes.c_int32),
                ("Xc", ctypes.c_void_p), ("Q", ctypes.c_void_p), ("edges", ctypes.c_void_p),
                ("idx", ctypes.c_void_p), ("valid", ctypes.c_void_p)]


class LaunchConfig(ctypes.Structure):
    _fields_ = [("tile_config", ctypes.c_int32), ("grid", ctypes.c_int32), ("xcd_remap", ctypes.c_int32),
                ("ray_margin", ctypes.c_int32), ("lm_unroll", ctypes.c_int32)]


M3S_PATH_COUNTERS = 8
M3S_NOALLOC_MAX_PIXELS = 1 << 18
PATH_NAMES = ["lm_global", "refine_global", "refine_query", "bwd_direct", "refine_bands"]


class M3SError(RuntimeError):
    def __init__(self, fn: str, status: int, detail: str):
        self.status = status
        super().__init__("%s failed: %s (%s)" % (fn, STATUS_NAMES.get(status, status), detail))


# Every symbol include/m3s.h declares, for the export check.
EXPORTS = ["m3s_default_params", "m3s_workspace_bytes", "m3s_match_fwd", "m3s_match_bwd",
           "m3s_batched_workspace_bytes", "m3s_match_batched", "m3s_batched_last_config",
           "m3s_clear_caches", "m3s_status_string", "m3s_last_error", "m3s_version",
           "m3s_timing_enable", "m3s_timing_read", "m3s_timing_reset", "m3s_stats_workspace_bytes",
           "m3s_match_stats", "m3s_default_track_params", "m3s_track_workspace_bytes", "m3s_track_pose",
           "m3s_fuse_pointmap", "m3s_default_backend_params", "m3s_backend_workspace_bytes", "m3s_backend_gn",
           "m3s_debug_set_launch", "m3s_path_counters", "m3s_match_fwd_noalloc",
           "m3s_bwd_batched_workspace_bytes", "m3s_match_bwd_batched", "m3s_batched_last_launch",
           "m3s_set_tune_cache"]

_lib = None


def load(path: str = LIB_PATH):
    """Load libm3s.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libm3s.so is not built (%s); run `python -m paper_2412_12392_amd.build`" % path)
    lib = ctypes.CDLL(path)
    P, PP, PO, PE = ctypes.POINTER(Params), ctypes.POINTER(Pair), ctypes.POINTER(Outputs), ctypes.POINTER(Edge)
    vp, sz, i32, u32 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32, ctypes.c_uint32
    lib.m3s_default_params.argtypes = [P]
    lib.m3s_default_params.restype = None
    lib.m3s_workspace_bytes.argtypes = [PP, P]
    lib.m3s_workspace_bytes.restype = sz
    lib.m3s_match_fwd.argtypes = [PP, P, PO, vp, sz, vp]
    lib.m3s_match_fwd.restype = ctypes.c_int
    lib.m3s_match_fwd_noalloc.argtypes = [PP, P, PO, vp]
    lib.m3s_match_fwd_noalloc.restype = ctypes.c_int
    lib.m3s_match_bwd.argtypes = [PP, PO, vp, vp, vp, vp, vp]
    lib.m3s_match_bwd.restype = ctypes.c_int
    lib.m3s_bwd_batched_workspace_bytes.argtypes = [i32]
    lib.m3s_bwd_batched_workspace_bytes.restype = sz
    lib.m3s_match_bwd_batched.argtypes = [ctypes.POINTER(BwdEdge), i32, u32, vp, sz, vp]
    lib.m3s_match_bwd_batched.restype = ctypes.c_int
    lib.m3s_batched_workspace_bytes.argtypes = [PE, i32, P]
    lib.m3s_batched_workspace_bytes.restype = sz
    lib.m3s_match_batched.argtypes = [PE, i32, P, u32, vp, sz, vp]
    lib.m3s_match_batched.restype = ctypes.c_int
    lib.m3s_batched_last_config.argtypes = [ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.m3s_batched_last_config.restype = None
    lib.m3s_clear_caches.argtypes = []
    lib.m3s_clear_caches.restype = None
    lib.m3s_status_string.argtypes = [ctypes.c_int]
    lib.m3s_status_string.restype = ctypes.c_char_p
    lib.m3s_last_error.argtypes = []
    lib.m3s_last_error.restype = ctypes.c_char_p
    lib.m3s_version.argtypes = []
    lib.m3s_version.restype = i32
    lib.m3s_timing_enable.argtypes = [i32]
    lib.m3s_timing_enable.restype = None
    lib.m3s_timing_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
    lib.m3s_timing_read.restype = ctypes.c_int
    lib.m3s_timing_reset.argtypes = []
    lib.m3s_timing_reset.restype = None
    lib.m3s_stats_workspace_bytes.argtypes = [i32, i32]
    lib.m3s_stats_workspace_bytes.restype = sz
    lib.m3s_match_stats.argtypes = [PO, i32, i32, vp, vp, sz, vp]
    lib.m3s_match_stats.restype = ctypes.c_int
    TP, TPr = ctypes.POINTER(TrackParams), ctypes.POINTER(TrackProblem)
    lib.m3s_default_track_params.argtypes = [TP]
    lib.m3s_default_track_params.restype = None
    lib.m3s_track_workspace_bytes.argtypes = [i32, i32]
    lib.m3s_track_workspace_bytes.restype = sz
    lib.m3s_track_pose.argtypes = [TPr, TP, vp, vp, vp, sz, vp]
    lib.m3s_track_pose.restype = ctypes.c_int
    lib.m3s_fuse_pointmap.argtypes = [ctypes.POINTER(FuseProblem), vp, vp]
    lib.m3s_fuse_pointmap.restype = ctypes.c_int
    BP, BPr = ctypes.POINTER(BackendParams), ctypes.POINTER(BackendProblem)
    lib.m3s_default_backend_params.argtypes = [BP]
    lib.m3s_default_backend_params.restype = None
    lib.m3s_backend_workspace_bytes.argtypes = [i32, i32, i32, i32]
    lib.m3s_backend_workspace_bytes.restype = sz
    lib.m3s_backend_gn.argtypes = [BPr, BP, vp, vp, vp, sz, vp]
    lib.m3s_backend_gn.restype = ctypes.c_int
    lib.m3s_debug_set_launch.argtypes = [ctypes.POINTER(LaunchConfig)]
    lib.m3s_debug_set_launch.restype = None
    lib.m3s_batched_last_launch.argtypes = [ctypes.POINTER(LaunchConfig)]
    lib.m3s_batched_last_launch.restype = None
    lib.m3s_set_tune_cache.argtypes = [ctypes.c_char_p]
    lib.m3s_set_tune_cache.restype = ctypes.c_int
    lib.m3s_path_counters.argtypes = [ctypes.POINTER(ctypes.c_int64), i32]
    lib.m3s_path_counters.restype = ctypes.c_int
    if path == LIB_PATH:
        _lib = lib
    return lib


def check(lib, fn: str, status: int):
    if status != M3S_OK:
        raise M3SError(fn, status, lib.m3s_last_error().decode(errors="replace"))


def default_params(lib=None, **overrides) -> Params:
    lib = lib or load()
    p = Params()
    lib.m3s_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise TypeError("unknown parameter %s" % k)
        setattr(p, k, v)
    return p


def default_track_params(lib=None, **overrides) -> TrackParams:
    lib = lib or load()
    p = TrackParams()
    lib.m3s_default_track_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise TypeError("unknown parameter %s" % k)
        setattr(p, k, v)
    return p


def default_backend_params(lib=None, **overrides) -> BackendParams:
    lib = lib or load()
    p = BackendParams()
    lib.m3s_default_backend_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise TypeError("unknown parameter %s" % k)
        setattr(p, k, v)
    return p
