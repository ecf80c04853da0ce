"""ctypes view of the libgbs C ABI (include/gbs.h).

Loads the in-tree libgbs.so; raises if it is missing (there is no fallback).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgbs.so")

GBS_OK = 0
GBS_E_INVALID = -1
GBS_E_OOM = -2
GBS_E_HIP = -3
GBS_E_UNSUPPORTED = -4
GBS_E_STATE = -5

MODES = {"f64": 0, "mix": 1, "f32": 2}

FLAG_TABLE_HOST = 1
FLAG_VALIDATE = 2
FLAG_COUNT_ACTIVE = 4
FLAG_TIME_KERNELS = 8

c_int32, c_int64, c_double, c_void_p = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class GbsRays(ctypes.Structure):
    _fields_ = [("n_src", c_int32), ("n_rays", c_int64), ("ray_ptr", c_void_p), ("ray_w", c_void_p),
                ("ray_src", c_void_p)]


class GbsSegs(ctypes.Structure):
    _fields_ = [("n_segs", c_int64), ("a", c_void_p), ("t", c_void_p), ("s0", c_void_p), ("lo", c_void_p),
                ("hi", c_void_p), ("face_ptr", c_void_p), ("face_ids", c_void_p), ("e1", c_void_p)]


class GbsFaces(ctypes.Structure):
    _fields_ = [("n_faces", c_int32), ("gamma", c_void_p)]


class GbsParams(ctypes.Structure):
    _fields_ = [("c", c_double), ("gate_G", c_double), ("mode", c_int32), ("flags", c_int32),
                ("chunk_segs", c_int64), ("rcv_per_lane", c_int32), ("work_chunk", c_int32), ("alpha", c_void_p),
                ("eps_e2", c_void_p)]


class GbsScene(ctypes.Structure):
    _fields_ = [("n_boxes", c_int32), ("panels", c_int32), ("boxes", c_void_p), ("s_max", c_double),
                ("max_refl", c_int32), ("image_complete", c_int32)]


class GbsFan(ctypes.Structure):
    _fields_ = [("n_src", c_int32), ("src_xyz", c_void_p), ("n_rays", c_int64), ("dirs", c_void_p),
                ("ray_src", c_void_p), ("s_max_src", c_void_p), ("e1", c_void_p)]


class GbsStats(ctypes.Structure):
    _fields_ = [("dense_pairs", c_int64), ("listed_pairs", c_int64), ("active_pairs", c_int64),
                ("n_items", c_int64), ("n_chunks", c_int32), ("patch_rcv", c_int32), ("ms_pairs", c_double),
                ("ms_cull", c_double), ("grid", c_int32), ("blocks_per_cu", c_int32),
                ("scratch_bytes", c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


EXPORTS = ("gbs_create", "gbs_destroy", "gbs_set_stream", "gbs_forward", "gbs_forward_noalloc", "gbs_backward",
           "gbs_get_stats", "gbs_graph_create", "gbs_graph_launch", "gbs_graph_destroy", "gbs_autotune", "gbs_trace_count",
           "gbs_trace", "gbs_air_absorption_db", "gbs_impulse_response", "gbs_last_error", "gbs_version")

_lib = None


class GbsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libgbs error {code}: {msg}")
        self.code = code


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libgbs.so is not built ({LIB_PATH}); run paper_2501_13382_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    lib.gbs_create.argtypes = [P(c_void_p), ctypes.c_int, c_void_p]
    lib.gbs_create.restype = ctypes.c_int
    lib.gbs_destroy.argtypes = [c_void_p]
    lib.gbs_destroy.restype = None
    lib.gbs_set_stream.argtypes = [c_void_p, c_void_p]
    lib.gbs_set_stream.restype = ctypes.c_int
    common = [c_void_p, P(GbsRays), P(GbsSegs), P(GbsFaces), c_void_p, c_int64, c_void_p, c_int32, c_void_p,
              P(GbsParams)]
    lib.gbs_forward.argtypes = common + [c_void_p, c_void_p]
    lib.gbs_forward.restype = ctypes.c_int
    lib.gbs_forward_noalloc.argtypes = common + [c_void_p, c_void_p]
    lib.gbs_forward_noalloc.restype = ctypes.c_int
    lib.gbs_backward.argtypes = common + [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.gbs_backward.restype = ctypes.c_int
    lib.gbs_get_stats.argtypes = [c_void_p, P(GbsStats)]
    lib.gbs_get_stats.restype = ctypes.c_int
    lib.gbs_graph_create.argtypes = common + [c_void_p, c_void_p, P(c_void_p)]
    lib.gbs_graph_create.restype = ctypes.c_int
    lib.gbs_graph_launch.argtypes = [c_void_p]
    lib.gbs_graph_launch.restype = ctypes.c_int
    lib.gbs_graph_destroy.argtypes = [c_void_p]
    lib.gbs_graph_destroy.restype = None
    lib.gbs_autotune.argtypes = common + [c_void_p, P(c_int32), P(c_int32)]
    lib.gbs_autotune.restype = ctypes.c_int
    lib.gbs_trace_count.argtypes = [c_void_p, P(GbsScene), P(GbsFan), P(c_int64), P(c_int64), P(c_int64)]
    lib.gbs_trace_count.restype = ctypes.c_int
    lib.gbs_trace.argtypes = [c_void_p, P(GbsScene), P(GbsFan), c_int64, c_int64, c_int64] + [c_void_p] * 9 + \
        [P(c_int64), P(c_int64)]
    lib.gbs_trace.restype = ctypes.c_int
    lib.gbs_impulse_response.argtypes = [c_void_p, P(GbsRays), P(GbsSegs), P(GbsFaces), c_void_p, c_int64, c_double,
                                         c_int32, c_int32, c_void_p, c_void_p, P(GbsParams), c_int32, c_int32,
                                         c_void_p]
    lib.gbs_impulse_response.restype = ctypes.c_int
    lib.gbs_air_absorption_db.argtypes = [c_double, c_double, c_double, c_double]
    lib.gbs_air_absorption_db.restype = c_double
    lib.gbs_last_error.argtypes = [c_void_p]
    lib.gbs_last_error.restype = ctypes.c_char_p
    lib.gbs_version.argtypes = []
    lib.gbs_version.restype = ctypes.c_int
    _lib = lib
    return lib


def check(rc: int, ctx) -> None:
    if rc != GBS_OK:
        msg = load().gbs_last_error(ctx)
        raise GbsError(rc, msg.decode() if msg else "")
