"""ctypes binding of librtq.so: the C ABI of include/rt.h, same names.

Argument marshalling only.  Loading fails loudly when the library is not
built; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtq.so")

RT_SUCCESS = 0
RT_ERROR_INVALID_VALUE = 1
RT_ERROR_OUT_OF_MEMORY = 2
RT_ERROR_NO_DEVICE = 3
RT_ERROR_HIP = 4
RT_ERROR_UNSUPPORTED = 5
RT_ERROR_INDEX_OUT_OF_RANGE = 6
RT_ERROR_STACK_OVERFLOW = 7
RT_INVALID_ID = 0xFFFFFFFF
RT_NOALLOC_SCRATCH_BYTES = 64 << 20

EXPORTS = [
    "rt_context_create", "rt_context_destroy", "rt_context_set_variant", "rt_context_get_variant",
    "rt_context_set_timing", "rt_context_read_timing",
    "rt_build", "rt_accel_destroy", "rt_accel_get_info",
    "rt_trace_closest", "rt_trace_closest_noalloc", "rt_trace_any", "rt_trace_backward",
    "rt_trace_backward_instances",
    "rt_trace_closest_ex", "rt_trace_any_ex", "rt_trace_all", "rt_accel_set_instance_masks", "rt_update_instances",
    "rt_ao_rays", "rt_ao_rays_instances", "rt_ao_resolve",
    "rt_trace_counters", "rt_trace_counters_ex", "rt_refit",
    "rt_autotune",
    "rt_batch_plan_create", "rt_batch_plan_create_instances", "rt_batch_plan_launch", "rt_batch_plan_graph", "rt_batch_plan_destroy",
    "rt_status_string", "rt_last_error_message", "rt_version",
]


class rt_ray(C.Structure):
    _fields_ = [(n, C.c_float) for n in ("ox", "oy", "oz", "tmin", "dx", "dy", "dz", "tmax")]


class rt_hit(C.Structure):
    _fields_ = [("t", C.c_float), ("prim_id", C.c_uint32), ("u", C.c_float), ("v", C.c_float)]


class rt_srt(C.Structure):
    _fields_ = [(n, C.c_float) for n in ("sx", "sy", "sz", "qx", "qy", "qz", "qw", "tx", "ty", "tz")]


class rt_mesh_desc(C.Structure):
    _fields_ = [
        ("vertices", C.c_void_p), ("vertex_count", C.c_uint32), ("vertex_stride", C.c_uint32),
        ("indices", C.c_void_p), ("triangle_count", C.c_uint32), ("index_stride", C.c_uint32),
    ]


class rt_build_options(C.Structure):
    _fields_ = [("node_width", C.c_uint32), ("max_leaf_size", C.c_uint32), ("flags", C.c_uint32)]


class rt_variant(C.Structure):
    _fields_ = [("stack_entries", C.c_uint32), ("workgroup", C.c_uint32)]


class rt_query_options(C.Structure):
    _fields_ = [("ray_masks", C.c_void_p), ("skip_inst", C.c_void_p), ("skip_prim", C.c_void_p)]


RT_MAX_HIT_CAPACITY = 64
RT_BUILD_DEVICE = 0x1


class rt_tune_entry(C.Structure):
    _fields_ = [("node_width", C.c_uint32), ("stack_entries", C.c_uint32), ("workgroup", C.c_uint32),
                ("ms", C.c_float)]


class rt_accel_info(C.Structure):
    _fields_ = [
        ("node_width", C.c_uint32), ("node_count", C.c_uint32), ("triangle_count", C.c_uint32),
        ("input_triangles", C.c_uint32), ("instance_count", C.c_uint32), ("max_depth", C.c_uint32),
        ("max_stack", C.c_uint32), ("leaf_count", C.c_uint32), ("sah_cost", C.c_double),
        ("device_bytes", C.c_uint64),
    ]


_lock = threading.Lock()
_lib = None


def load():
    """Loads librtq.so (once).  Raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2603_00292_amd.build_lib`")
        lib = C.CDLL(LIB_PATH)
        P, U32, I32 = C.c_void_p, C.c_uint32, C.c_int
        sig = {
            "rt_context_create": [I32, P],
            "rt_context_destroy": [P],
            "rt_context_set_variant": [P, P],
            "rt_context_get_variant": [P, P],
            "rt_context_set_timing": [P, U32],
            "rt_context_read_timing": [P, P, U32, P],
            "rt_build": [P, P, U32, P, P, U32, P, P, P],
            "rt_accel_destroy": [P],
            "rt_accel_get_info": [P, P],
            "rt_trace_closest": [P, P, U32, P, P, P],
            "rt_trace_closest_noalloc": [P, P, U32, P, P, P],
            "rt_trace_any": [P, P, U32, P, P],
            "rt_trace_backward": [P, P, P, P, U32, P, P, P, P],
            "rt_trace_backward_instances": [P, P, P, P, P, U32, P, P, P, P, P],
            "rt_trace_counters": [P, P, U32, I32, P, P, P, P],
            "rt_trace_counters_ex": [P, P, U32, I32, P, P, P, U32, P],
            "rt_trace_closest_ex": [P, P, U32, P, P, P, P],
            "rt_trace_any_ex": [P, P, U32, P, P, P],
            "rt_trace_all": [P, P, U32, P, U32, P, P, P, P],
            "rt_accel_set_instance_masks": [P, P, P],
            "rt_update_instances": [P, P, P],
            "rt_ao_rays": [P, P, P, U32, U32, P, C.c_float, C.c_float, P, P],
            "rt_ao_rays_instances": [P, P, P, P, U32, U32, P, C.c_float, C.c_float, P, P],
            "rt_ao_resolve": [P, U32, U32, P, P],
            "rt_refit": [P, P, P],
            "rt_autotune": [P, P, P, U32, U32, P, P, P, U32, P],
            "rt_batch_plan_create": [P, P, P, P, P, U32, P],
            "rt_batch_plan_create_instances": [P, P, P, P, P, P, U32, P],
            "rt_batch_plan_launch": [P, P],
            "rt_batch_plan_graph": [P, P, P],
            "rt_batch_plan_destroy": [P],
        }
        for name, args in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = C.c_int
        lib.rt_status_string.argtypes = [C.c_int]
        lib.rt_status_string.restype = C.c_char_p
        lib.rt_last_error_message.argtypes = []
        lib.rt_last_error_message.restype = C.c_char_p
        lib.rt_version.argtypes = []
        lib.rt_version.restype = C.c_uint32
        _lib = lib
        return lib


class RtError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        name = lib.rt_status_string(status).decode()
        msg = lib.rt_last_error_message().decode()
        super().__init__(f"{where}: {name}: {msg}")
        self.status = status


def check(status: int, where: str) -> None:
    if status != RT_SUCCESS:
        raise RtError(status, where)


def call(name: str, *args) -> int:
    """Calls a C-ABI function and raises RtError on failure."""
    lib = load()
    st = getattr(lib, name)(*args)
    check(st, name)
    return st
