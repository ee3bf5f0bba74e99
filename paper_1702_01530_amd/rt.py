"""ctypes binding of libstereort.so (include/stereort.h), with the same names.

Argument marshalling only: every step of the ray tracing runs in the HIP
library.  PyTorch is used for device memory and streams.  If the library has
not been built this module raises on first use; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstereort.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "stereort.h")

RT_OK, RT_ERR_INVALID_ARGUMENT, RT_ERR_BUFFER_TOO_SMALL, RT_ERR_DEVICE, RT_ERR_UNSUPPORTED = range(5)
STATUS_NAMES = {0: "RT_OK", 1: "RT_ERR_INVALID_ARGUMENT", 2: "RT_ERR_BUFFER_TOO_SMALL", 3: "RT_ERR_DEVICE",
                4: "RT_ERR_UNSUPPORTED"}
RT_ACCEL_PLOC, RT_ACCEL_NONE, RT_ACCEL_KARRAS = 0, 1, 2
RT_ACCEL_LBVH, RT_ACCEL_LBVH_KARRAS = RT_ACCEL_PLOC, RT_ACCEL_KARRAS  # earlier names
RT_FLAG_PATH_IDS, RT_FLAG_COUNT_WORK, RT_FLAG_BRUTE_FORCE, RT_FLAG_READBACK_KERNEL = 1, 2, 4, 8
RT_MAX_LIGHTS, RT_MAX_DEPTH = 8, 8
RT_COMPOSE_ANAGLYPH_RED_CYAN, RT_COMPOSE_SIDE_BY_SIDE = 0, 1
RT_NUM_COUNTERS = 8
COUNTER_NAMES = ["primary", "reflection", "shadow", "closest_nodes", "closest_tris", "any_nodes", "any_tris", "errors"]
RT_NUM_STAGES = 8
STAGE_NAMES = ["trace", "shade", "resolve", "setup", "readback"]


class RtError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class rt_material(C.Structure):
    _fields_ = [("albedo", C.c_float * 3), ("specular", C.c_float * 3), ("reflectance", C.c_float * 3),
                ("shininess", C.c_float)]


class rt_light(C.Structure):
    _fields_ = [("position", C.c_float * 3), ("intensity", C.c_float * 3)]


class rt_scene_desc(C.Structure):
    _fields_ = [
        ("num_triangles", C.c_int64), ("triangles", C.c_void_p), ("tri_material", C.c_void_p),
        ("num_spheres", C.c_int32), ("spheres", C.c_void_p), ("sphere_material", C.c_void_p),
        ("num_planes", C.c_int32), ("planes", C.c_void_p), ("plane_material", C.c_void_p),
        ("num_materials", C.c_int32), ("materials", C.POINTER(rt_material)),
        ("num_lights", C.c_int32), ("lights", C.POINTER(rt_light)),
        ("ambient", C.c_float * 3), ("background", C.c_float * 3), ("flags", C.c_uint32),
    ]


class rt_scene_info(C.Structure):
    _fields_ = [
        ("num_triangles", C.c_int64), ("num_spheres", C.c_int64), ("num_planes", C.c_int64),
        ("num_lights", C.c_int64), ("num_materials", C.c_int64), ("bvh_depth", C.c_int32), ("leaf_size", C.c_int32),
        ("num_nodes", C.c_int64), ("node_bytes", C.c_int64), ("triangle_bytes", C.c_int64),
        ("bounds_lo", C.c_float * 3), ("bounds_hi", C.c_float * 3), ("builder", C.c_int32), ("reserved", C.c_int32),
    ]


class rt_stereo_camera(C.Structure):
    _fields_ = [
        ("center", C.c_float * 3), ("forward", C.c_float * 3), ("up", C.c_float * 3),
        ("hfov_deg", C.c_float), ("baseline", C.c_float), ("convergence", C.c_float),
        ("width", C.c_int32), ("height", C.c_int32), ("max_depth", C.c_int32),
    ]


class rt_stereo_output(C.Structure):
    _fields_ = [
        ("radiance", C.c_void_p * 2), ("hit_t", C.c_void_p * 2), ("hit_prim", C.c_void_p * 2),
        ("path_prims", C.c_void_p * 2), ("shadow_state", C.c_void_p * 2), ("host_radiance", C.c_void_p * 2),
        ("ray_counts", C.c_void_p),
    ]


class rt_batch_item(C.Structure):
    _fields_ = [("scene", C.c_void_p), ("camera", rt_stereo_camera), ("out", rt_stereo_output)]


class rt_tuning(C.Structure):
    _fields_ = [("trace_blocks_per_cu", C.c_int32), ("stream_blocks", C.c_int32), ("max_pass_paths", C.c_int64)]


class rt_timing(C.Structure):
    _fields_ = [("ms", C.c_double * RT_NUM_STAGES), ("launches", C.c_int64 * RT_NUM_STAGES)]


_lib = None

_SIGNATURES = {
    "rt_last_error": (C.c_char_p, []),
    "rt_version": (C.c_int32, []),
    "rt_scene_storage_size": (C.c_int, [C.POINTER(rt_scene_desc), C.POINTER(C.c_size_t), C.POINTER(C.c_size_t)]),
    "rt_scene_build": (C.c_int, [C.POINTER(rt_scene_desc), C.c_void_p, C.c_size_t, C.c_void_p, C.c_size_t,
                                 C.c_void_p, C.POINTER(C.c_void_p)]),
    "rt_scene_release": (C.c_int, [C.c_void_p]),
    "rt_scene_get_info": (C.c_int, [C.c_void_p, C.POINTER(rt_scene_info)]),
    "rt_render_workspace_size": (C.c_int, [C.POINTER(rt_stereo_camera), C.c_int32, C.POINTER(C.c_size_t)]),
    "rt_render_workspace_min": (C.c_int, [C.c_int32, C.POINTER(C.c_size_t)]),
    "rt_render_stereo": (C.c_int, [C.c_void_p, C.POINTER(rt_stereo_camera), C.POINTER(rt_stereo_output), C.c_void_p,
                                   C.c_size_t, C.c_uint32, C.c_void_p, C.c_void_p, C.c_void_p]),
    "rt_render_stereo_noalloc": (C.c_int, [C.c_void_p, C.POINTER(rt_stereo_camera), C.POINTER(rt_stereo_output),
                                           C.c_uint32, C.c_void_p, C.c_void_p]),
    "rt_render_batch_workspace_size": (C.c_int, [C.POINTER(rt_batch_item), C.c_int32, C.POINTER(C.c_size_t)]),
    "rt_render_batch": (C.c_int, [C.POINTER(rt_batch_item), C.c_int32, C.c_void_p, C.c_size_t, C.c_uint32,
                                  C.c_void_p, C.c_void_p]),
    "rt_batch_graph_create": (C.c_int, [C.POINTER(rt_batch_item), C.c_int32, C.c_void_p, C.c_size_t, C.c_uint32,
                                        C.c_void_p, C.POINTER(C.c_void_p)]),
    "rt_batch_graph_launch": (C.c_int, [C.c_void_p, C.POINTER(rt_batch_item), C.c_int32, C.c_void_p]),
    "rt_batch_graph_destroy": (C.c_int, [C.c_void_p]),
    "rt_get_tuning": (C.c_int, [C.POINTER(rt_tuning)]),
    "rt_set_tuning": (C.c_int, [C.POINTER(rt_tuning)]),
    "rt_autotune_batch": (C.c_int, [C.POINTER(rt_batch_item), C.c_int32, C.c_void_p, C.c_size_t, C.c_uint32,
                                    C.c_void_p, C.c_int32, C.POINTER(rt_tuning), C.POINTER(C.c_double)]),
    "rt_compose_stereo": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_float, C.c_void_p,
                                    C.c_void_p]),
    "rt_copy_to_host": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "rt_timer_create": (C.c_int, [C.POINTER(C.c_void_p)]),
    "rt_timer_destroy": (C.c_int, [C.c_void_p]),
    "rt_timer_read": (C.c_int, [C.c_void_p, C.POINTER(rt_timing)]),
}


def lib():
    """The loaded library.  Raises if it has not been built (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1702_01530_amd.build` "
                               "(or __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_functions() -> list:
    """Names of the functions include/stereort.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[\w\s\*]*?\b(rt_\w+)\s*\(", text, flags=re.M)))


def last_error() -> str:
    return lib().rt_last_error().decode()


def check(status: int):
    if status != RT_OK:
        raise RtError(status, last_error())


# Same names as the C ABI: thin wrappers that raise RtError on failure.

def rt_scene_storage_size(desc: rt_scene_desc):
    s, k = C.c_size_t(), C.c_size_t()
    check(lib().rt_scene_storage_size(C.byref(desc), C.byref(s), C.byref(k)))
    return s.value, k.value


def rt_scene_build(desc, storage_ptr, storage_bytes, scratch_ptr, scratch_bytes, stream):
    h = C.c_void_p()
    check(lib().rt_scene_build(C.byref(desc), storage_ptr, storage_bytes, scratch_ptr, scratch_bytes, stream,
                               C.byref(h)))
    return h.value


def rt_scene_release(handle):
    check(lib().rt_scene_release(handle))


def rt_scene_get_info(handle) -> dict:
    info = rt_scene_info()
    check(lib().rt_scene_get_info(handle, C.byref(info)))
    out = {k: getattr(info, k) for k, _ in rt_scene_info._fields_}
    out["bounds_lo"] = list(info.bounds_lo)
    out["bounds_hi"] = list(info.bounds_hi)
    return out


def rt_render_workspace_size(cam: rt_stereo_camera, num_lights: int) -> int:
    b = C.c_size_t()
    check(lib().rt_render_workspace_size(C.byref(cam), num_lights, C.byref(b)))
    return b.value


def rt_render_workspace_min(num_lights: int) -> int:
    b = C.c_size_t()
    check(lib().rt_render_workspace_min(num_lights, C.byref(b)))
    return b.value


def rt_render_stereo(handle, cam, out, ws_ptr, ws_bytes, flags, stream, copy_stream=None, timer=None):
    check(lib().rt_render_stereo(handle, C.byref(cam), C.byref(out), ws_ptr, ws_bytes, flags, stream, copy_stream,
                                 timer))


def rt_render_stereo_noalloc(handle, cam, out, flags, stream, copy_stream=None):
    check(lib().rt_render_stereo_noalloc(handle, C.byref(cam), C.byref(out), flags, stream, copy_stream))


def rt_render_batch_workspace_size(items) -> int:
    b = C.c_size_t()
    check(lib().rt_render_batch_workspace_size(items, len(items), C.byref(b)))
    return b.value


def rt_render_batch(items, ws_ptr, ws_bytes, flags, stream, timer=None):
    check(lib().rt_render_batch(items, len(items), ws_ptr, ws_bytes, flags, stream, timer))


def rt_batch_graph_create(items, ws_ptr, ws_bytes, flags, stream):
    g = C.c_void_p()
    check(lib().rt_batch_graph_create(items, len(items), ws_ptr, ws_bytes, flags, stream, C.byref(g)))
    return g.value


def rt_batch_graph_launch(graph, items, stream):
    check(lib().rt_batch_graph_launch(graph, items, len(items), stream))


def rt_batch_graph_destroy(graph):
    check(lib().rt_batch_graph_destroy(graph))


def rt_get_tuning() -> dict:
    t = rt_tuning()
    check(lib().rt_get_tuning(C.byref(t)))
    return {k: getattr(t, k) for k, _ in rt_tuning._fields_}


def rt_set_tuning(trace_blocks_per_cu=0, stream_blocks=8192, max_pass_paths=1 << 25):
    t = rt_tuning(trace_blocks_per_cu, stream_blocks, max_pass_paths)
    check(lib().rt_set_tuning(C.byref(t)))


def rt_autotune_batch(items, ws_ptr, ws_bytes, flags, stream, repeats=2):
    t = rt_tuning()
    ms = C.c_double()
    check(lib().rt_autotune_batch(items, len(items), ws_ptr, ws_bytes, flags, stream, repeats, C.byref(t),
                                  C.byref(ms)))
    return {k: getattr(t, k) for k, _ in rt_tuning._fields_}, ms.value


def rt_compose_stereo(left_ptr, right_ptr, width, height, mode, exposure, out_ptr, stream):
    check(lib().rt_compose_stereo(left_ptr, right_ptr, width, height, mode, exposure, out_ptr, stream))


def rt_copy_to_host(dev_ptr, host_ptr, nbytes, stream):
    check(lib().rt_copy_to_host(dev_ptr, host_ptr, nbytes, stream))


def rt_timer_create():
    t = C.c_void_p()
    check(lib().rt_timer_create(C.byref(t)))
    return t.value


def rt_timer_destroy(t):
    check(lib().rt_timer_destroy(t))


def rt_timer_read(t) -> dict:
    tm = rt_timing()
    check(lib().rt_timer_read(t, C.byref(tm)))
    return {name: (tm.ms[i], tm.launches[i]) for i, name in enumerate(STAGE_NAMES)}


# ---------------------------------------------------------------------------------------------
# Struct builders
# ---------------------------------------------------------------------------------------------

def _f3(v):
    a = np.asarray(v, np.float32).reshape(3)
    return (C.c_float * 3)(*[float(x) for x in a])


def make_camera_struct(cam) -> rt_stereo_camera:
    """From any object with center, forward, up, hfov_deg, baseline, convergence, width, height, max_depth."""
    c = rt_stereo_camera()
    c.center, c.forward, c.up = _f3(cam.center), _f3(cam.forward), _f3(cam.up)
    c.hfov_deg, c.baseline, c.convergence = float(cam.hfov_deg), float(cam.baseline), float(cam.convergence)
    c.width, c.height, c.max_depth = int(cam.width), int(cam.height), int(cam.max_depth)
    return c


def make_materials(mats) -> C.Array:
    mats = np.asarray(mats, np.float32).reshape(-1, 10)
    arr = (rt_material * max(1, len(mats)))()
    for i, m in enumerate(mats):
        arr[i].albedo = (C.c_float * 3)(*m[0:3].tolist())
        arr[i].specular = (C.c_float * 3)(*m[3:6].tolist())
        arr[i].reflectance = (C.c_float * 3)(*m[6:9].tolist())
        arr[i].shininess = float(m[9])
    return arr


def make_lights(lights) -> C.Array:
    lights = np.asarray(lights, np.float32).reshape(-1, 6)
    arr = (rt_light * max(1, len(lights)))()
    for i, l in enumerate(lights):
        arr[i].position = (C.c_float * 3)(*l[0:3].tolist())
        arr[i].intensity = (C.c_float * 3)(*l[3:6].tolist())
    return arr
