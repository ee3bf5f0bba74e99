"""FP64 brute-force stereo Whitted ray-tracing oracle (ctypes binding).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.

``render(..., accel="bvh")`` answers the same queries through an FP64 triangle
hierarchy instead of testing every primitive: the same radiance and signature
(the tests check it against the brute-force mode), no margins.  The C++
source (``oracle.cpp``) shares no code with the GPU path.

``render`` returns, per sampled path (path id = eye*H*W + row*W + col):
radiance [n,3] f64, primary hit t and id, the ray-tree signature (closest-hit id
per depth, shadow state per depth and light: 0 not cast, 1 occluded, 2 visible)
and the decision margins used to certify FP32/FP64 disagreements.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

# No contraction, no fast-math: every operation is one correctly rounded binary64 operation.
CXXFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-pthread"]


def build(force: bool = False) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["g++", *CXXFLAGS, _SRC, "-o", tmp], check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Scene(C.Structure):
    _fields_ = [
        ("num_triangles", C.c_int64), ("triangles", C.c_void_p), ("tri_material", C.c_void_p),
        ("num_spheres", C.c_int32), ("spheres", C.c_void_p), ("sphere_material", C.c_void_p),
        ("num_planes", C.c_int32), ("planes", C.c_void_p), ("plane_material", C.c_void_p),
        ("num_materials", C.c_int32), ("materials", C.c_void_p),
        ("num_lights", C.c_int32), ("lights", C.c_void_p),
        ("ambient", C.c_float * 3), ("background", C.c_float * 3),
    ]


class _Camera(C.Structure):
    _fields_ = [
        ("center", C.c_float * 3), ("forward", C.c_float * 3), ("up", C.c_float * 3),
        ("hfov_deg", C.c_float), ("baseline", C.c_float), ("convergence", C.c_float),
        ("width", C.c_int32), ("height", C.c_int32), ("max_depth", C.c_int32),
    ]


class _Output(C.Structure):
    _fields_ = [
        ("radiance", C.c_void_p), ("hit_t", C.c_void_p), ("hit_prim", C.c_void_p), ("path_prims", C.c_void_p),
        ("shadow_state", C.c_void_p), ("hit_margin", C.c_void_p), ("shadow_margin", C.c_void_p),
        ("shadow_contrib", C.c_void_p), ("path_t", C.c_void_p), ("hit_cos", C.c_void_p),
        ("ray_counts", C.c_int64 * 3), ("seconds", C.c_double * 2),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        for name in ("orc_render", "orc_render_bvh"):
            f = getattr(_lib, name)
            f.restype = C.c_int
            f.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.c_void_p, C.c_int64, C.c_int32, C.POINTER(_Output)]
        _lib.orc_render_shifted.restype = C.c_int
        _lib.orc_render_shifted.argtypes = [C.POINTER(_Scene), C.POINTER(_Camera), C.c_void_p, C.c_int64, C.c_int32,
                                            C.c_int32, C.c_void_p, C.POINTER(_Output)]
        _lib.orc_primary_ray.argtypes = [C.POINTER(_Camera), C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p]
        _lib.orc_primary_ray.restype = None
        d = C.c_void_p
        _lib.orc_intersect_triangle.argtypes = [d, d, d, d, d, C.c_double, C.c_double, d, d, d, d]
        _lib.orc_intersect_triangle.restype = C.c_int32
        _lib.orc_intersect_sphere.argtypes = [d, d, d, C.c_double, C.c_double, C.c_double, d, d]
        _lib.orc_intersect_sphere.restype = C.c_int32
        _lib.orc_intersect_plane.argtypes = [d, d, d, C.c_double, C.c_double, C.c_double, d, d]
        _lib.orc_intersect_plane.restype = C.c_int32
        _lib.orc_closest_hits.argtypes = [C.POINTER(_Scene), d, d, C.c_int64, C.c_double, d, d, d, d]
        _lib.orc_closest_hits.restype = C.c_int32
        _lib.orc_occluded.argtypes = [C.POINTER(_Scene), d, d, C.c_int64, C.c_double, d, d, d, d]
        _lib.orc_occluded.restype = C.c_int32
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class _Held:
    """Keeps the contiguous arrays a ctypes struct points into alive."""

    def __init__(self):
        self.arrays = []

    def f32(self, a):
        a = np.ascontiguousarray(a, dtype=np.float32)
        self.arrays.append(a)
        return a

    def u32(self, a):
        a = np.ascontiguousarray(a, dtype=np.uint32)
        self.arrays.append(a)
        return a


def _scene_struct(scene, held: _Held) -> _Scene:
    s = _Scene()
    s.num_triangles = scene.triangles.shape[0]
    s.triangles = _ptr(held.f32(scene.triangles))
    s.tri_material = _ptr(held.u32(scene.tri_material))
    s.num_spheres = scene.spheres.shape[0]
    s.spheres = _ptr(held.f32(scene.spheres))
    s.sphere_material = _ptr(held.u32(scene.sphere_material))
    s.num_planes = scene.planes.shape[0]
    s.planes = _ptr(held.f32(scene.planes))
    s.plane_material = _ptr(held.u32(scene.plane_material))
    s.num_materials = scene.materials.shape[0]
    s.materials = _ptr(held.f32(scene.materials))
    s.num_lights = scene.lights.shape[0]
    s.lights = _ptr(held.f32(scene.lights))
    s.ambient = (C.c_float * 3)(*[float(x) for x in np.asarray(scene.ambient, np.float32)])
    s.background = (C.c_float * 3)(*[float(x) for x in np.asarray(scene.background, np.float32)])
    return s


def _camera_struct(cam) -> _Camera:
    c = _Camera()
    c.center = (C.c_float * 3)(*np.asarray(cam.center, np.float32).tolist())
    c.forward = (C.c_float * 3)(*np.asarray(cam.forward, np.float32).tolist())
    c.up = (C.c_float * 3)(*np.asarray(cam.up, np.float32).tolist())
    c.hfov_deg = float(np.float32(cam.hfov_deg))
    c.baseline = float(np.float32(cam.baseline))
    c.convergence = float(np.float32(cam.convergence))
    c.width, c.height, c.max_depth = int(cam.width), int(cam.height), int(cam.max_depth)
    return c


def default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def render(scene, cam, samples=None, nthreads=None, accel="brute", t_shift=None) -> dict:
    """Oracle render of the sampled paths (None: every path of both eyes).

    accel="brute" tests every primitive for every query and returns the decision margins; accel="bvh"
    answers the same queries through an FP64 triangle hierarchy (the same radiance and ray-tree signature,
    margins NaN), for whole frames of large scenes.  t_shift ([n, D+1], optional) moves each path's hit
    point at each depth along its ray by that signed distance, keeping the primitive hit."""
    if accel not in ("brute", "bvh"):
        raise ValueError(f"unknown accel {accel!r}")
    held = _Held()
    s = _scene_struct(scene, held)
    c = _camera_struct(cam)
    if samples is None:
        n = 2 * cam.width * cam.height
        samp = None
    else:
        samp = np.ascontiguousarray(samples, dtype=np.int64)
        n = samp.shape[0]
        if n and (samp.min() < 0 or samp.max() >= 2 * cam.width * cam.height):
            raise ValueError("sample path id out of range")
    D1 = cam.max_depth + 1
    L = scene.lights.shape[0]
    res = {
        "radiance": np.zeros((n, 3)), "hit_t": np.zeros(n), "hit_prim": np.zeros(n, np.int32),
        "path_prims": np.zeros((n, D1), np.int32), "shadow_state": np.zeros((n, D1, L), np.uint8),
        "hit_margin": np.zeros((n, D1)), "shadow_margin": np.zeros((n, D1, L)),
        "shadow_contrib": np.zeros((n, D1, L)), "path_t": np.zeros((n, D1)), "hit_cos": np.zeros(n),
    }
    o = _Output()
    for k in ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state", "hit_margin", "shadow_margin",
              "shadow_contrib", "path_t", "hit_cos"):
        setattr(o, k, _ptr(res[k]))
    nt = int(nthreads or default_threads())
    if t_shift is not None:
        shift = np.ascontiguousarray(t_shift, dtype=np.float64)
        if shift.shape != (n, D1) or not np.isfinite(shift).all():
            raise ValueError(f"t_shift must be finite with shape {(n, D1)}")
        rc = lib().orc_render_shifted(C.byref(s), C.byref(c), _ptr(samp), n, nt, int(accel == "bvh"),
                                      _ptr(shift), C.byref(o))
    else:
        fn = lib().orc_render if accel == "brute" else lib().orc_render_bvh
        rc = fn(C.byref(s), C.byref(c), _ptr(samp), n, nt, C.byref(o))
    if rc != 0:
        raise ValueError("oracle render rejected its arguments")
    res["ray_counts"] = np.array(list(o.ray_counts), np.int64)
    res["seconds"] = {"tree_build": float(o.seconds[0]), "trace": float(o.seconds[1])}
    res["samples"] = samp if samp is not None else np.arange(n, dtype=np.int64)
    return res


def primary_ray(cam, eye: int, col: int, row: int):
    c = _camera_struct(cam)
    O = np.zeros(3)
    d = np.zeros(3)
    lib().orc_primary_ray(C.byref(c), eye, col, row, O.ctypes.data, d.ctypes.data)
    return O, d


def _v(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def intersect_triangle(O, d, v0, v1, v2, tmin=0.0, tmax=np.inf, with_margin=False):
    """(hit, t, u, v) of one ray and one triangle; with_margin adds the decision margin."""
    O, d, v0, v1, v2 = map(_v, (O, d, v0, v1, v2))
    t, u, v, m = np.zeros(1), np.zeros(1), np.zeros(1), np.zeros(1)
    hit = lib().orc_intersect_triangle(O.ctypes.data, d.ctypes.data, v0.ctypes.data, v1.ctypes.data,
                                       v2.ctypes.data, tmin, tmax, t.ctypes.data, u.ctypes.data, v.ctypes.data,
                                       m.ctypes.data)
    res = (bool(hit), float(t[0]), float(u[0]), float(v[0]))
    return res + (float(m[0]),) if with_margin else res


def intersect_sphere(O, d, c, r, tmin=0.0, tmax=np.inf, with_margin=False):
    """(hit, t) of one ray (unit d) and one sphere; with_margin adds disc / r^2."""
    O, d, c = map(_v, (O, d, c))
    t, m = np.zeros(1), np.zeros(1)
    hit = lib().orc_intersect_sphere(O.ctypes.data, d.ctypes.data, c.ctypes.data, float(r), tmin, tmax, t.ctypes.data,
                                     m.ctypes.data)
    res = (bool(hit), float(t[0]))
    return res + (float(m[0]),) if with_margin else res


def intersect_plane(O, d, n, dist, tmin=0.0, tmax=np.inf, with_margin=False):
    """(hit, t) of one ray and the plane n.x = dist; with_margin adds the sine of the grazing angle."""
    O, d, n = map(_v, (O, d, n))
    t, m = np.zeros(1), np.zeros(1)
    hit = lib().orc_intersect_plane(O.ctypes.data, d.ctypes.data, n.ctypes.data, float(dist), tmin, tmax,
                                    t.ctypes.data, m.ctypes.data)
    res = (bool(hit), float(t[0]))
    return res + (float(m[0]),) if with_margin else res


def encode8(x, exposure=1.0):
    """Display code of linear values: floor(255 * sqrt(clamp(x * exposure, 0, 1)) + 0.5), each step one
    correctly rounded float32 operation (the same precision as the device path, which decides the same
    integers)."""
    x = np.asarray(x, np.float32)
    v = np.float32(x * np.float32(exposure))
    v = np.minimum(np.maximum(v, np.float32(0.0)), np.float32(1.0))
    g = np.sqrt(v, dtype=np.float32)
    m = np.float32(np.float32(255.0) * g)
    return np.floor(np.float32(m + np.float32(0.5))).astype(np.uint8)


def compose_stereo(left, right, mode="anaglyph", exposure=1.0):
    """Stereo-pair building for a display (the paper's post-processing, Section 3, Fig. 2): a red-cyan
    anaglyph (red from the left eye, green and blue from the right) or the two images side by side,
    as 8-bit RGBA with alpha 255.  left/right: [H, W, 3] linear radiance."""
    left = np.asarray(left, np.float32)
    right = np.asarray(right, np.float32)
    H, W, _ = left.shape
    if mode == "anaglyph":
        rgb = np.stack([encode8(left[..., 0], exposure), encode8(right[..., 1], exposure),
                        encode8(right[..., 2], exposure)], axis=-1)
    elif mode == "side_by_side":
        rgb = np.concatenate([encode8(left, exposure), encode8(right, exposure)], axis=1)
    else:
        raise ValueError(mode)
    alpha = np.full(rgb.shape[:2] + (1,), 255, np.uint8)
    return np.concatenate([rgb, alpha], axis=-1)


def closest_hits(scene, O, d, tmin=0.0, exclude=None):
    """Closest hit (t, prim id, margin) of explicit rays [n,3] against every primitive of the scene."""
    held = _Held()
    s = _scene_struct(scene, held)
    O = _v(O).reshape(-1, 3)
    d = _v(d).reshape(-1, 3)
    n = O.shape[0]
    ex = None if exclude is None else np.ascontiguousarray(exclude, dtype=np.int64)
    t = np.zeros(n)
    p = np.zeros(n, np.int64)
    m = np.zeros(n)
    lib().orc_closest_hits(C.byref(s), O.ctypes.data, d.ctypes.data, n, float(tmin), _ptr(ex), t.ctypes.data,
                           p.ctypes.data, m.ctypes.data)
    return t, p, m


def occluded(scene, O, d, tmax, tmin=1e-4, exclude=None):
    """Occlusion (t in (tmin, tmax)) of explicit segments [n,3] by any primitive but `exclude`, and the
    decision margin of each."""
    held = _Held()
    s = _scene_struct(scene, held)
    O = _v(O).reshape(-1, 3)
    d = _v(d).reshape(-1, 3)
    n = O.shape[0]
    tm = np.ascontiguousarray(np.broadcast_to(np.asarray(tmax, np.float64), (n,)))
    ex = None if exclude is None else np.ascontiguousarray(exclude, dtype=np.int64)
    occ = np.zeros(n, np.int32)
    m = np.zeros(n)
    lib().orc_occluded(C.byref(s), O.ctypes.data, d.ctypes.data, n, float(tmin), tm.ctypes.data, _ptr(ex),
                       occ.ctypes.data, m.ctypes.data)
    return occ.astype(bool), m
