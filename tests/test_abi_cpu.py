"""The C ABI on the host: the library loads without a GPU, exports every declared
function, and validates arguments before touching a device."""
import ctypes as C

import numpy as np
import pytest

import scenegen as sg
from paper_1702_01530_amd import rt


def test_library_exports_every_declared_function():
    L = rt.lib()
    names = rt.header_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing
    assert set(names) == set(rt._SIGNATURES)
    assert rt.lib().rt_version() >= 100


def _desc(T=10, S=0, P=0, M=1, L=1):
    d = rt.rt_scene_desc()
    d.num_triangles, d.num_spheres, d.num_planes, d.num_materials, d.num_lights = T, S, P, M, L
    return d


def test_storage_size_queries():
    s0, k0 = rt.rt_scene_storage_size(_desc(T=1000))
    s1, k1 = rt.rt_scene_storage_size(_desc(T=2000))
    assert s1 > s0 >= 999 * 64 + 1000 * 48 and k1 > k0 > 0
    d = _desc(T=1000)
    d.flags = rt.RT_ACCEL_NONE
    s2, _ = rt.rt_scene_storage_size(d)
    assert s2 < s0  # no nodes without a BVH
    s3, _ = rt.rt_scene_storage_size(_desc(T=0, S=3, P=1))
    assert s3 > 0


@pytest.mark.parametrize("field,value,needle", [
    ("num_triangles", -1, "num_triangles"),
    ("num_materials", 0, "num_materials"),
    ("num_lights", 9, "num_lights"),
    ("flags", 8, "flags"),
    ("flags", 3, "flags"),
])
def test_descriptor_validation(field, value, needle):
    d = _desc()
    setattr(d, field, value)
    with pytest.raises(rt.RtError) as ei:
        rt.rt_scene_storage_size(d)
    assert ei.value.status == rt.RT_ERR_INVALID_ARGUMENT
    assert needle in rt.last_error()


def test_tree_builders_plan_their_own_scratch():
    """Both tree builders are accepted with the same storage.  The clustering build's scratch is the larger,
    so a clustering tree too deep for the traversal stack can be rebuilt by emission + refit in place."""
    sizes = {}
    for flags in (rt.RT_ACCEL_PLOC, rt.RT_ACCEL_KARRAS, rt.RT_ACCEL_NONE):
        d = _desc(T=100000)
        d.flags = flags
        sizes[flags] = rt.rt_scene_storage_size(d)
    assert sizes[rt.RT_ACCEL_PLOC][0] == sizes[rt.RT_ACCEL_KARRAS][0] > sizes[rt.RT_ACCEL_NONE][0]
    assert sizes[rt.RT_ACCEL_PLOC][1] > sizes[rt.RT_ACCEL_KARRAS][1] > sizes[rt.RT_ACCEL_NONE][1]
    assert (rt.RT_ACCEL_LBVH, rt.RT_ACCEL_LBVH_KARRAS) == (rt.RT_ACCEL_PLOC, rt.RT_ACCEL_KARRAS)  # earlier names


def test_build_rejects_bad_pointers_before_device_use():
    d = _desc(T=5)
    with pytest.raises(rt.RtError) as ei:
        rt.rt_scene_build(d, None, 0, None, 0, None)
    assert ei.value.status == rt.RT_ERR_INVALID_ARGUMENT and "NULL" in str(ei.value)
    assert rt.lib().rt_scene_build(None, None, 0, None, 0, None, None) == rt.RT_ERR_INVALID_ARGUMENT


def test_camera_validation_and_workspace():
    _, cam = sg.make_terrain_1080p()
    c = rt.make_camera_struct(cam)
    full = rt.rt_render_workspace_size(c, 4)
    mn = rt.rt_render_workspace_min(4)
    assert full > mn > 0
    c2 = rt.make_camera_struct(cam.resized(3840, 2160))
    assert rt.rt_render_workspace_size(c2, 4) > full
    for field, value in (("hfov_deg", 180.0), ("width", 0), ("max_depth", 9), ("baseline", -1.0)):
        bad = rt.make_camera_struct(cam)
        setattr(bad, field, value)
        with pytest.raises(rt.RtError) as ei:
            rt.rt_render_workspace_size(bad, 4)
        assert ei.value.status == rt.RT_ERR_INVALID_ARGUMENT
    bad = rt.make_camera_struct(cam.with_(forward=np.float32([0, 1, 0])))
    with pytest.raises(rt.RtError, match="parallel"):
        rt.rt_render_workspace_size(bad, 4)


def test_compose_validation_without_device():
    L = rt.lib()
    assert L.rt_compose_stereo(None, None, 4, 4, 0, 1.0, None, None) == rt.RT_ERR_INVALID_ARGUMENT
    assert L.rt_compose_stereo(8, 8, 4, 4, 7, 1.0, 8, None) == rt.RT_ERR_INVALID_ARGUMENT
    assert "mode" in rt.last_error()
    assert L.rt_compose_stereo(8, 8, 4, 4, 0, -1.0, 8, None) == rt.RT_ERR_INVALID_ARGUMENT
    assert L.rt_copy_to_host(None, None, 4, None) == rt.RT_ERR_INVALID_ARGUMENT


def test_tuning_validation():
    saved = rt.rt_get_tuning()
    assert saved["max_pass_paths"] >= 4096 and saved["stream_blocks"] >= 1
    for bad in ({"trace_blocks_per_cu": -1}, {"stream_blocks": 0}, {"max_pass_paths": 100}):
        args = dict(saved)
        args.update(bad)
        with pytest.raises(rt.RtError):
            rt.rt_set_tuning(**args)
    rt.rt_set_tuning(2, 512, 1 << 20)
    assert rt.rt_get_tuning() == {"trace_blocks_per_cu": 2, "stream_blocks": 512, "max_pass_paths": 1 << 20}
    rt.rt_set_tuning(**saved)


def test_render_argument_checks_without_device():
    _, cam = sg.make_spheres_scene()
    c = rt.make_camera_struct(cam)
    out = rt.rt_stereo_output()
    assert rt.lib().rt_render_stereo(None, C.byref(c), C.byref(out), None, 0, 0, None, None, None) == \
        rt.RT_ERR_INVALID_ARGUMENT
    assert "scene" in rt.last_error()
    assert rt.lib().rt_timer_read(None, None) == rt.RT_ERR_INVALID_ARGUMENT
    t = rt.rt_timer_create()
    rt.rt_timer_destroy(t)


_NO_DEVICE_BUILD = r"""
import ctypes as C, numpy as np
from paper_1702_01530_amd import rt
tris = np.zeros((1, 3, 3), np.float32)
tris[0, 1, 0] = tris[0, 2, 1] = 1.0
mat = np.zeros(1, np.uint32)
mats, lights = (rt.rt_material * 1)(), (rt.rt_light * 1)()
mats[0].shininess = 8.0
lights[0].intensity[0] = 1.0
d = rt.rt_scene_desc()
d.num_triangles, d.num_materials, d.num_lights = 1, 1, 1
d.triangles, d.tri_material = tris.ctypes.data, mat.ctypes.data
d.materials, d.lights = C.cast(mats, C.POINTER(rt.rt_material)), C.cast(lights, C.POINTER(rt.rt_light))
sb, kb = rt.rt_scene_storage_size(d)
h = C.c_void_p()
# storage and scratch addresses are never dereferenced: without a device the build stops at its first HIP call
st = rt.lib().rt_scene_build(C.byref(d), C.c_void_p(1 << 20), sb, C.c_void_p(1 << 24), kb, None, C.byref(h))
print(st, h.value is None)
print(rt.last_error())
"""


def test_valid_build_without_a_device_reports_a_device_error():
    """A valid scene build on a host without a GPU returns RT_ERR_DEVICE with the runtime's message and no
    handle, and the process goes on (no abort).  Run in a child process so that the HIP runtime's state does
    not carry over; skipped where a device exists (the dummy storage addresses would then reach a build)."""
    import os
    import subprocess
    import sys
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a device is present")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    p = subprocess.run([sys.executable, "-c", _NO_DEVICE_BUILD], capture_output=True, text=True, timeout=120, cwd=root)
    assert p.returncode == 0, p.stderr
    status, msg = p.stdout.strip().splitlines()
    assert status.split() == [str(rt.RT_ERR_DEVICE), "True"] and "device" in msg.lower(), p.stdout
