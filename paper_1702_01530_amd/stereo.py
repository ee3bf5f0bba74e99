"""PyTorch-facing helpers over the C ABI: device memory and streams come from torch,
every computation runs in libstereort.so.

    gs = GpuScene(scene)              # uploads the arrays and builds the LBVH on the device
    out = render_stereo(gs, camera)   # both eyes, device tensors
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import rt


def stream_handle(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def aligned_buffer(nbytes: int, device) -> tuple:
    """A uint8 device tensor holding at least nbytes from a 256-byte aligned address."""
    t = torch.empty(int(nbytes) + 256, dtype=torch.uint8, device=device)
    ptr = t.data_ptr()
    return t, ptr + ((-ptr) % 256)


def _dev(a, dtype, device):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=dtype)).to(device)


class GpuScene:
    """A scene built into device storage.  `scene` is any object with the FP32 arrays
    triangles [T,3,3], tri_material [T], spheres [S,4], sphere_material [S], planes [P,4],
    plane_material [P], materials [M,10], lights [L,6], ambient [3], background [3]."""

    ACCEL = {"ploc": rt.RT_ACCEL_PLOC, "karras": rt.RT_ACCEL_KARRAS, "none": rt.RT_ACCEL_NONE,
             "lbvh": rt.RT_ACCEL_PLOC, "lbvh_karras": rt.RT_ACCEL_KARRAS}  # the last two: earlier names
    BUILDERS = {rt.RT_ACCEL_PLOC: "ploc", rt.RT_ACCEL_KARRAS: "karras", rt.RT_ACCEL_NONE: "none"}

    def __init__(self, scene, accel: str = "ploc", device=None, stream=None):
        """accel: "ploc" (binary tree by locally-ordered clustering over the Morton order, the default),
        "karras" (the linear BVH: Karras emission over the Morton codes + refit) or "none" (brute force).
        info()["builder"] names the builder that made the tree (a too-deep clustering tree falls back to
        "karras")."""
        if accel not in self.ACCEL:
            raise ValueError(f"accel must be one of {sorted(self.ACCEL)}")
        self.device = torch.device(device or "cuda")
        tri = _dev(scene.triangles, np.float32, self.device)
        # material indices are uint32 in the ABI; int32 tensors carry the same bits for values < 2^31
        tmat = _dev(np.asarray(scene.tri_material, np.uint32).view(np.int32), np.int32, self.device)
        sph = _dev(scene.spheres, np.float32, self.device)
        smat = _dev(np.asarray(scene.sphere_material, np.uint32).view(np.int32), np.int32, self.device)
        pl = _dev(scene.planes, np.float32, self.device)
        pmat = _dev(np.asarray(scene.plane_material, np.uint32).view(np.int32), np.int32, self.device)
        self._materials = rt.make_materials(scene.materials)
        self._lights = rt.make_lights(scene.lights)
        d = rt.rt_scene_desc()
        d.num_triangles = int(tri.shape[0])
        d.triangles, d.tri_material = tri.data_ptr(), tmat.data_ptr()
        d.num_spheres = int(sph.shape[0])
        d.spheres, d.sphere_material = sph.data_ptr(), smat.data_ptr()
        d.num_planes = int(pl.shape[0])
        d.planes, d.plane_material = pl.data_ptr(), pmat.data_ptr()
        d.num_materials = int(np.asarray(scene.materials).reshape(-1, 10).shape[0])
        d.materials = C.cast(self._materials, C.POINTER(rt.rt_material))
        d.num_lights = int(np.asarray(scene.lights).reshape(-1, 6).shape[0])
        d.lights = C.cast(self._lights, C.POINTER(rt.rt_light))
        d.ambient = rt._f3(scene.ambient)
        d.background = rt._f3(scene.background)
        d.flags = self.ACCEL[accel]
        self.desc = d
        storage, scratch = rt.rt_scene_storage_size(d)
        self._storage, sptr = aligned_buffer(storage, self.device)
        self.storage_offset = sptr - self._storage.data_ptr()  # where the built scene starts in _storage
        scratch_t, kptr = aligned_buffer(scratch, self.device)
        self.storage_bytes, self.scratch_bytes = storage, scratch
        self.handle = rt.rt_scene_build(d, sptr, storage, kptr, scratch, stream_handle(stream))
        del scratch_t, tri, tmat, sph, smat, pl, pmat  # the build blocked; storage holds all it needs
        self.num_lights = d.num_lights
        self.num_triangles = d.num_triangles

    def info(self) -> dict:
        out = rt.rt_scene_get_info(self.handle)
        out["builder_name"] = self.BUILDERS.get(out["builder"], str(out["builder"]))
        return out

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize(self.device)
            rt.rt_scene_release(self.handle)
            self.handle = None
            self._storage = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Workspace:
    """A reusable render workspace (device bytes)."""

    def __init__(self, nbytes: int, device=None):
        self.device = torch.device(device or "cuda")
        self.nbytes = int(nbytes)
        self._buf, self.ptr = aligned_buffer(self.nbytes, self.device)

    @staticmethod
    def for_camera(cam, num_lights: int, device=None) -> "Workspace":
        return Workspace(rt.rt_render_workspace_size(rt.make_camera_struct(cam), num_lights), device)


def alloc_outputs(cam, num_lights: int, device, path_ids=False, host=False, counts=True) -> dict:
    H, W, D1 = int(cam.height), int(cam.width), int(cam.max_depth) + 1
    o = {
        "radiance": torch.empty((2, H, W, 3), dtype=torch.float32, device=device),
        "hit_t": torch.empty((2, H, W), dtype=torch.float32, device=device),
        "hit_prim": torch.empty((2, H, W), dtype=torch.int32, device=device),
    }
    if path_ids:
        o["path_prims"] = torch.empty((2, H, W, D1), dtype=torch.int32, device=device)
        o["shadow_state"] = torch.empty((2, H, W, D1, max(num_lights, 1)), dtype=torch.uint8, device=device)
    if host:
        o["host_radiance"] = torch.empty((2, H, W, 3), dtype=torch.float32, pin_memory=True)
    if counts:
        o["ray_counts"] = torch.zeros(rt.RT_NUM_COUNTERS, dtype=torch.int64, device=device)
    return o


def output_struct(o: dict) -> rt.rt_stereo_output:
    s = rt.rt_stereo_output()
    for k in ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state", "host_radiance"):
        if k in o and o[k] is not None:
            t = o[k]
            getattr(s, k)[0] = t[0].data_ptr()
            getattr(s, k)[1] = t[1].data_ptr()
    if o.get("ray_counts") is not None:
        s.ray_counts = o["ray_counts"].data_ptr()
    return s


def render_stereo(gs: GpuScene, cam, *, path_ids=False, count_work=False, brute_force=False, host=False,
                  workspace: Workspace | None = None, outputs: dict | None = None, stream=None, copy_stream=None,
                  timer=None, readback_kernel=False) -> dict:
    """Renders both eyes; returns the output tensors (valid after the stream is synchronised)."""
    flags = (rt.RT_FLAG_PATH_IDS if path_ids else 0) | (rt.RT_FLAG_COUNT_WORK if count_work else 0) | (
        rt.RT_FLAG_BRUTE_FORCE if brute_force else 0) | (rt.RT_FLAG_READBACK_KERNEL if readback_kernel else 0)
    camst = rt.make_camera_struct(cam)
    if workspace is None:
        workspace = Workspace(rt.rt_render_workspace_size(camst, gs.num_lights), gs.device)
    o = outputs if outputs is not None else alloc_outputs(cam, gs.num_lights, gs.device, path_ids, host)
    st = output_struct(o)
    rt.rt_render_stereo(gs.handle, camst, st, workspace.ptr, workspace.nbytes, flags, stream_handle(stream),
                        copy_stream.cuda_stream if copy_stream is not None else None, timer)
    return o


def _flags(path_ids=False, count_work=False, brute_force=False, readback_kernel=False) -> int:
    return (rt.RT_FLAG_PATH_IDS if path_ids else 0) | (rt.RT_FLAG_COUNT_WORK if count_work else 0) | (
        rt.RT_FLAG_BRUTE_FORCE if brute_force else 0) | (rt.RT_FLAG_READBACK_KERNEL if readback_kernel else 0)


def batch_items(pairs, outs) -> C.Array:
    items = (rt.rt_batch_item * len(pairs))()
    for i, (gs, cam) in enumerate(pairs):
        items[i].scene = gs.handle
        items[i].camera = rt.make_camera_struct(cam)
        items[i].out = output_struct(outs[i])
    return items


def batch_outputs(pairs, path_ids=False, host=False) -> list:
    return [alloc_outputs(cam, gs.num_lights, gs.device, path_ids, host, counts=(i == 0))
            for i, (gs, cam) in enumerate(pairs)]


def render_batch(pairs, *, path_ids=False, count_work=False, brute_force=False, host=False,
                 workspace: Workspace | None = None, outputs: list | None = None, stream=None, timer=None,
                 readback_kernel=False) -> list:
    """Renders a batch of (GpuScene, camera) pairs as one pipeline; returns one output dict per pair.
    The batch's total ray counts go to the first pair's ``ray_counts``."""
    flags = _flags(path_ids, count_work, brute_force, readback_kernel)
    outs = outputs if outputs is not None else batch_outputs(pairs, path_ids, host)
    items = batch_items(pairs, outs)
    if workspace is None:
        workspace = Workspace(rt.rt_render_batch_workspace_size(items), pairs[0][0].device)
    rt.rt_render_batch(items, workspace.ptr, workspace.nbytes, flags, stream_handle(stream), timer)
    return outs


class BatchGraph:
    """A batch's render passes captured into a HIP graph; launch() replays them for any batch of the same
    shape (item count, sizes, depths, light counts) with new scenes, poses and outputs."""

    def __init__(self, pairs, outputs: list, workspace: Workspace, *, path_ids=False, readback_kernel=False,
                 stream=None):
        self.flags = _flags(path_ids=path_ids, readback_kernel=readback_kernel)
        self.workspace = workspace
        self._stream = stream if stream is not None else torch.cuda.Stream()
        items = batch_items(pairs, outputs)
        self.handle = rt.rt_batch_graph_create(items, workspace.ptr, workspace.nbytes, self.flags,
                                               self._stream.cuda_stream)

    def launch(self, pairs, outputs: list, stream=None):
        items = batch_items(pairs, outputs)
        rt.rt_batch_graph_launch(self.handle, items, stream_handle(stream))
        return outputs

    def close(self):
        if getattr(self, "handle", None):
            torch.cuda.synchronize()
            rt.rt_batch_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def autotune_batch(pairs, outputs: list, workspace: Workspace, repeats=2, stream=None) -> tuple:
    """Times the batch under each candidate launch tuning, installs the fastest and returns (tuning, ms)."""
    items = batch_items(pairs, outputs)
    return rt.rt_autotune_batch(items, workspace.ptr, workspace.nbytes, 0, stream_handle(stream), repeats)


def compose(out: dict, mode: str = "anaglyph", exposure: float = 1.0, stream=None) -> torch.Tensor:
    """Builds the 8-bit RGBA display image of a rendered stereo pair on the device
    ("anaglyph": red-cyan, H x W x 4; "side_by_side": H x 2W x 4)."""
    m = {"anaglyph": rt.RT_COMPOSE_ANAGLYPH_RED_CYAN, "side_by_side": rt.RT_COMPOSE_SIDE_BY_SIDE}[mode]
    rad = out["radiance"]
    H, W = rad.shape[1], rad.shape[2]
    img = torch.empty((H, W * (2 if m == rt.RT_COMPOSE_SIDE_BY_SIDE else 1), 4), dtype=torch.uint8, device=rad.device)
    rt.rt_compose_stereo(rad[0].data_ptr(), rad[1].data_ptr(), W, H, m, float(exposure), img.data_ptr(),
                         stream_handle(stream))
    return img


class Timer:
    def __init__(self):
        self.handle = rt.rt_timer_create()

    def read(self) -> dict:
        return rt.rt_timer_read(self.handle)

    def close(self):
        if self.handle:
            rt.rt_timer_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
