"""Serving stereo renders with continuous batching.

Requests (scene id, stereo camera) arrive at any time.  The server keeps the
scenes resident, admits waiting requests while the HBM budget and a free batch
slot allow, renders each admitted group as one batch (rt_render_batch) on that
slot's stream, and completes requests as their batch's readback lands in pinned
host memory.  Several slots are in flight at once, so requests that arrive while
others are on the GPU start as soon as a slot frees up and their work overlaps
on the device with the batches already running.

Admission is first-come first-served with bounded bypass: when the oldest
waiting request does not fit the remaining budget, younger ones that fit may
go ahead, but at most ``max_bypass`` batches in a row; after that admission
waits for the oldest request, so no request starves.  A request that is
invalid or whose render fails is failed alone; the others in its batch
complete.

The scheduler (``Server``) is independent of the GPU: it drives any object
with the ``Renderer`` interface; ``GpuRenderer`` renders through the HIP
library.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any, Callable, Optional


@dataclasses.dataclass
class Request:
    rid: int
    scene_id: Any
    camera: Any
    arrival: float = 0.0
    admitted: Optional[float] = None
    done: Optional[float] = None
    result: Any = None
    error: Optional[str] = None
    bypassed: int = 0  # batches launched ahead of this request while it waited at the head

    @property
    def latency(self) -> Optional[float]:
        return None if self.done is None else self.done - self.arrival


class Renderer:
    """Interface the scheduler drives (implemented by GpuRenderer and by test fakes)."""

    slots: int = 1

    def bytes_needed(self, req: Request) -> int:  # device bytes the request holds while in flight
        raise NotImplementedError

    def paths(self, req: Request) -> int:  # work units the request adds to a batch
        raise NotImplementedError

    def validate(self, req: Request) -> Optional[str]:  # error text for a request that cannot be rendered
        return None

    def cost(self, req: Request) -> float:  # relative device work of the request (any unit)
        return float(self.paths(req))

    def reserved_bytes(self) -> int:  # device bytes the renderer holds for itself (not per request)
        return 0

    def launch(self, slot: int, reqs: list) -> Any:  # enqueue the batch; returns a handle
        raise NotImplementedError

    def poll(self, handle) -> bool:  # True once the batch's results are in host memory
        raise NotImplementedError

    def collect(self, handle) -> list:  # per request: (result, error or None)
        raise NotImplementedError


class Server:
    def __init__(self, renderer: Renderer, hbm_budget: int, max_batch_paths: int, max_batch: int = 64,
                 max_bypass: int = 4, clock: Callable[[], float] = time.perf_counter,
                 on_complete: Optional[Callable[[Request], None]] = None, group_ratio: Optional[float] = None):
        self.r = renderer
        self.budget = int(hbm_budget) - int(renderer.reserved_bytes())
        if self.budget <= 0:
            raise ValueError("the renderer's own device memory leaves no budget for requests")
        if group_ratio is not None and group_ratio < 1.0:
            raise ValueError("group_ratio must be >= 1")
        self.group_ratio = group_ratio  # None: requests of any cost share a batch
        self.max_batch_paths = int(max_batch_paths)
        self.max_batch = int(max_batch)
        self.max_bypass = int(max_bypass)
        self.clock = clock
        self.waiting: collections.deque = collections.deque()
        self.free_slots = list(range(renderer.slots))
        self.inflight = {}  # slot -> (handle, [requests])
        self.in_use = 0
        self.peak_in_use = 0
        self.completed: list = []
        self.on_complete = on_complete
        self.batches = 0
        self.batch_sizes: list = []

    # ------------------------------------------------------------------ API
    def submit(self, req: Request):
        if req.arrival == 0.0:
            req.arrival = self.clock()
        err = self.r.validate(req)
        if err is None and self.r.bytes_needed(req) > self.budget:
            err = "request needs more device memory than the whole budget"
        if err is None and self.r.paths(req) > self.max_batch_paths:
            err = "request exceeds the largest batch"
        if err is not None:
            req.error = err
            req.done = self.clock()
            self.completed.append(req)
            return
        self.waiting.append(req)

    def idle(self) -> bool:
        return not self.waiting and not self.inflight

    def step(self):
        """Completes finished batches, then launches new batches into free slots."""
        for slot in list(self.inflight):
            handle, reqs = self.inflight[slot]
            if not self.r.poll(handle):
                continue
            now = self.clock()
            outs = self.r.collect(handle)
            for req, (res, err) in zip(reqs, outs):
                req.result, req.error, req.done = res, err, now
                self.in_use -= self.r.bytes_needed(req)
                self.completed.append(req)
                if self.on_complete:
                    self.on_complete(req)
            del self.inflight[slot]
            self.free_slots.append(slot)
        while self.free_slots and self.waiting:
            batch = self._admit()
            if not batch:
                break
            slot = self.free_slots.pop(0)
            now = self.clock()
            for req in batch:
                req.admitted = now
            try:
                handle = self.r.launch(slot, batch)
            except Exception as exc:  # the launch itself failed: fail this batch, keep serving
                for req in batch:
                    req.error, req.done = f"launch failed: {exc}", self.clock()
                    self.in_use -= self.r.bytes_needed(req)
                    self.completed.append(req)
                self.free_slots.append(slot)
                continue
            self.inflight[slot] = (handle, batch)
            self.batches += 1
            self.batch_sizes.append(len(batch))

    def run(self, arrivals: list, timeout_s: float = 600.0):
        """Plays back (time offset, request) arrivals against the clock and serves until all complete."""
        t0 = self.clock()
        pending = sorted(arrivals, key=lambda x: x[0])
        i = 0
        while i < len(pending) or not self.idle():
            now = self.clock()
            while i < len(pending) and t0 + pending[i][0] <= now:
                req = pending[i][1]
                req.arrival = t0 + pending[i][0]
                self.submit(req)
                i += 1
            self.step()
            if now - t0 > timeout_s:
                raise TimeoutError("serving did not drain")
        return self.completed

    # ------------------------------------------------------------ admission
    def _admit(self) -> list:
        batch, paths = [], 0
        head = self.waiting[0]
        head_fits = self.in_use + self.r.bytes_needed(head) <= self.budget
        may_bypass = head.bypassed < self.max_bypass
        kept = collections.deque()
        lead_cost = None  # cost of the batch's first request (cost-class grouping)
        while self.waiting and len(batch) < self.max_batch:
            req = self.waiting.popleft()
            need = self.r.bytes_needed(req)
            fits = self.in_use + need <= self.budget and paths + self.r.paths(req) <= self.max_batch_paths
            if fits and batch and self.group_ratio is not None:
                c = self.r.cost(req)
                fits = lead_cost / self.group_ratio <= c <= lead_cost * self.group_ratio
            if fits and (req is head or head_fits or may_bypass):
                if not batch:
                    lead_cost = self.r.cost(req)
                batch.append(req)
                paths += self.r.paths(req)
                self.in_use += need
            else:
                kept.append(req)
                if req is head and not may_bypass:
                    break  # the head has waited long enough: admit nothing past it
        kept.extend(self.waiting)
        self.waiting = kept
        if batch and head not in batch:
            head.bypassed += 1
        self.peak_in_use = max(self.peak_in_use, self.in_use)
        return batch


def latency_stats(done: list) -> dict:
    import numpy as np
    lat = np.array([r.latency for r in done if r.error is None and r.latency is not None])
    if lat.size == 0:
        return {"n": 0}
    t0 = min(r.arrival for r in done)
    t1 = max(r.done for r in done)
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "stereo_fps": float(lat.size / (t1 - t0)), "span_s": float(t1 - t0),
            "errors": int(sum(r.error is not None for r in done))}


class GpuRenderer(Renderer):
    """Renders admitted batches with rt_render_batch on one stream per slot, reading the radiance of both
    eyes back into pinned host memory; a request's device outputs live from launch to completion."""

    def __init__(self, scenes: dict, slots: int = 3, workspace_bytes: int = 4 << 30, device=None,
                 path_ids: bool = False):
        import torch

        from . import rt
        from .stereo import Workspace
        self.torch, self.rt = torch, rt
        self.scenes = scenes  # scene id -> GpuScene
        self.slots = int(slots)
        self.device = torch.device(device or "cuda")
        self.streams = [torch.cuda.Stream(self.device) for _ in range(self.slots)]
        self.workspaces = [Workspace(workspace_bytes, self.device) for _ in range(self.slots)]
        self.path_ids = path_ids
        self._pinned = collections.defaultdict(list)  # shape -> free pinned buffers

    def output_bytes(self, cam, num_lights: int = 0) -> int:
        """Device bytes of one request's outputs: radiance, hit t and id per pixel of both eyes, and the
        ray-tree signature (path ids, shadow states) when it is recorded."""
        n = 2 * int(cam.width) * int(cam.height)
        per_pixel = 12 + 4 + 4
        if self.path_ids:
            d1 = int(cam.max_depth) + 1
            per_pixel += 4 * d1 + d1 * max(int(num_lights), 1)
        return n * per_pixel

    def bytes_needed(self, req: Request) -> int:
        gs = self.scenes.get(req.scene_id)
        return self.output_bytes(req.camera, gs.num_lights if gs is not None else 0)

    def paths(self, req: Request) -> int:
        tiles = -(-int(req.camera.width) // 8) * -(-int(req.camera.height) // 8)
        return 2 * 64 * tiles

    def cost(self, req: Request) -> float:
        """Relative device work: paths, weighted by the shadow rays (one per light) and the mirror bounces
        a path can spawn."""
        gs = self.scenes.get(req.scene_id)
        lights = gs.num_lights if gs is not None else 0
        return self.paths(req) * (1.0 + 0.5 * lights) * (1.0 + 0.15 * int(req.camera.max_depth))

    def reserved_bytes(self) -> int:
        return sum(ws.nbytes for ws in self.workspaces)

    def validate(self, req: Request) -> Optional[str]:
        if req.scene_id not in self.scenes:
            return f"unknown scene {req.scene_id!r}"
        try:
            self.rt.rt_render_workspace_size(self.rt.make_camera_struct(req.camera),
                                             self.scenes[req.scene_id].num_lights)
        except self.rt.RtError as exc:
            return str(exc)
        return None

    def _host_buffer(self, cam):
        key = (int(cam.height), int(cam.width))
        if self._pinned[key]:
            return self._pinned[key].pop()
        return self.torch.empty((2,) + key + (3,), dtype=self.torch.float32, pin_memory=True)

    def release(self, host):
        """Returns a result's pinned host buffer to the pool."""
        self._pinned[(host.shape[1], host.shape[2])].append(host)

    def prewarm(self, sizes, count: int):
        """Allocates `count` pinned host buffers per (width, height) ahead of serving."""
        for w, h in sizes:
            for _ in range(count):
                self._pinned[(int(h), int(w))].append(
                    self.torch.empty((2, int(h), int(w), 3), dtype=self.torch.float32, pin_memory=True))

    def launch(self, slot: int, reqs: list):
        from .stereo import alloc_outputs, batch_items
        torch = self.torch
        pairs = [(self.scenes[r.scene_id], r.camera) for r in reqs]
        outs = []
        for gs, cam in pairs:
            o = alloc_outputs(cam, gs.num_lights, self.device, path_ids=self.path_ids, counts=False)
            o["host_radiance"] = self._host_buffer(cam)
            outs.append(o)
        items = batch_items(pairs, outs)
        stream = self.streams[slot]
        ws = self.workspaces[slot]
        flags = self.rt.RT_FLAG_PATH_IDS if self.path_ids else 0
        with torch.cuda.stream(stream):
            self.rt.rt_render_batch(items, ws.ptr, ws.nbytes, flags, stream.cuda_stream, None)
            ev = torch.cuda.Event()
            ev.record(stream)
        return (ev, outs, stream)

    def poll(self, handle) -> bool:
        return handle[0].query()

    def collect(self, handle) -> list:
        ev, outs, stream = handle
        ev.synchronize()
        res = []
        for o in outs:
            host = o.pop("host_radiance")
            res.append(({"radiance": host, "device": o}, None))
        return res
