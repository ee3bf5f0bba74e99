"""Benchmark: stereo Whitted ray tracing throughput on one MI355X.

One step = one stereo frame (both eyes, every ray of the Whitted tree: primary,
shadow and mirror rays) of the 3.4M-triangle terrain scene at 1920x1080 per eye,
reflection depth 4, 4 point lights.  Inputs are seeded and synthetic and are
resident in HBM (the scene is built once) before the timed region starts.

Prints one JSON line.  `value` is Mrays/s (all rays of the frame / device time
per frame); stereo frames/s is reported beside it, device-only and end to end
(including the pinned asynchronous readback of both eyes' radiance).  Frames are
rendered continuously with --frames-in-flight of them on their own streams (2 by
default); the time per frame with one frame in flight is reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mrays/s and stereo frames/s (1080p, 2M tris) at 1 GPU; p50/p99 latency served"
HBM_PEAK_GBS = 8000.0
# VALU: 256 CUs x 4 SIMDs x 16 lanes, one lane operation per lane per clock at 2.4 GHz (an FMA counts once;
# packed FP32 is not used by this build).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12

# Algorithmic work of the traversal: what the method has to compute per unit, however it is coded.
# A visit of a four-wide node is four ray-box slab tests; each is 6 plane distances (one FMA each, the ray
# origin pre-scaled by 1/d), 3 max and 3 min for the entry and exit distances (against tmin and tmax) and
# one compare: 13 lane operations per child box, 52 per visit.  A Moller-Trumbore triangle test is 38:
# T = o - v0 (3), P = d x e2 (6), det (3), 1/det (1), u (4), Q = T x e1 (6), v (4), t (4), the four
# barycentric checks with u + v (5) and the t range (2).
OPS_PER_NODE_VISIT = 52
OPS_PER_TRI_TEST = 38
# Algorithmic bytes (what the traversal reads and writes if nothing were cached): a visit reads the whole
# node record (64 B four-wide quantised, 128 B four-wide FP32), a triangle test its 48 B record.
NODE_VISIT_BYTES = {64: 64, 128: 128}  # node record size -> bytes one visit reads
TRI_BYTES = 48       # one triangle record test
CLOSEST_RAY_IO = 32 + 8   # ray in (origin+path, direction+exclude) + hit out (t, key)
ANY_RAY_IO = 32 + 1       # shadow record in + visibility byte out
COUNTER_SOURCES = ["paper_1702_01530_amd/csrc/render.hip", "paper_1702_01530_amd/csrc/lbvh.hip",
                   "paper_1702_01530_amd/csrc/rt_internal.h", "paper_1702_01530_amd/csrc/ploc_rule.h"]


def sources_sha256(sources) -> str:
    import hashlib
    h = hashlib.sha256()
    for src in sources:
        h.update(open(os.path.join(ROOT, src), "rb").read())
    return h.hexdigest()


def stored_counters(workload_name: str):
    """The traversal kernel's rocprofv3 counter figures committed under profiles/ (HBM bytes per launch,
    VALU instructions, lane utilisation), if the kernel sources are still the ones that were profiled
    (else None): counters are never carried over to a changed kernel."""
    path = os.path.join(ROOT, "profiles", f"k_trace_{workload_name}_counters.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    return t if sources_sha256(t["sources"]) == t["sources_sha256"] else None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name: str):
    import scenegen as sg
    if name == "terrain3.4M_1080p":
        return sg.make_terrain_3m()
    if name == "terrain3.4M_4k":
        s, c = sg.make_terrain_3m()
        return s, c.resized(3840, 2160)
    if name == "terrain212k_1080p":
        return sg.make_terrain_1080p()
    if name == "spheres8_256":
        return sg.make_spheres_scene()
    raise SystemExit(f"unknown workload {name}")


def cpu_threads() -> int:
    """Threads for the host oracle: the CPUs this process may run on, at most 16 (a GPU's share of the host)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail))


def cpu_baseline(scene, cam, rays_per_frame: int, target_s: float = 15.0):
    """The FP64 brute-force oracle as it stands, timed on the host on a seeded sample of the same frame's paths:
    with every thread of the process's CPU share (at most 16) and with one thread.  Returns the baseline
    record, and the oracle's result on the sample (for the parity check of the GPU frame)."""
    import numpy as np
    import oracle
    import scenegen as sg
    threads = cpu_threads()
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = None
    n = threads * 2
    while True:
        samples = sg.sample_paths(cam, n, seed=99)
        t0 = time.perf_counter()
        r = oracle.render(scene, cam, samples=samples, nthreads=threads)
        dt = time.perf_counter() - t0
        if dt >= target_s * 0.66 or n >= 2 * cam.width * cam.height:
            break
        n = int(min(2 * cam.width * cam.height, max(2 * n, n * target_s / max(dt, 1e-3))))
    rays = int(r["ray_counts"].sum())
    rate = rays / dt
    # one thread, on a smaller seeded sample of the same frame (a fifth of the time budget)
    n1 = max(4, int(n * (target_s / 5) / (dt * threads)))
    t0 = time.perf_counter()
    r1 = oracle.render(scene, cam, samples=sg.sample_paths(cam, n1, seed=98), nthreads=1)
    dt1 = time.perf_counter() - t0
    rays1 = int(r1["ray_counts"].sum())
    base = {"value": rate / 1e6, "unit": "Mrays/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} seeded paths of the same stereo frame ({rays} rays, FP64 brute force over all "
                      f"{scene.num_prims} primitives per ray, {dt:.1f} s on {threads} threads)",
            "seconds": dt, "paths": n, "rays": rays,
            "ray_primitive_tests_per_s": rays * scene.num_prims / dt,
            "host_nproc": os.cpu_count(), "host_cpus_available": avail,
            "one_thread": {"value": rays1 / dt1 / 1e6, "unit": "Mrays/s", "paths": n1, "rays": rays1,
                           "seconds": dt1},
            "frame_seconds": rays_per_frame / rate, "frame_seconds_is": "extrapolated from the sample's rate"}
    # the oracle's FP64 hierarchy mode, a fairer CPU baseline: the same answers from a tree over the triangles,
    # on a larger seeded sample that starts with the brute-force sample (checked identical on it).  The oracle
    # times its one-thread tree build and its tracing separately.
    nb = min(2 * cam.width * cam.height, 1 << 18)
    more = sg.sample_paths(cam, nb, seed=97)
    rb = oracle.render(scene, cam, samples=np.concatenate([samples, more]), nthreads=threads, accel="bvh")
    same = all(np.array_equal(rb[k][:len(samples)], r[k], equal_nan=k == "hit_cos")
               for k in ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state", "shadow_contrib", "path_t",
                         "hit_cos"))
    raysb = int(rb["ray_counts"].sum())
    trace_s, build_s = rb["seconds"]["trace"], rb["seconds"]["tree_build"]
    base["hierarchy_mode"] = {
        "value": raysb / trace_s / 1e6, "unit": "Mrays/s", "cores": threads, "paths": len(samples) + nb,
        "rays": raysb, "trace_seconds": trace_s, "tree_build_seconds": build_s,
        "identical_to_brute_force_on_sample": same,
        "frame_seconds": build_s + rays_per_frame * trace_s / raysb,
        "note": "FP64 median-split tree over the triangles, built on one thread; the trace rate excludes the build"}
    return base, r


def bench_batch(args):
    """Batched mode: 64 stereo pairs of mixed resolution over 8 resident scenes (1k-500k triangles),
    rendered as one batch (rt_render_batch) versus one rt_render_stereo launch sequence per pair."""
    import numpy as np
    import torch
    import scenegen as sg
    from paper_1702_01530_amd import rt
    from paper_1702_01530_amd.stereo import GpuScene, Workspace, alloc_outputs, render_batch, render_stereo
    dev = torch.device("cuda:0")
    scenes, spec = sg.make_batch_workload()
    gss = [GpuScene(s) for s in scenes]
    pairs = [(gss[k], cam) for k, cam in spec]
    paths = sum(2 * c.width * c.height for _, c in pairs)
    log(f"[batch] {len(pairs)} stereo pairs, {len(scenes)} scenes ({min(s.num_triangles for s in scenes)}-"
        f"{max(s.num_triangles for s in scenes)} triangles), {paths / 1e6:.1f}M paths")
    outs = [alloc_outputs(cam, gs.num_lights, dev, counts=(i == 0)) for i, (gs, cam) in enumerate(pairs)]
    ws_single = Workspace(max(rt.rt_render_workspace_size(rt.make_camera_struct(c), g.num_lights) for g, c in pairs))
    items = (rt.rt_batch_item * len(pairs))()
    for i, (g, c) in enumerate(pairs):
        items[i].scene, items[i].camera = g.handle, rt.make_camera_struct(c)
    ws_batch = Workspace(rt.rt_render_batch_workspace_size(items))
    log(f"[batch] workspaces: per-frame {ws_single.nbytes / 1e9:.2f} GB, batch {ws_batch.nbytes / 1e9:.2f} GB")
    outs[0]["ray_counts"].zero_()
    render_batch(pairs, outputs=outs, workspace=ws_batch)
    torch.cuda.synchronize()
    rays = int(outs[0]["ray_counts"][:3].sum())

    def per_frame():
        for (g, c), o in zip(pairs, outs):
            render_stereo(g, c, workspace=ws_single, outputs=o)

    def batched():
        render_batch(pairs, outputs=outs, workspace=ws_batch)

    from paper_1702_01530_amd.stereo import BatchGraph, autotune_batch
    stream = torch.cuda.current_stream()
    graph = BatchGraph(pairs, outs, ws_batch, stream=stream)

    def graphed():
        graph.launch(pairs, outs)

    res = {}
    for name, fn in (("per_frame", per_frame), ("batched", batched), ("graph", graphed)):
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
        for _ in range(args.steps):
            fn()
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / args.steps
        res[name] = {"ms_per_batch": ms, "stereo_fps": len(pairs) / (ms * 1e-3), "mrays_s": rays / (ms * 1e-3) / 1e6}
        log(f"[batch] {name}: {ms:.2f} ms per 64 pairs = {res[name]['stereo_fps']:.1f} stereo frames/s, "
            f"{res[name]['mrays_s']:.0f} Mrays/s")
    t0 = time.perf_counter()
    tuning, tuned_ms = autotune_batch(pairs, outs, ws_batch, repeats=1)
    log(f"[batch] autotune ({time.perf_counter() - t0:.1f} s): {tuning} -> {tuned_ms:.2f} ms per batch")
    graph.close()
    graph = BatchGraph(pairs, outs, ws_batch, stream=stream)  # recaptured with the tuned launch shape
    for name, fn in (("batched_tuned", batched), ("graph_tuned", graphed)):
        fn()
        torch.cuda.synchronize()
        t0e, t1e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0e.record()
        for _ in range(args.steps):
            fn()
        t1e.record()
        torch.cuda.synchronize()
        ms = t0e.elapsed_time(t1e) / args.steps
        res[name] = {"ms_per_batch": ms, "stereo_fps": len(pairs) / (ms * 1e-3), "mrays_s": rays / (ms * 1e-3) / 1e6}
        log(f"[batch] {name}: {ms:.2f} ms per 64 pairs = {res[name]['stereo_fps']:.1f} stereo frames/s")
    graph.close()
    best = min(("batched", "graph", "batched_tuned", "graph_tuned"), key=lambda k: res[k]["ms_per_batch"])
    out = {"metric": "stereo frames/s, batched vs per-frame (64 mixed pairs, 8 resident scenes)",
           "value": res[best]["stereo_fps"], "unit": "stereo frames/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": res[best]["ms_per_batch"], "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "batch64", "pairs": len(pairs), "scenes": len(scenes), "paths": paths,
                      "rays_per_batch": rays},
           "modes": res, "best_mode": best, "tuning": tuning,
           "speedup": res["per_frame"]["ms_per_batch"] / res[best]["ms_per_batch"]}
    for g in gss:
        g.close()
    print(json.dumps(out), flush=True)


def bench_serve(args):
    """Serving: Poisson arrivals over 8 resident scenes (10k-2M triangles), 640x480 to 3840x2160, depth 1-4.
    Continuous batching (3 in-flight batch slots, batches grouped by cost class) versus one request at a time
    and versus 3 slots with requests of any cost in one batch, on the same arrival trace."""
    import numpy as np
    import torch
    import scenegen as sg
    from paper_1702_01530_amd.serve import GpuRenderer, Request, Server, latency_stats
    from paper_1702_01530_amd.stereo import GpuScene
    scenes, trace = sg.make_serving_workload(n_requests=args.requests, rate_hz=args.rate)
    gss = {k: GpuScene(s) for k, s in enumerate(scenes)}
    log(f"[serve] {len(trace)} requests at {args.rate:.0f}/s over {len(scenes)} scenes "
        f"({min(s.num_triangles for s in scenes)}-{max(s.num_triangles for s in scenes)} triangles)")
    out = {}
    modes = (("continuous_batching", 3, 64, args.group_ratio), ("one_at_a_time", 1, 1, None),
             ("continuous_ungrouped", 3, 64, None))
    for name, slots, max_batch, group in modes:
        rend = GpuRenderer(gss, slots=slots, workspace_bytes=6 << 30)
        rend.prewarm(sorted({(c.width, c.height) for _, _, c in trace}), count=12)

        def consume(req):  # the client takes the image, the pinned buffer goes back to the pool
            if req.result is not None:
                rend.release(req.result["radiance"])
                req.result = None

        server = Server(rend, hbm_budget=48 << 30, max_batch_paths=1 << 25, max_batch=max_batch, on_complete=consume,
                        group_ratio=group)
        server.run([(0.0, Request(-1 - i, k, cam)) for i, (_, k, cam) in enumerate(trace[:4])])  # warm-up
        torch.cuda.synchronize()
        server = Server(rend, hbm_budget=48 << 30, max_batch_paths=1 << 25, max_batch=max_batch, on_complete=consume,
                        group_ratio=group)
        done = server.run([(t, Request(i, k, cam)) for i, (t, k, cam) in enumerate(trace)])
        st = latency_stats(done)
        st["batches"] = server.batches
        st["mean_batch"] = float(np.mean(server.batch_sizes)) if server.batch_sizes else 0.0
        st["slots"], st["group_ratio"] = slots, group
        out[name] = st
        log(f"[serve] {name}: p50 {st['p50_ms']:.1f} ms, p99 {st['p99_ms']:.1f} ms, "
            f"{st['stereo_fps']:.1f} stereo frames/s, {st['batches']} batches (mean {st['mean_batch']:.1f})")
        del rend, server
        torch.cuda.synchronize()
    res = {"metric": "p50/p99 latency and stereo frames/s served (Poisson arrivals)",
           "value": out["continuous_batching"]["stereo_fps"], "unit": "stereo frames/s", "n_gpus": 1,
           "steps": args.requests, "warmup": 4, "ms_per_step": 1e3 / out["continuous_batching"]["stereo_fps"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "serve", "requests": args.requests, "rate_hz": args.rate, "scenes": len(scenes),
                      "group_ratio": args.group_ratio},
           "p50_ms": out["continuous_batching"]["p50_ms"], "p99_ms": out["continuous_batching"]["p99_ms"],
           "modes": out}
    for g in gss.values():
        g.close()
    print(json.dumps(res), flush=True)


def bench_paper_shapes(args):
    """The shapes of the paper's experiments (Section 4, Figs 3-8) measured on this GPU: synthesis time
    against the number of objects and lights (brute force and LBVH), against the launch configuration,
    and the split of a frame into computation, transfer and other time."""
    import numpy as np
    import torch
    import scenegen as sg
    from paper_1702_01530_amd import rt
    from paper_1702_01530_amd.stereo import GpuScene, Workspace, alloc_outputs, render_stereo, Timer

    def time_frames(gs, cam, n=5, **kw):
        ws = Workspace.for_camera(cam, gs.num_lights)
        out = alloc_outputs(cam, gs.num_lights, torch.device("cuda:0"))
        render_stereo(gs, cam, workspace=ws, outputs=out, **kw)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            render_stereo(gs, cam, workspace=ws, outputs=out, **kw)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    res = {}
    # (1) objects: the first k of the five-polyhedra scene (Fig. 6) plus a sixth solid, 1 light, 256x256 stereo
    base, cam = sg.make_paper5_scene()
    counts = np.cumsum([0] + [f for _, f in base.info["solids"]])
    rows = []
    for k in range(1, 6):
        T = int(counts[k])
        sc = sg.Scene(name=f"paper{k}", seed=6, triangles=base.triangles[:T], tri_material=base.tri_material[:T],
                      spheres=base.spheres, sphere_material=base.sphere_material, planes=base.planes,
                      plane_material=base.plane_material, materials=base.materials, lights=base.lights,
                      ambient=base.ambient, background=base.background)
        row = {"objects": k, "triangles": T}
        for accel in ("none", "lbvh"):
            gs = GpuScene(sc, accel=accel)
            row[f"ms_{accel}"] = time_frames(gs, cam)
            gs.close()
        rows.append(row)
        log(f"[shapes] {k} objects ({T} tris): brute {row['ms_none']:.3f} ms, lbvh {row['ms_lbvh']:.3f} ms")
    res["objects"] = rows
    # (2) polygon count: terrain scenes from 2k to 800k triangles, brute force while it stays cheap
    rows = []
    for grid in (24, 48, 96, 192, 384, 640):
        sc, c2 = sg.make_small_terrain(seed=21, grid=grid, n_spheres=4, level=2, lights=1, depth=1)
        c2 = c2.resized(256, 256)
        row = {"triangles": sc.num_triangles}
        for accel in (("none", "lbvh") if sc.num_triangles <= 20000 else ("lbvh",)):
            gs = GpuScene(sc, accel=accel)
            row[f"ms_{accel}"] = time_frames(gs, c2, n=3 if accel == "none" else 5)
            gs.close()
        rows.append(row)
        log(f"[shapes] {sc.num_triangles} tris: " + ", ".join(f"{k} {v:.3f}" for k, v in row.items() if k != "triangles"))
    res["triangles"] = rows
    # (3) lights: 1..4 on the 3.4M-triangle scene at 1080p
    big, bcam = sg.make_terrain_3m()
    rows = []
    for L in (1, 2, 3, 4):
        gs = GpuScene(big.with_lights(big.lights[:L]))
        rows.append({"lights": L, "ms": time_frames(gs, bcam)})
        gs.close()
        log(f"[shapes] {L} lights: {rows[-1]['ms']:.3f} ms")
    res["lights"] = rows
    # (4) launch configuration ("network size"): traversal workgroups per CU
    gs = GpuScene(big)
    saved = rt.rt_get_tuning()
    rows = []
    for per_cu in (1, 2, 3, 4, 5, 6, 7):
        rt.rt_set_tuning(per_cu, saved["stream_blocks"], saved["max_pass_paths"])
        t = Timer()
        ws = Workspace.for_camera(bcam, gs.num_lights)
        out = alloc_outputs(bcam, gs.num_lights, torch.device("cuda:0"))
        render_stereo(gs, bcam, workspace=ws, outputs=out)
        torch.cuda.synchronize()
        for _ in range(3):
            render_stereo(gs, bcam, workspace=ws, outputs=out, timer=t.handle)
        st = t.read()
        rows.append({"blocks_per_cu": per_cu, "trace_ms": st["trace"][0] / 3, "frame_ms": sum(v[0] for v in st.values()) / 3})
        t.close()
        log(f"[shapes] {per_cu} blocks/CU: trace {rows[-1]['trace_ms']:.3f} ms")
    rt.rt_set_tuning(**saved)
    res["launch_config"] = rows
    # (5) stage split of one frame (Fig. 7): computation, transfer, other; sequential and overlapped readback
    ws = Workspace.for_camera(bcam, gs.num_lights)
    out = alloc_outputs(bcam, gs.num_lights, torch.device("cuda:0"), host=True)
    t = Timer()
    render_stereo(gs, bcam, workspace=ws, outputs=out)
    torch.cuda.synchronize()
    n = 5
    t0 = time.perf_counter()
    for _ in range(n):
        render_stereo(gs, bcam, workspace=ws, outputs=out, timer=t.handle)  # readback on the same stream
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / n
    st = t.read()
    comp = sum(st[k][0] for k in ("trace", "shade", "resolve")) / n
    xfer = st["readback"][0] / n
    res["stage_split"] = {"frame_ms_wall": wall, "compute_ms": comp, "transfer_ms": xfer,
                          "other_ms": max(0.0, wall - comp - xfer), "compute_share": comp / wall,
                          "transfer_share": xfer / wall}
    log(f"[shapes] stage split (sequential readback): compute {comp:.3f} ms, transfer {xfer:.3f} ms, wall {wall:.3f} ms")
    t.close()
    gs.close()
    print(json.dumps({"metric": "paper experiment shapes", "config": {"workload": "paper_shapes"}, **res}), flush=True)


def bench_builders(args):
    """The two tree builders on the benchmark scene: build time, node visits per ray, frame time."""
    import numpy as np
    import torch
    from paper_1702_01530_amd.stereo import GpuScene, Workspace, alloc_outputs, render_stereo
    scene, cam = workload("terrain3.4M_1080p")
    dev = torch.device("cuda")
    res = {"workload": "terrain3.4M_1080p", "builders": {}}
    for accel in ("ploc", "karras"):
        GpuScene(scene, accel=accel).close()  # first build pays one-time costs (code loading, allocation)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gs = GpuScene(scene, accel=accel)
        torch.cuda.synchronize()
        build_ms = (time.perf_counter() - t0) * 1e3
        ws = Workspace.for_camera(cam, gs.num_lights)
        out = alloc_outputs(cam, gs.num_lights, dev)
        render_stereo(gs, cam, count_work=True, workspace=ws, outputs=out)
        torch.cuda.synchronize()
        c = out["ray_counts"].cpu().numpy().astype(np.int64)
        for _ in range(3):
            render_stereo(gs, cam, workspace=ws, outputs=out)
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record()
        for _ in range(args.steps):
            render_stereo(gs, cam, workspace=ws, outputs=out)
        stop.record()
        torch.cuda.synchronize()
        info = gs.info()
        r = {"build_ms": build_ms, "ms_per_frame_one_in_flight": start.elapsed_time(stop) / args.steps,
             "closest_nodes_per_ray": float(c[3] / (c[0] + c[1])), "shadow_nodes_per_ray": float(c[5] / c[2]),
             "closest_tris_per_ray": float(c[4] / (c[0] + c[1])), "shadow_tris_per_ray": float(c[6] / c[2]),
             "bvh_depth": info["bvh_depth"], "nodes": info["num_nodes"]}
        res["builders"][accel] = r
        log(f"[builders] {accel}: build {build_ms:.1f} ms, {r['closest_nodes_per_ray']:.1f} / "
            f"{r['shadow_nodes_per_ray']:.1f} nodes per closest / shadow ray, {r['ms_per_frame_one_in_flight']:.3f} ms/frame")
        gs.close()
    print(json.dumps(res), flush=True)


def copy_peak_gbs(dev) -> float:
    """Device-to-device copy bandwidth (bytes read + written per second) of a 1 GiB buffer: the HBM rate a
    plain streaming kernel reaches here, beside the 8 TB/s datasheet peak."""
    import torch
    n = 1 << 30
    a = torch.empty(n, dtype=torch.uint8, device=dev)
    b = torch.empty(n, dtype=torch.uint8, device=dev)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 5
    del a, b
    return 2 * n / (ms * 1e-3) / 1e9


def summarize_counters(args):
    """Reads the rocprofv3 counter CSVs of the traversal kernel's runs and writes its per-launch figures:
    HBM bytes (FETCH_SIZE and WRITE_SIZE, scaled by what the same counters read for a 1 GiB copy), VALU
    wave instructions and lane utilisation.  The JSON carries a hash of the kernel sources."""
    import csv
    import glob
    import re
    if len(args.pmc_dirs) != 5:
        raise SystemExit("--pmc-dirs needs the fetch, write, copy-fetch, copy-write and SQ run directories")
    kre = re.compile(r"k_trace<false, false>")
    cre = re.compile(r"copyBuffer|copy_kernel|elementwise")

    def load(d, kernel_re):
        per = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                name = r.get("Kernel_Name", "")
                if not kernel_re.search(name):
                    continue
                key = (f, r.get("Dispatch_Id"))
                row = per.setdefault(key, {})
                row[r["Counter_Name"]] = row.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        if not per:
            raise SystemExit(f"no matching dispatches under {d}")
        return list(per.values())

    def mean(rows, c):
        return sum(r[c] for r in rows) / len(rows)

    fetch, write, cfetch, cwrite, sq = (load(d, kre if i in (0, 1, 4) else cre)
                                        for i, d in enumerate(args.pmc_dirs))
    copy_kib = (1 << 30) / 1024
    cf = max(r["FETCH_SIZE"] for r in cfetch)
    cw = max(r["WRITE_SIZE"] for r in cwrite)
    fs, ws = copy_kib / cf, copy_kib / cw
    f_kib, w_kib = mean(fetch, "FETCH_SIZE"), mean(write, "WRITE_SIZE")
    out = {"kernel": "k_trace<false, false>", "workload": "terrain3.4M_1080p", "launches_measured": len(fetch),
           "fetch_kib_per_launch_raw": f_kib, "write_kib_per_launch_raw": w_kib,
           "copy_fetch_kib_raw": cf, "copy_write_kib_raw": cw, "fetch_scale": fs, "write_scale": ws,
           "hbm_bytes_per_launch": (f_kib * fs + w_kib * ws) * 1024,
           "valu_wave_instr_per_launch": mean(sq, "SQ_INSTS_VALU"),
           "valu_lane_util": sum(r["SQ_THREAD_CYCLES_VALU"] for r in sq) /
                             (64 * sum(r["SQ_ACTIVE_INST_VALU"] for r in sq)),
           "sq_per_launch": {c: mean(sq, c) for c in sorted(sq[0])},
           "sources": COUNTER_SOURCES, "sources_sha256": sources_sha256(COUNTER_SOURCES)}
    with open(args.summarize_counters, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="terrain3.4M_1080p")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--requests", type=int, default=200, help="serving workload: number of requests")
    ap.add_argument("--rate", type=float, default=100.0, help="serving workload: Poisson arrival rate (1/s)")
    ap.add_argument("--group-ratio", type=float, default=4.0,
                    help="serving workload: a batch takes requests within this factor of its first request's cost")
    ap.add_argument("--no-end-to-end", action="store_true")
    ap.add_argument("--frames-in-flight", type=int, default=2,
                    help="frames rendered concurrently on their own streams (1: strictly one after another)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for scaling HBM traffic counters)")
    ap.add_argument("--dump-signature", default=None,
                    help="write the ray-tree signature of a seeded sample of the frame's paths to this .npz")
    ap.add_argument("--dump-paths", type=int, default=1 << 17)
    ap.add_argument("--dump-seed", type=int, default=17)
    ap.add_argument("--summarize-counters", default=None,
                    help="read rocprofv3 counter CSVs (--pmc-dirs) and write the traversal kernel's figures to "
                         "this JSON")
    ap.add_argument("--pmc-dirs", nargs="*", default=[],
                    help="with --summarize-counters: directories of the FETCH_SIZE, WRITE_SIZE, copy FETCH_SIZE, "
                         "copy WRITE_SIZE and SQ runs, in that order")
    args = ap.parse_args()

    if args.summarize_counters:
        return summarize_counters(args)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the render path has no multi-GPU "
                                   "mode (each GPU would render its own tiles with no exchange)", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1702_01530_amd import rt
    from paper_1702_01530_amd.stereo import GpuScene, Workspace, alloc_outputs, render_stereo, Timer

    assert torch.cuda.is_available(), "needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.copy_calibration:
        n = 1 << 30
        a = torch.empty(n, dtype=torch.uint8, device=dev)
        b = torch.empty(n, dtype=torch.uint8, device=dev)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": n, "copies": 3}))
        return

    rt.lib()
    if args.workload == "paper_shapes":
        return bench_paper_shapes(args)
    if args.workload == "builders":
        return bench_builders(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "batch64":
        with torch.cuda.stream(torch.cuda.Stream()):  # graph capture needs a stream other than the null stream
            return bench_batch(args)
    import scenegen
    scene, cam = workload(args.workload)
    log(f"[bench] workload {args.workload}: {scene.num_triangles} triangles, {cam.width}x{cam.height} per eye, "
        f"depth {cam.max_depth}, {scene.num_lights} lights")
    t0 = time.perf_counter()
    gs = GpuScene(scene)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    info = gs.info()
    log(f"[bench] scene built in {build_ms:.1f} ms (incl. upload), BVH depth {info['bvh_depth']}")

    ws = Workspace.for_camera(cam, gs.num_lights)
    out = alloc_outputs(cam, gs.num_lights, dev)

    # work counts for the algorithmic-byte figures (instrumented kernels, not timed)
    out["ray_counts"].zero_()
    render_stereo(gs, cam, count_work=True, workspace=ws, outputs=out)
    torch.cuda.synchronize()
    cnt = out["ray_counts"].cpu().numpy().astype(np.int64)
    if cnt[7] != 0:
        raise SystemExit("internal consistency check fired during the counting pass")
    rays = int(cnt[0] + cnt[1] + cnt[2])
    closest_rays, any_rays = int(cnt[0] + cnt[1]), int(cnt[2])
    node_visit = NODE_VISIT_BYTES.get(info["node_bytes"] // max(info["num_nodes"], 1), 0)  # 0: no BVH
    closest_bytes = node_visit * cnt[3] + TRI_BYTES * cnt[4] + CLOSEST_RAY_IO * closest_rays
    any_bytes = node_visit * cnt[5] + TRI_BYTES * cnt[6] + ANY_RAY_IO * any_rays
    log(f"[bench] rays/frame {rays} (primary {cnt[0]}, mirror {cnt[1]}, shadow {cnt[2]}); "
        f"closest: {cnt[3] / max(closest_rays, 1):.1f} nodes + {cnt[4] / max(closest_rays, 1):.1f} tris per ray; "
        f"shadow: {cnt[5] / max(any_rays, 1):.1f} nodes + {cnt[6] / max(any_rays, 1):.1f} tris per ray")

    # Frames are rendered round-robin over F streams (frames in flight), each with its own workspace
    # and outputs, the way a renderer runs continuously: the small, latency-bound launches at the end
    # of one frame's recursion overlap the next frame's work.  Every frame is rendered in full.
    F = max(1, args.frames_in_flight)
    streams = [torch.cuda.Stream() for _ in range(F)]
    wss = [ws] + [Workspace.for_camera(cam, gs.num_lights) for _ in range(F - 1)]
    outs_f = [out] + [alloc_outputs(cam, gs.num_lights, dev) for _ in range(F - 1)]

    def run_frames(n, nstreams, timer=None, per_frame=None):
        """Device milliseconds for n frames over the first nstreams streams (events bracket the run)."""
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(streams[0])
        for st in streams[1:nstreams]:
            st.wait_event(start)
        for i in range(n):
            k = i % nstreams
            if per_frame is not None:
                e0 = torch.cuda.Event(enable_timing=True)
                e0.record(streams[k])
            render_stereo(gs, cam, workspace=wss[k], outputs=outs_f[k], stream=streams[k], timer=timer)
            if per_frame is not None:
                e1 = torch.cuda.Event(enable_timing=True)
                e1.record(streams[k])
                per_frame.append((e0, e1))
        for st in streams[1:nstreams]:
            ev = torch.cuda.Event()
            ev.record(st)
            streams[0].wait_event(ev)
        stop.record(streams[0])
        torch.cuda.synchronize()
        return start.elapsed_time(stop)

    run_frames(args.warmup, F)
    log(f"[bench] warmup done ({args.warmup} frames)")
    single_ms = run_frames(args.steps, 1) / args.steps  # one stream, no timer: frames back to back
    log(f"[bench] one frame in flight: {single_ms:.3f} ms/frame")
    # isolated launches: the same frames one at a time with a HIP event pair around every launch, so each
    # kernel's duration is its own (the roofline figures use these)
    timer_iso = Timer()
    run_frames(args.steps, 1, timer=timer_iso.handle)
    iso = timer_iso.read()
    timer_iso.close()
    log(f"[bench] isolated launches: trace {iso['trace'][0] / args.steps:.3f} ms/frame over "
        f"{iso['trace'][1] // args.steps} launches, shade {iso['shade'][0] / args.steps:.3f}, "
        f"resolve {iso['resolve'][0] / args.steps:.3f}")

    # per-stage device time with F frames in flight (launches overlap): its own run, since the event pair
    # around every launch costs time of its own
    timer = Timer()
    run_frames(args.steps, F, timer=timer.handle)
    stages = timer.read()
    # the timed region: K frames, F in flight, no per-launch events
    frame_ms = []
    t_wall = time.perf_counter()
    total_ms = run_frames(args.steps, F, per_frame=frame_ms)
    wall_s = time.perf_counter() - t_wall
    per_frame = [a.elapsed_time(b) for a, b in frame_ms]
    # the frame time's distribution: with F frames in flight they complete in groups, so each sample is the
    # time between the completions of frames i - F and i, over F
    intervals = [frame_ms[i - F][1].elapsed_time(frame_ms[i][1]) / F for i in range(F, len(frame_ms))]
    ms_per_step = total_ms / args.steps
    log(f"[bench] timed {args.steps} frames, {F} in flight: {ms_per_step:.3f} ms/frame "
        f"(frame latency median {np.median(per_frame):.3f} ms), wall {wall_s:.2f} s")
    for k, (ms, n) in stages.items():
        if n:
            log(f"[bench]   {k:14s} {ms / args.steps:8.3f} ms/frame over {n // args.steps} launches/frame")

    # end to end: render + pinned async readback, each render stream with its own copy stream and
    # two host buffers, for both readback modes (hipMemcpyAsync, and the narrow copy kernel writing
    # through the pinned buffer)
    e2e = {}
    if not args.no_end_to_end:
        outs = [alloc_outputs(cam, gs.num_lights, dev, host=True, counts=False) for _ in range(2 * F)]
        copies = [torch.cuda.Stream() for _ in range(F)]
        e2e_frames = max(args.steps, 30)  # wall-clock timing: enough frames to average out host jitter

        def stream_frames(mode, n):
            done = []
            for i in range(n):
                k = i % F
                o = outs[i % (2 * F)]
                if i >= 2 * F:
                    done[i - 2 * F].synchronize()  # the host buffer's previous frame has been consumed
                render_stereo(gs, cam, workspace=wss[k], outputs=o, stream=streams[k], copy_stream=copies[k],
                              readback_kernel=(mode == "kernel"))
                ev = torch.cuda.Event()
                ev.record(copies[k])
                done.append(ev)
            torch.cuda.synchronize()

        for mode in ("memcpy", "kernel"):
            stream_frames(mode, 3 * F)  # warm-up: first use of the mode's copy path and the pinned pages
            t1 = time.perf_counter()
            stream_frames(mode, e2e_frames)
            e2e[mode] = (time.perf_counter() - t1) * 1e3 / e2e_frames
            log(f"[bench] end to end with pinned readback ({mode}): {e2e[mode]:.3f} ms/frame over {e2e_frames} frames")
        # display path: both eyes composed on the device into one RGBA8 red-cyan anaglyph (Section 3,
        # Fig. 2), and only that image crosses PCIe: 4 bytes per pixel instead of 24
        H, W = int(cam.height), int(cam.width)
        imgs = [torch.empty((H, W, 4), dtype=torch.uint8, device=dev) for _ in range(2 * F)]
        hosts = [torch.empty((H, W, 4), dtype=torch.uint8, pin_memory=True) for _ in range(2 * F)]

        def stream_composed(n):
            done = []
            for i in range(n):
                k, j = i % F, i % (2 * F)
                if i >= 2 * F:
                    done[i - 2 * F].synchronize()
                o = outs_f[k]
                render_stereo(gs, cam, workspace=wss[k], outputs=o, stream=streams[k])
                rt.rt_compose_stereo(o["radiance"][0].data_ptr(), o["radiance"][1].data_ptr(), W, H,
                                     rt.RT_COMPOSE_ANAGLYPH_RED_CYAN, 1.0, imgs[j].data_ptr(), streams[k].cuda_stream)
                ev = torch.cuda.Event()
                ev.record(streams[k])
                copies[k].wait_event(ev)
                with torch.cuda.stream(copies[k]):
                    hosts[j].copy_(imgs[j], non_blocking=True)
                ev2 = torch.cuda.Event()
                ev2.record(copies[k])
                done.append(ev2)
            torch.cuda.synchronize()

        stream_composed(3 * F)
        t1 = time.perf_counter()
        stream_composed(e2e_frames)
        e2e["anaglyph_rgba8"] = (time.perf_counter() - t1) * 1e3 / e2e_frames
        log(f"[bench] end to end with an RGBA8 anaglyph composed on the device and read back: "
            f"{e2e['anaglyph_rgba8']:.3f} ms/frame over {e2e_frames} frames")
    e2e_best = e2e.get("memcpy")  # the library's default readback

    # The dominant kernel is the fused traversal (closest-hit rays of depth d + shadow rays of depth d-1).
    # It is not bound by HBM: its scene (247 MB) sits in the Infinity Cache and the measured DRAM traffic is
    # a small fraction of the algorithmic bytes.  Its roofline is the VALU: algorithmic lane operations per
    # launch over the isolated launch time, against 39.3 T lane operations/s.
    iso_trace_ms, iso_launches = iso["trace"]
    launches_per_frame = iso_launches / args.steps
    avg_launch_ms = iso_trace_ms / iso_launches
    ops_frame = OPS_PER_NODE_VISIT * int(cnt[3] + cnt[5]) + OPS_PER_TRI_TEST * int(cnt[4] + cnt[6])
    ops_per_launch = ops_frame / launches_per_frame
    achieved = ops_per_launch / (avg_launch_ms * 1e-3) / 1e12
    bytes_per_launch = (closest_bytes + any_bytes) / launches_per_frame
    stored = stored_counters(args.workload)
    traffic = stored["hbm_bytes_per_launch"] if stored else None
    copy_gbs = copy_peak_gbs(dev)
    trace_s_frame = iso_trace_ms / args.steps * 1e-3
    valu = None
    if stored:
        wave_instr_frame = stored["valu_wave_instr_per_launch"] * launches_per_frame
        issue = wave_instr_frame * 4 / (1024 * 2.4e9) / trace_s_frame
        valu = {"source": "stored rocprofv3 counters (profiles/k_trace_%s_counters.json)" % args.workload,
                "wave_instr_per_frame": wave_instr_frame, "lane_util": stored["valu_lane_util"],
                "issue_frac": issue, "lane_ops_frac": issue * stored["valu_lane_util"],
                "lane_ops_per_node_visit": wave_instr_frame * 64 * stored["valu_lane_util"] / max(1, int(cnt[3] + cnt[5]))}
    roofline = {
        "bound": "alu", "kernel": "k_trace",
        "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tops/s", "frac": achieved / VALU_PEAK_TOPS,
        "traffic": traffic,
        "ops_per_launch": ops_per_launch, "ops_per_unit": {"node_visit": OPS_PER_NODE_VISIT,
                                                           "triangle_test": OPS_PER_TRI_TEST},
        "avg_launch_ms": avg_launch_ms, "launches_per_frame": launches_per_frame,
        "timing": "HIP events around each launch on its stream, frames one at a time (isolated launches)",
        "valu": valu,
        # the same algorithmic lane operations over the whole frame's device time (F frames in flight, so
        # shading, resolve and the latency-bound tails of the recursion are included)
        "whole_frame": {"achieved": ops_frame / (ms_per_step * 1e-3) / 1e12,
                        "frac": ops_frame / (ms_per_step * 1e-3) / 1e12 / VALU_PEAK_TOPS,
                        "trace_share_of_isolated_frame": iso_trace_ms / sum(v[0] for v in iso.values())},
        "memory": {"algorithmic_bytes_per_launch": bytes_per_launch, "node_visit_bytes": node_visit,
                   "algorithmic_gbs": bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9,
                   "dram_bytes_per_launch": traffic,
                   "dram_gbs": traffic / (avg_launch_ms * 1e-3) / 1e9 if traffic else None,
                   "dram_frac_of_peak": traffic / (avg_launch_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if traffic else None,
                   "hbm_peak_gbs": HBM_PEAK_GBS, "copy_peak_gbs": copy_gbs,
                   "note": "algorithmic bytes count every node visit as a fetch; most are served by LDS, L2 and "
                           "the Infinity Cache, so they are not quoted against the HBM peak"},
    }
    log(f"[bench] k_trace: {achieved:.2f} T algorithmic lane-ops/s = {achieved / VALU_PEAK_TOPS:.3f} of the VALU "
        f"peak; copy kernel {copy_gbs:.0f} GB/s")

    res = {
        "metric": METRIC,
        "value": rays / (ms_per_step * 1e-3) / 1e6,
        "unit": "Mrays/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": args.workload, "triangles": scene.num_triangles, "width": cam.width,
                   "height": cam.height, "eyes": 2, "max_depth": cam.max_depth, "lights": scene.num_lights,
                   "accel": info.get("builder_name", "ploc")},
        "stereo_fps": 1e3 / ms_per_step,
        "stereo_fps_end_to_end": (1e3 / e2e_best) if e2e_best else None,
        "ms_per_step_end_to_end": e2e_best,
        "ms_per_step_end_to_end_by_readback": e2e or None,
        "frames_in_flight": F,
        "environment": {"gpu": torch.cuda.get_device_name(dev),
                        "arch": getattr(torch.cuda.get_device_properties(dev), "gcnArchName", None),
                        "hip": torch.version.hip, "torch": torch.__version__, "host_nproc": os.cpu_count(),
                        "scene_seed": int(scene.seed), "scene_digest": scenegen.digest(scene, cam)},
        "ms_per_step_one_in_flight": single_ms,
        "frame_latency_ms_p50": float(np.median(per_frame)),
        "frame_ms": {"median": float(np.median(intervals)), "p10": float(np.percentile(intervals, 10)),
                     "p90": float(np.percentile(intervals, 90)), "n": len(intervals),
                     "is": "(completion of frame i - completion of frame i - F) / F, F frames in flight"}
        if intervals else None,
        "rays_per_frame": rays,
        "ray_counts": {"primary": int(cnt[0]), "mirror": int(cnt[1]), "shadow": int(cnt[2])},
        "stage_ms_per_frame": {k: v[0] / args.steps for k, v in stages.items() if v[1]},
        "stage_ms_per_frame_isolated": {k: v[0] / args.steps for k, v in iso.items() if v[1]},
        "work_per_frame": {"closest_node_visits": int(cnt[3]), "closest_tri_tests": int(cnt[4]),
                           "shadow_node_visits": int(cnt[5]), "shadow_tri_tests": int(cnt[6])},
        "build_ms": build_ms,
        "roofline": roofline,
    }
    need_ids = (not args.no_cpu_baseline) or args.dump_signature
    if need_ids:
        # one frame with ray-tree signatures; the kernels timed above write the same image
        out_ids = render_stereo(gs, cam, path_ids=True)
        plain = render_stereo(gs, cam)
        torch.cuda.synchronize()
        same = all(torch.equal(out_ids[k], plain[k]) for k in ("radiance", "hit_t", "hit_prim"))
        del plain
        from tests.parity import gpu_flat
        g_ids = gpu_flat(out_ids)
        del out_ids
        if args.dump_signature:
            import scenegen as sg
            samp = sg.sample_paths(cam, args.dump_paths, seed=args.dump_seed)
            np.savez(args.dump_signature, digest=sg.digest(scene, cam), samples=samp, workload=args.workload,
                     seed=args.dump_seed, **{k: g_ids[k][samp] for k in g_ids})
            log(f"[bench] wrote the signature of {len(samp)} sampled paths to {args.dump_signature}")
    if not args.no_cpu_baseline:
        log("[bench] timing the FP64 oracle on a host sample ...")
        res["cpu_baseline"], orc = cpu_baseline(scene, cam, rays)
        cb = res["cpu_baseline"]
        log(f"[bench] cpu baseline {cb['value']:.5f} Mrays/s on {cb['cores']} threads (host nproc "
            f"{cb['host_nproc']}), {cb['one_thread']['value']:.5f} Mrays/s on 1 thread; a full frame would take "
            f"{cb['frame_seconds']:.0f} s (extrapolated)")
        from tests.parity import compare
        pr = compare(g_ids, orc, allow_min_one=False, scene=scene, cam=cam)
        res["parity"] = {"n": pr["n"], "ties": pr["ties"], "tie_rate_upper95": pr["tie_rate_upper95"],
                         "uncertified": len(pr["uncertified"]), "certified_by_shift": len(pr["certified_by_shift"]),
                         "max_err": pr["max_err"], "max_rel_t_err": pr.get("max_rel_t_err"),
                         "max_t_offset": pr.get("max_t_offset"), "passed": pr["passed"],
                         "timed_kernels_equal": same,
                         "sample": "the cpu_baseline sample: GPU frame with ray-tree signatures vs the FP64 oracle"}
        log(f"[bench] parity on {pr['n']} paths: ties {pr['ties']} (95% bound {pr['tie_rate_upper95']:.2e}), "
            f"max radiance error {pr['max_err']:.2e}, timed kernels equal: {same}")
    timer.close()
    gs.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
