"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle."""
import math
import sys

import numpy as np
import pytest

import oracle
import scenegen as sg
from tests.helpers import make_scene, material, mono_camera, f32, oracle_sampled, coincident_scene, flat_scene, \
    corners_scene, nested_scene
from tests.parity import compare, compare_full, assert_parity, gpu_flat

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_01530_amd import rt
    rt.lib()
    return torch


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def render(torch, scene, cam, accel="ploc", **kw):
    from paper_1702_01530_amd.stereo import GpuScene, render_stereo
    gs = GpuScene(scene, accel=accel)
    out = render_stereo(gs, cam, path_ids=True, **kw)
    torch.cuda.synchronize()
    return gs, out


def check_parity(torch, scene, cam, samples=None, accel="ploc", **kw):
    say(f"[parity] {scene.name} {cam.width}x{cam.height} D={cam.max_depth} accel={accel} "
        f"samples={'all' if samples is None else len(samples)}")
    gs, out = render(torch, scene, cam, accel=accel)
    assert int(out["ray_counts"][7]) == 0, "internal consistency check fired"
    g = gpu_flat(out)
    orc = oracle.render(scene, cam) if samples is None else oracle_sampled(scene, cam, samples, say=say)
    res = compare(g, orc, scene=scene, cam=cam, **kw)
    say(f"[parity] ties={res['ties']} max_err={res['max_err']:.3g} t_err={res.get('max_rel_t_err', 0):.3g}")
    assert_parity(res)
    gs.close()
    return g, orc, res


def test_spheres_full_frame(torch_cuda):
    scene, cam = sg.make_spheres_scene()
    g, orc, res = check_parity(torch_cuda, scene, cam, allow_min_one=False)
    assert res["n"] == 2 * 256 * 256


def test_paper5_full_frame_lbvh_and_brute(torch_cuda):
    scene, cam = sg.make_paper5_scene()
    gl, _, _ = check_parity(torch_cuda, scene, cam)
    gb, _, _ = check_parity(torch_cuda, scene, cam, accel="none")
    for k in ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state"):
        assert np.array_equal(gl[k], gb[k]), k


@pytest.mark.parametrize("grid,spheres,level,lights,depth,size,accel", [
    (24, 4, 1, 2, 3, (96, 64), "ploc"),
    (40, 6, 2, 4, 4, (77, 45), "ploc"),   # ragged tiles on both axes
    (40, 6, 2, 4, 4, (77, 45), "karras"),
])
def test_small_terrain_full_frame(torch_cuda, grid, spheres, level, lights, depth, size, accel):
    scene, cam = sg.make_small_terrain(seed=11 + grid, grid=grid, n_spheres=spheres, level=level, lights=lights,
                                       depth=depth)
    cam = cam.resized(*size)
    g, orc, res = check_parity(torch_cuda, scene, cam, accel=accel)
    # the tree path and the brute-force path agree bitwise
    gs, ob = render(torch_cuda, scene, cam, accel=accel, brute_force=True)
    b = gpu_flat(ob)
    for k in ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state"):
        assert np.array_equal(g[k], b[k]), k
    # ray counts: every ray the oracle traced, the GPU traced (ties aside)
    counts = ob["ray_counts"].cpu().numpy()
    assert counts[0] == 2 * cam.width * cam.height
    assert abs(counts[1] - orc["ray_counts"][1]) <= res["ties"] * cam.max_depth
    assert abs(counts[2] - orc["ray_counts"][2]) <= res["ties"] * (cam.max_depth + 1) * scene.num_lights


def test_chunking_and_repeat_bitwise(torch_cuda):
    torch = torch_cuda
    from paper_1702_01530_amd import rt
    from paper_1702_01530_amd.stereo import GpuScene, Workspace, render_stereo
    scene, cam = sg.make_small_terrain(seed=5, grid=32, n_spheres=5, level=2, lights=3, depth=3)
    cam = cam.resized(200, 120)  # 2*25*15 tiles = 96000 paths: several minimum-size passes
    gs = GpuScene(scene)
    full = render_stereo(gs, cam, path_ids=True)
    ws_min = Workspace(rt.rt_render_workspace_min(scene.num_lights))
    small = render_stereo(gs, cam, path_ids=True, workspace=ws_min)
    again = render_stereo(gs, cam, path_ids=True)
    torch.cuda.synchronize()
    for k in ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state"):
        assert torch.equal(full[k], small[k]), k
        assert torch.equal(full[k], again[k]), k
    with pytest.raises(rt.RtError) as ei:
        render_stereo(gs, cam, workspace=Workspace(ws_min.nbytes - 4096))
    assert ei.value.status == rt.RT_ERR_BUFFER_TOO_SMALL
    gs.close()


@pytest.mark.parametrize("accel", ["ploc", "karras"])
def test_builds_and_renders_repeat_bitwise(torch_cuda, accel):
    """The build and the render are deterministic despite their atomics (refit flags, clustering rounds, work
    counters, queue appends): three builds of one scene store the same node and triangle bytes, and ten renders
    of a frame, with their rays taken from the queues in whatever order the waves arrive, write the same bytes."""
    torch = torch_cuda
    from paper_1702_01530_amd.stereo import GpuScene, render_stereo
    scene, cam = sg.make_small_terrain(seed=8, grid=64, n_spheres=6, level=2, lights=3, depth=4)
    cam = cam.resized(160, 96)
    stores = []
    for _ in range(3):
        gs = GpuScene(scene, accel=accel)
        info = gs.info()
        nbytes = -(-((scene.num_triangles - 1) * (info["node_bytes"] // info["num_nodes"])) // 256) * 256 \
            + 48 * scene.num_triangles
        torch.cuda.synchronize()
        stores.append(gs._storage[gs.storage_offset:gs.storage_offset + nbytes].cpu())
        gs.close()
    assert all(torch.equal(stores[0], x) for x in stores[1:])
    gs = GpuScene(scene, accel=accel)
    ref = render_stereo(gs, cam, path_ids=True)
    for _ in range(9):
        again = render_stereo(gs, cam, path_ids=True)
        torch.cuda.synchronize()
        for k in ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state", "ray_counts"):
            assert torch.equal(ref[k], again[k]), k
    gs.close()


def test_batch_equals_single_renders(torch_cuda):
    """A batch mixing scenes (with and without spheres/planes), resolutions, depths and light counts gives
    every item exactly its standalone render, with one pass and with many small passes."""
    torch = torch_cuda
    from paper_1702_01530_amd import rt
    from paper_1702_01530_amd.stereo import GpuScene, Workspace, render_batch, render_stereo
    s1, c1 = sg.make_small_terrain(seed=5, grid=20, n_spheres=3, level=1, lights=2, depth=3)
    s2, c2 = sg.make_spheres_scene()
    s3, c3 = sg.make_small_terrain(seed=9, grid=30, n_spheres=4, level=2, lights=4, depth=2)
    s4, c4 = sg.make_paper5_scene()
    g = [GpuScene(x) for x in (s1, s2, s3, s4)]
    pairs = [(g[0], c1.resized(40, 24)), (g[1], c2.resized(64, 48)), (g[2], c3.resized(77, 45)),
             (g[3], c4.resized(33, 17)), (g[0], c1.resized(96, 64).with_(max_depth=1)),
             (g[1], c2.resized(23, 71).with_(max_depth=0))]
    single = [render_stereo(gs, cam, path_ids=True) for gs, cam in pairs]
    batched = render_batch(pairs, path_ids=True)
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(single, batched)):
        for k in ("radiance", "hit_t", "hit_prim", "path_prims"):
            assert torch.equal(a[k], b[k]), (i, k)
        L = pairs[i][0].num_lights
        assert torch.equal(a["shadow_state"][..., :L], b["shadow_state"][..., :L]), i
    total = sum(int(o["ray_counts"][0]) for o in single)
    assert int(batched[0]["ray_counts"][0]) == total
    # every item of the batch against the oracle, full frame (the batch kernels find each ray's item and
    # scene per lane: this checks them against the definition, not only against single renders)
    scenes = {id(g[0]): s1, id(g[1]): s2, id(g[2]): s3, id(g[3]): s4}
    for i, (gs, cam) in enumerate(pairs):
        b = dict(batched[i])
        b["shadow_state"] = b["shadow_state"][..., :gs.num_lights]
        res = compare(gpu_flat(b), oracle.render(scenes[id(gs)], cam), scene=scenes[id(gs)], cam=cam)
        say(f"[batch] item {i}: {cam.width}x{cam.height} D={cam.max_depth} ties={res['ties']} "
            f"max_err={res['max_err']:.3g}")
        assert_parity(res)
    # a workspace a little above the minimum: passes that straddle item boundaries
    need_min = rt.rt_render_workspace_min(4) + 4096
    multi = render_batch(pairs, path_ids=True, workspace=Workspace(need_min))
    torch.cuda.synchronize()
    for i, (a, b) in enumerate(zip(single, multi)):
        for k in ("radiance", "hit_t", "hit_prim", "path_prims"):
            assert torch.equal(a[k], b[k]), (i, k, "small workspace")
    for x in g:
        x.close()


@pytest.mark.timeout(900)
def test_batch64_every_item_against_oracle(torch_cuda):
    """The benchmark's batched workload (64 stereo pairs of mixed sizes, baselines and depths over 8 resident
    scenes, 108M paths) rendered as one batch, and every path of every item compared with the oracle."""
    torch = torch_cuda
    from paper_1702_01530_amd.stereo import GpuScene, render_batch
    scenes, spec = sg.make_batch_workload()
    gss = [GpuScene(x) for x in scenes]
    pairs = [(gss[k], cam) for k, cam in spec]
    say(f"[batch64] {len(pairs)} pairs, {sum(2 * c.width * c.height for _, c in pairs)} paths")
    batched = render_batch(pairs, path_ids=True)
    torch.cuda.synchronize()
    n = ties = 0
    worst = 0.0
    for i, (k, cam) in enumerate(spec):
        b = dict(batched[i])
        b["shadow_state"] = b["shadow_state"][..., :gss[k].num_lights]
        g = gpu_flat(b)
        batched[i] = None
        res = compare_full(g, scenes[k], cam, say=lambda *a: None)
        say(f"[batch64] item {i}: scene {k} ({scenes[k].num_triangles} tris) {cam.width}x{cam.height} "
            f"D={cam.max_depth} ties={res['ties']} shift={len(res['certified_by_shift'])} max_err={res['max_err']:.3g}")
        assert_parity(res)
        n, ties, worst = n + res["n"], ties + res["ties"], max(worst, res["max_err"])
    say(f"[batch64] {n} paths, {ties} ties ({ties / n:.2e}), max radiance error {worst:.3g}")
    for x in gss:
        x.close()


def test_batch_graph_replays_match_eager(torch_cuda):
    """A captured batch replays bitwise like eager batches, with eager work and syncs between replays, and
    accepts new poses of the same shape; a different shape is refused."""
    torch = torch_cuda
    from paper_1702_01530_amd import rt
    from paper_1702_01530_amd.stereo import BatchGraph, GpuScene, Workspace, batch_items, batch_outputs, \
        render_batch, render_stereo
    s1, c1 = sg.make_small_terrain(seed=5, grid=20, n_spheres=3, level=1, lights=2, depth=3)
    s2, c2 = sg.make_spheres_scene()
    g1, g2 = GpuScene(s1), GpuScene(s2)
    pairs_a = [(g1, c1.resized(40, 24)), (g2, c2.resized(64, 48))]
    moved = c1.with_(center=np.float32(c1.center + np.array([0.3, 0.1, -0.2])), baseline=0.09)
    pairs_b = [(g1, moved.resized(40, 24)), (g2, c2.resized(64, 48).with_(baseline=0.03))]
    eager_a = render_batch(pairs_a, path_ids=True)
    eager_b = render_batch(pairs_b, path_ids=True)
    outs = batch_outputs(pairs_a, path_ids=True)
    ws = Workspace(rt.rt_render_batch_workspace_size(batch_items(pairs_a, outs)))
    stream = torch.cuda.Stream()
    graph = BatchGraph(pairs_a, outs, ws, path_ids=True, stream=stream)
    stream.synchronize()
    for rep, (pairs, eager) in enumerate([(pairs_a, eager_a), (pairs_b, eager_b), (pairs_a, eager_a),
                                          (pairs_b, eager_b)]):
        for o in outs:
            o["radiance"].fill_(-7.0)
        render_stereo(g2, c2.resized(16, 16))  # eager work between replays
        torch.cuda.synchronize()
        graph.launch(pairs, outs, stream=stream)
        stream.synchronize()
        for i in range(2):
            for k in ("radiance", "hit_t", "hit_prim", "path_prims"):
                assert torch.equal(outs[i][k], eager[i][k]), (rep, i, k)
    with pytest.raises(rt.RtError):
        graph.launch([(g1, c1.resized(48, 24)), (g2, c2.resized(64, 48))], outs, stream=stream)
    graph.close()
    g1.close()
    g2.close()


def test_tuning_does_not_change_results(torch_cuda):
    torch = torch_cuda
    from paper_1702_01530_amd import rt
    from paper_1702_01530_amd.stereo import GpuScene, Workspace, autotune_batch, batch_items, batch_outputs, \
        render_batch
    s1, c1 = sg.make_small_terrain(seed=8, grid=24, n_spheres=3, level=1, lights=2, depth=2)
    g1 = GpuScene(s1)
    pairs = [(g1, c1.resized(96, 64)), (g1, c1.resized(50, 30).with_(max_depth=1))]
    ref = render_batch(pairs)
    saved = rt.rt_get_tuning()
    try:
        for per_cu, passes in ((1, 4096), (3, 1 << 16), (0, 1 << 25)):
            rt.rt_set_tuning(per_cu, 64, passes)
            out = render_batch(pairs)
            torch.cuda.synchronize()
            for i in range(2):
                assert torch.equal(out[i]["radiance"], ref[i]["radiance"]), (per_cu, passes, i)
        outs = batch_outputs(pairs)
        ws = Workspace(rt.rt_render_batch_workspace_size(batch_items(pairs, outs)))
        best, ms = autotune_batch(pairs, outs, ws, repeats=1)
        assert ms > 0 and best["max_pass_paths"] >= 4096
        assert rt.rt_get_tuning() == best
        torch.cuda.synchronize()
        for i in range(2):
            assert torch.equal(outs[i]["radiance"], ref[i]["radiance"])
    finally:
        rt.rt_set_tuning(**saved)
    g1.close()


@pytest.mark.parametrize("group_ratio", [None, 2.0])
def test_served_results_equal_standalone_renders(torch_cuda, group_ratio):
    """Requests served in a mix (continuous batching over two in-flight slots, with and without cost-class
    grouping) give exactly the image each request gets when rendered alone."""
    torch = torch_cuda
    from paper_1702_01530_amd.serve import GpuRenderer, Request, Server, latency_stats
    from paper_1702_01530_amd.stereo import GpuScene, render_stereo
    s1, c1 = sg.make_small_terrain(seed=5, grid=20, n_spheres=3, level=1, lights=2, depth=3)
    s2, c2 = sg.make_spheres_scene()
    scenes = {"terrain": GpuScene(s1), "spheres": GpuScene(s2)}
    rend = GpuRenderer(scenes, slots=2, workspace_bytes=512 << 20)
    # the slots' workspaces come off the budget; 64 MiB are left for the requests' outputs
    server = Server(rend, hbm_budget=rend.reserved_bytes() + (64 << 20), max_batch_paths=1 << 16, max_batch=4,
                    group_ratio=group_ratio)
    specs = [("terrain", c1.resized(64, 40)), ("spheres", c2.resized(48, 48)), ("terrain", c1.resized(33, 17)),
             ("spheres", c2.resized(80, 60).with_(max_depth=0)), ("terrain", c1.resized(96, 64)),
             ("spheres", c2.resized(20, 90)), ("nope", c2), ("terrain", c1.with_(hfov_deg=200.0))]
    arrivals = [(0.0005 * i, Request(i, sid, cam)) for i, (sid, cam) in enumerate(specs)]
    done = {q.rid: q for q in server.run(arrivals, timeout_s=120)}
    assert done[6].error and done[7].error  # unknown scene, invalid camera: failed alone
    assert server.batches >= 2
    host_scenes = {"terrain": s1, "spheres": s2}
    for i, (sid, cam) in enumerate(specs[:6]):
        assert done[i].error is None, done[i].error
        alone = render_stereo(scenes[sid], cam, host=True)
        torch.cuda.synchronize()
        assert torch.equal(done[i].result["radiance"], alone["host_radiance"]), i
        # the served image against the oracle: it equals the request's standalone render with ray-tree
        # signatures byte for byte, and that render is compared with the oracle over the full frame
        sig = render_stereo(scenes[sid], cam, path_ids=True)
        torch.cuda.synchronize()
        assert torch.equal(done[i].result["radiance"], sig["radiance"].cpu()), i
        res = compare(gpu_flat(sig), oracle.render(host_scenes[sid], cam), scene=host_scenes[sid], cam=cam)
        say(f"[serve] request {i}: {cam.width}x{cam.height} ties={res['ties']} max_err={res['max_err']:.3g}")
        assert_parity(res)
    assert latency_stats(list(done.values()))["n"] == 6
    for g in scenes.values():
        g.close()


@pytest.mark.parametrize("mode", ["anaglyph", "side_by_side"])
def test_compose_matches_oracle(torch_cuda, mode):
    """Stereo-pair building on the device decides the same 8-bit codes as the oracle's definition."""
    torch = torch_cuda
    from paper_1702_01530_amd.stereo import GpuScene, compose, render_stereo
    scene, cam = sg.make_spheres_scene()
    cam = cam.resized(45, 31)
    gs = GpuScene(scene)
    out = render_stereo(gs, cam)
    for exposure in (1.0, 0.7, 3.0):
        img = compose(out, mode, exposure)
        torch.cuda.synchronize()
        rad = out["radiance"].cpu().numpy()
        ref = oracle.compose_stereo(rad[0], rad[1], mode, exposure)
        assert np.array_equal(img.cpu().numpy(), ref), (mode, exposure)
    gs.close()


def test_degenerate_scenes(torch_cuda):
    torch = torch_cuda
    bg = (0.25, 0.5, 0.75)
    cam = mono_camera(width=13, height=7, depth=2)
    # empty scene: every pixel is the background
    empty = make_scene(background=bg)
    gs, out = render(torch, empty, cam)
    assert torch.allclose(out["radiance"].cpu(), torch.tensor(bg, dtype=torch.float32).expand(2, 7, 13, 3))
    assert (out["hit_prim"].cpu() == -1).all()
    # a single triangle (a BVH that is one leaf), two triangles, no lights, 1x1 image, depth 0
    tri = [[-1, 0, 4], [1, 0, 4], [0, 2, 4]]
    for scene in (make_scene(tris=[tri], background=bg, ambient=(0.1, 0.2, 0.3)),
                  make_scene(tris=[tri, [[-3, 0, 6], [3, 0, 6], [0, 3, 6]]], lights=[[0, 5, 0, 1, 1, 1]],
                             materials=[material(kr=(0.5, 0.5, 0.5))], ambient=(0.05,) * 3)):
        for c in (cam, cam.resized(1, 1), cam.with_(max_depth=0)):
            check_parity(torch, scene, c, allow_min_one=False)


@pytest.mark.parametrize("accel", ["ploc", "karras"])
def test_coincident_and_zero_area_triangles(torch_cuda, accel):
    """Hundreds of copies of one triangle (equal Morton codes, equal boxes, exact ties in t that only the
    smaller id decides), zero-area triangles (collinear and point-like: never hit) and a mirror floor."""
    scene, cam = coincident_scene()
    g, orc, res = check_parity(torch_cuda, scene, cam, accel=accel, allow_min_one=False)
    ids = g["path_prims"].reshape(-1)
    assert (ids == 0).any() and (ids == 420).any()  # the front triangle and the floor are both seen
    assert not np.isin(ids, np.arange(1, 300)).any()  # a copy of the front triangle never beats copy 0
    assert not np.isin(ids, np.arange(300, 420)).any()  # zero-area triangles are never hit


def test_maximum_lights_and_depth(torch_cuda):
    """RT_MAX_LIGHTS point lights (eight shadow queues per depth) and RT_MAX_DEPTH mirror bounces: mirror
    planes on both sides and at the back keep most paths bouncing to the last depth."""
    import dataclasses
    from paper_1702_01530_amd import rt
    scene, cam = sg.make_small_terrain(seed=13, grid=20, n_spheres=5, level=1, lights=1, depth=3)
    L = 8
    assert rt.RT_MAX_LIGHTS == L and rt.RT_MAX_DEPTH == 8
    ang = np.linspace(0.0, 2.0 * np.pi, L, endpoint=False)
    lights = [[8 * np.cos(a), 5 + 2 * (k % 3), 8 + 8 * np.sin(a), 0.25, 0.2 + 0.02 * k, 0.15] for k, a in enumerate(ang)]
    scene = scene.with_lights(lights)
    M = scene.materials.shape[0]
    mirror = np.float32([[0.05, 0.05, 0.05, 0, 0, 0, 0.8, 0.8, 0.8, 16]])
    scene = dataclasses.replace(scene, planes=np.float32([[1, 0, 0, -9], [-1, 0, 0, -9], [0, 0, -1, -30]]),
                                plane_material=np.uint32([M, M, M]), materials=np.vstack([scene.materials, mirror]))
    cam = cam.resized(48, 32).with_(max_depth=8)
    g, orc, _ = check_parity(torch_cuda, scene, cam)
    assert (orc["path_prims"][:, 8] >= 0).sum() > 1000  # most paths bounce to the last depth


@pytest.mark.parametrize("accel", ["ploc", "karras"])
def test_flat_scene(torch_cuda, accel):
    """Every triangle in the plane y = 0 (boxes of zero height: the quantisation grid and the padding
    must still give every box a slab the rays can enter), a mirror stripe, grazing and axis-parallel
    rays."""
    scene, cam = flat_scene()
    check_parity(torch_cuda, scene, cam, accel=accel)


def test_headlight_lambert_closed_form_gpu(torch_cuda):
    """Sphere lit from the eye: radiance = rho I cos(theta) + ks I max(0, cos 2theta)^n (closed form)."""
    c = np.array([0.3, 0.9, 6.0])
    r = 1.3
    rho = np.array([0.7, 0.4, 0.2])
    I = np.array([0.9, 1.1, 0.5])
    eye = np.array([0.0, 1.0, 0.0])
    scene = make_scene(spheres=[list(c) + [r]], materials=[material(kd=rho, ks=(0.5, 0.5, 0.5))],
                       lights=[list(eye) + list(I)], background=(0.1, 0.2, 0.3))
    cam = mono_camera(center=eye, width=48, height=48, hfov=30.0)
    gs, out = render(torch_cuda, scene, cam)
    L = out["radiance"][0].cpu().numpy().astype(np.float64)
    cf, rf, rhof, If = f32(c), f32(r), f32(rho), f32(I)
    n = 0
    for j in range(48):
        for i in range(48):
            O, d = oracle.primary_ray(cam, 0, i, j)
            w = cf - O
            h = np.linalg.norm(w - (w @ d) * d)
            if abs(h - rf) < 1e-3:
                continue
            if h < rf:
                q = (h / rf) ** 2
                expect = rhof * If * math.sqrt(1 - q) + 0.5 * If * max(0.0, 1 - 2 * q) ** 32
                n += 1
            else:
                expect = f32([0.1, 0.2, 0.3])
            np.testing.assert_allclose(L[j, i], expect, atol=1e-4)
    assert n > 400
    assert np.array_equal(out["radiance"][0].cpu().numpy(), out["radiance"][1].cpu().numpy())


def test_pinned_readback_and_timer(torch_cuda):
    torch = torch_cuda
    from paper_1702_01530_amd.stereo import GpuScene, render_stereo, Timer
    scene, cam = sg.make_spheres_scene()
    gs = GpuScene(scene, accel="none")
    timer = Timer()
    copy = torch.cuda.Stream()
    out = render_stereo(gs, cam, host=True, copy_stream=copy, timer=timer.handle)
    copy.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(out["host_radiance"], out["radiance"].cpu())
    t = timer.read()
    assert t["trace"][1] == cam.max_depth + 2 and t["trace"][0] > 0
    assert t["shade"][1] == cam.max_depth + 1 and t["resolve"][1] == cam.max_depth + 1
    assert t["readback"][1] == 1 and t["readback"][0] > 0
    timer.close()
    gs.close()


@pytest.mark.parametrize("size", [(256, 256), (37, 23)])  # the second eye of 37x23 is not 16-byte aligned
@pytest.mark.parametrize("kernel", [False, True])
def test_readback_matches_device(torch_cuda, size, kernel):
    torch = torch_cuda
    from paper_1702_01530_amd.stereo import GpuScene, render_stereo
    scene, cam = sg.make_spheres_scene()
    cam = cam.resized(*size)
    gs = GpuScene(scene)
    copy = torch.cuda.Stream()
    out = render_stereo(gs, cam, host=True, copy_stream=copy, readback_kernel=kernel)
    copy.synchronize()
    torch.cuda.synchronize()
    assert torch.equal(out["host_radiance"], out["radiance"].cpu())
    gs.close()


def test_largest_coordinates_and_axis_parallel_rays(torch_cuda):
    """Two small triangles at opposite corners of the largest supported coordinates (+-1e12) stretch the
    tree's top nodes to the widest grid steps, over a mirrored pyramid on a floor near the origin, seen
    straight down: the rays of the centre column have d.x = 0 exactly and those of the centre row d.z = 0,
    so 1/d takes its clamped value against those steps.  (A triangle as large as the coordinates would test
    FP32 triangle arithmetic instead: its hit distance cancels from products near 1e36.)"""
    L = 1e12
    e = 1e7  # FP32 spacing near 1e12 is 65536
    tris = [[[-L, -L, -L], [-L + e, -L, -L], [-L, -L + e, -L]], [[L, L, L], [L - e, L, L], [L, L - e, L]],
            [[-5, 0, -5], [5, 0, -5], [5, 0, 5]], [[-5, 0, -5], [5, 0, 5], [-5, 0, 5]]]
    apex, base = [0.1, 1.2, 0.05], [[-0.6, 0, -0.5], [0.7, 0, -0.4], [0.5, 0, 0.6], [-0.4, 0, 0.5]]
    for i in range(4):
        tris.append([base[i], base[(i + 1) % 4], apex])
    mats = [material(kd=(0.6, 0.6, 0.5)), material(kd=(0.1, 0.1, 0.1), ks=(0.3, 0.3, 0.3), kr=(0.7, 0.7, 0.7))]
    scene = make_scene(tris=tris, tri_mat=[0, 0, 0, 0, 1, 1, 1, 1], spheres=[[1.5, 0.5, 1.0, 0.5]], sphere_mat=[1],
                       materials=mats, lights=[[3, 8, -2, 0.7, 0.7, 0.7], [-4, 6, 3, 0.4, 0.4, 0.4]])
    cam = mono_camera(center=(0.3, 6.0, 0.2), forward=(0, -1, 0), up=(0, 0, 1), width=33, height=25, depth=2,
                      hfov=50.0)
    g, orc, res = check_parity(torch_cuda, scene, cam)
    col = np.arange(cam.height) * cam.width + cam.width // 2
    assert (orc["hit_prim"][col] >= 2).all() and (g["hit_prim"][col] == orc["hit_prim"][col]).all()
    assert res["ties"] <= 1


def test_invalid_arguments_gpu(torch_cuda):
    torch = torch_cuda
    from paper_1702_01530_amd import rt
    from paper_1702_01530_amd.stereo import GpuScene
    scene, _ = sg.make_paper5_scene()
    bad = make_scene(tris=scene.triangles.copy())
    bad.triangles[3, 1, 2] = np.nan
    with pytest.raises(rt.RtError) as ei:
        GpuScene(bad)
    assert ei.value.status == rt.RT_ERR_INVALID_ARGUMENT and "finite" in str(ei.value)
    bad = make_scene(tris=scene.triangles.copy())
    bad.triangles[5, 2, 0] = -2e12  # finite but beyond the largest supported coordinate (1e12)
    with pytest.raises(rt.RtError) as ei:
        GpuScene(bad)
    assert ei.value.status == rt.RT_ERR_INVALID_ARGUMENT and "magnitude" in str(ei.value)
    bad = make_scene(tris=scene.triangles, tri_mat=np.full(scene.num_triangles, 7))
    with pytest.raises(rt.RtError) as ei:
        GpuScene(bad)
    assert "material" in str(ei.value)
    bad = make_scene(spheres=[[0, 0, 5, -1.0]])
    with pytest.raises(rt.RtError):
        GpuScene(bad)


def _decode_children(rec: np.ndarray):
    """Child boxes (lo [3,4], hi [3,4], FP64 exact values), references [4] and a validity mask [4] of one
    BVH4 node record (128-byte FP32 layout or 64-byte quantised layout)."""
    f, u = rec.view(np.float32), rec.view(np.uint32)
    if rec.nbytes == 128:
        lo = f[0:24].reshape(6, 4)[0::2].astype(np.float64)
        hi = f[0:24].reshape(6, 4)[1::2].astype(np.float64)
        refs = u[24:28].view(np.int32)
        valid = np.isfinite(lo).all(axis=0)
        return lo, hi, refs, valid
    assert rec.nbytes == 64
    p = f[0:3].astype(np.float64)
    step = np.array([f[3], f[14], f[15]], np.float64) / 2.0 ** 24  # the node stores 2^24 times the step
    assert np.all(np.frexp(step)[0] == 0.5)  # powers of two
    refs = u[4:8].view(np.int32)
    words = [(u[8], u[9]), (u[10], u[11]), (u[12], u[13])]
    qlo = np.array([[(int(w[0]) >> (8 * k)) & 0xFF for k in range(4)] for w in words], np.float64)
    qhi = np.array([[(int(w[1]) >> (8 * k)) & 0xFF for k in range(4)] for w in words], np.float64)
    valid = (qlo <= qhi).all(axis=0)
    return p[:, None] + qlo * step[:, None], p[:, None] + qhi * step[:, None], refs, valid


def _morton_keys(tris: np.ndarray) -> np.ndarray:
    """63-bit Morton codes of the triangles' box centroids, quantised to 2^21 cells per axis of the centroids'
    bounds, written out in FP32 numpy (each operation rounded once) and interleaved bit by bit (x highest)."""
    t = tris.astype(np.float32)
    lo, hi = t.min(axis=1), t.max(axis=1)
    c = np.float32(0.5) * lo + np.float32(0.5) * hi
    clo, chi = c.min(axis=0), c.max(axis=0)
    ext = chi - clo
    cells = np.float32(2 ** 21)
    with np.errstate(divide="ignore", invalid="ignore"):
        s = np.where(ext > 0, (c - clo) / ext * cells, np.float32(0.0)).astype(np.float32)
    q = np.clip(s, np.float32(0.0), cells - np.float32(1.0)).astype(np.uint64)
    key = np.zeros(len(t), np.uint64)
    for b in range(21):
        for a in range(3):
            key |= ((q[:, a] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + 2 - a)
    return key


def _record_ids(gs, T: int) -> np.ndarray:
    """Original triangle id of each of the built scene's triangle records, in storage order."""
    info = gs.info()
    rec_bytes = info["node_bytes"] // info["num_nodes"]
    raw = gs._storage[gs.storage_offset:].cpu().numpy()
    tris_off = -(-((T - 1) * rec_bytes) // 256) * 256
    return raw[tris_off:tris_off + 48 * T].view(np.int32).reshape(T, 12)[:, 3]


@pytest.mark.parametrize("accel", ["ploc", "karras"])
def test_records_follow_the_stable_sort_of_morton_codes(torch_cuda, accel):
    """Steps 3-4 of the build against their definitions: the triangle records are written in the order of a
    stable sort of the centroids' Morton codes, the order numpy's stable argsort gives for the same codes.
    The scenes have equal codes (duplicated triangles, whose original order must be kept) and an axis of zero
    centroid extent (every code's bits on it zero)."""
    from paper_1702_01530_amd.stereo import GpuScene
    scene, _ = sg.make_small_terrain(seed=21, grid=40, n_spheres=4, level=2)
    dup = np.concatenate([scene.triangles, scene.triangles[::7], scene.triangles[5:9]])
    flat, _ = flat_scene()
    for tris in (scene.triangles, dup, flat.triangles):
        case = make_scene(tris=tris)
        T = len(tris)
        keys = _morton_keys(case.triangles)
        gs = GpuScene(case, accel=accel)
        ids = _record_ids(gs, T)
        gs.close()
        assert np.array_equal(ids, np.argsort(keys, kind="stable")), T


@pytest.mark.parametrize("accel", ["ploc", "karras"])
def test_bvh_structure(torch_cuda, accel):
    """Reads the built tree back and walks it: every node is reached once, every triangle is in exactly
    one leaf, and every child's box (as the traversal sees it) contains the triangles under it."""
    import torch
    from paper_1702_01530_amd.stereo import GpuScene
    scene, _ = sg.make_small_terrain(seed=3, grid=48, n_spheres=8, level=2)
    gs = GpuScene(scene, accel=accel)
    info = gs.info()
    T = scene.num_triangles
    n_nodes = info["num_nodes"]
    rec_bytes = info["node_bytes"] // n_nodes
    # a 4-wide tree collapsed from the T-1 binary nodes: between (T-1)/3 and T-1 nodes
    assert (T - 1) / 3 <= n_nodes <= T - 1 and rec_bytes in (64, 128) and info["node_bytes"] == rec_bytes * n_nodes
    assert math.log(T, 4) <= info["bvh_depth"] <= 40
    lo, hi = scene.triangles.reshape(-1, 3).min(0), scene.triangles.reshape(-1, 3).max(0)
    assert np.array_equal(np.array(info["bounds_lo"], np.float32), lo)
    assert np.array_equal(np.array(info["bounds_hi"], np.float32), hi)

    torch.cuda.synchronize()
    raw = gs._storage[gs.storage_offset:].cpu().numpy()
    nodes = raw[:n_nodes * rec_bytes].reshape(n_nodes, rec_bytes)
    tris_off = -(-((T - 1) * rec_bytes) // 256) * 256
    rec_ids = raw[tris_off:tris_off + 48 * T].view(np.int32).reshape(T, 12)[:, 3]
    tri = scene.triangles.astype(np.float64)
    seen_nodes = np.zeros(n_nodes, np.int32)
    seen_tris = np.zeros(T, np.int32)
    # entries: (node, intersection of the boxes entered on the way down)
    stack = [(0, np.full(3, -np.inf), np.full(3, np.inf))]
    while stack:
        i, plo, phi = stack.pop()
        seen_nodes[i] += 1
        clo, chi, refs, valid = _decode_children(nodes[i])
        assert valid[0]
        for k in range(4):
            if not valid[k]:
                continue
            blo, bhi = np.maximum(plo, clo[:, k]), np.minimum(phi, chi[:, k])
            r = int(refs[k])
            if r >= 0:
                assert r < n_nodes
                stack.append((r, blo, bhi))
                continue
            code = ~r
            first, count = code >> 2, (code & 3) + 1
            assert first + count <= T
            for j in range(first, first + count):
                seen_tris[j] += 1
                v = tri[rec_ids[j]]
                assert np.all(v >= blo) and np.all(v <= bhi), (i, k, j)
    assert np.all(seen_nodes == 1) and np.all(seen_tris == 1)
    assert np.array_equal(np.sort(rec_ids), np.arange(T))
    gs.close()


@pytest.fixture(scope="module")
def terrain_212k():
    return sg.make_terrain_1080p()


@pytest.fixture(scope="module")
def terrain_3m():
    return sg.make_terrain_3m()


# Full-size parity.  The tie budget is 1e-4 of the paths with no minimum of one: at 16,384 sampled paths
# at most one tie passes, and no ties bound the tie rate at 1.8e-4 (95%, Clopper-Pearson).  The oracle
# tests every primitive for every query, so these take minutes of host time.
HEADLINE_PATHS = 16384


@pytest.mark.timeout(900)
@pytest.mark.parametrize("accel", ["ploc", "karras"])
def test_terrain212k_1080p_sampled(torch_cuda, terrain_212k, accel):
    scene, cam = terrain_212k
    samples = sg.sample_paths(cam, HEADLINE_PATHS, seed=21)
    _, _, res = check_parity(torch_cuda, scene, cam, samples=samples, accel=accel, allow_min_one=False)
    say(f"[parity] tie rate upper bound (95%): {res['tie_rate_upper95']:.3g}")


@pytest.mark.timeout(900)
def test_terrain3m_1080p_sampled(torch_cuda, terrain_3m):
    """The benchmark workload at its full size, in the launch configuration the benchmark times.  The
    kernels the benchmark times (no ray-tree signatures) give the same bytes as the checked render."""
    torch = torch_cuda
    from paper_1702_01530_amd.stereo import GpuScene, render_stereo
    scene, cam = terrain_3m
    samples = sg.sample_paths(cam, HEADLINE_PATHS, seed=31)
    say(f"[parity] {scene.name} {cam.width}x{cam.height} D={cam.max_depth} samples={len(samples)}")
    gs = GpuScene(scene)
    out = render_stereo(gs, cam, path_ids=True)
    plain = render_stereo(gs, cam)
    torch.cuda.synchronize()
    assert int(out["ray_counts"][7]) == 0, "internal consistency check fired"
    for k in ("radiance", "hit_t", "hit_prim"):
        assert torch.equal(out[k], plain[k]), k
    g = gpu_flat(out)
    del out, plain
    gs.close()
    res = compare(g, oracle_sampled(scene, cam, samples, say=say), allow_min_one=False, scene=scene, cam=cam)
    say(f"[parity] ties={res['ties']} max_err={res['max_err']:.3g} t_err={res.get('max_rel_t_err', 0):.3g} "
        f"tie rate upper bound (95%): {res['tie_rate_upper95']:.3g}")
    assert_parity(res)


@pytest.mark.timeout(900)
def test_terrain3m_4k_sampled(torch_cuda, terrain_3m):
    """The 3.4M-triangle scene at 3840x2160 per eye (the roofline configuration), sampled paths."""
    scene, cam = terrain_3m
    cam = cam.resized(3840, 2160)
    samples = sg.sample_paths(cam, 4096, seed=41)
    check_parity(torch_cuda, scene, cam, samples=samples, allow_min_one=False)


def _full_frame(torch, scene, cam):
    """Every path of a frame against the oracle (hierarchy mode, ties certified by brute force)."""
    from paper_1702_01530_amd.stereo import GpuScene, render_stereo
    say(f"[full frame] {scene.name} {cam.width}x{cam.height} D={cam.max_depth}: {2 * cam.width * cam.height} paths")
    gs = GpuScene(scene)
    out = render_stereo(gs, cam, path_ids=True)
    torch.cuda.synchronize()
    assert int(out["ray_counts"][7]) == 0, "internal consistency check fired"
    g = gpu_flat(out)
    del out
    gs.close()
    res = compare_full(g, scene, cam, say=say)
    say(f"[full frame] n={res['n']} ties={res['ties']} ({res['tie_rate']:.2e}; budget {res['tie_budget']:.0f}) "
        f"certified by brute force {res['certified_by_brute_force']}, by a shift {res['certified_by_shift']} "
        f"max_err={res['max_err']:.3g} t_err={res.get('max_rel_t_err', 0):.3g} along the ray, "
        f"{res.get('max_t_offset', 0):.3g} normal to the surface")
    assert_parity(res)
    return res


@pytest.mark.timeout(900)
def test_serving_scenes_full_frames(torch_cuda):
    """Every resident scene of the serving workload (eight scenes of 10k to 2M triangles, log-uniform), each
    seen from its first request's orbit pose at 640x480 per eye and depth 4: every path against the oracle."""
    scenes, reqs = sg.make_serving_workload(n_requests=64)
    for k, scene in enumerate(scenes):
        cam = next(c for _, j, c in reqs if j == k).resized(640, 480)
        cam = cam.__class__(**{**cam.__dict__, "max_depth": 4})
        res = _full_frame(torch_cuda, scene, cam)
        assert res["n"] == 2 * 640 * 480


@pytest.mark.timeout(900)
def test_terrain3m_1080p_full_frame(torch_cuda, terrain_3m):
    """The benchmark frame, every one of its 4,147,200 paths against the oracle."""
    _full_frame(torch_cuda, *terrain_3m)


@pytest.mark.timeout(900)
def test_terrain212k_1080p_full_frame(torch_cuda, terrain_212k):
    _full_frame(torch_cuda, *terrain_212k)


@pytest.mark.timeout(900)
def test_terrain3m_4k_full_frame(torch_cuda, terrain_3m):
    """The 4K frame of the 3.4M-triangle scene, all 16,588,800 paths."""
    scene, cam = terrain_3m
    _full_frame(torch_cuda, scene, cam.resized(3840, 2160))


def test_frames_in_flight_equal_single(torch_cuda, terrain_3m):
    """The benchmark's launch configuration: two frames rendered concurrently on their own streams and
    workspaces give the same bytes as one frame rendered alone."""
    torch = torch_cuda
    from paper_1702_01530_amd.stereo import GpuScene, Workspace, alloc_outputs, render_stereo
    scene, cam = terrain_3m
    gs = GpuScene(scene)
    ref = render_stereo(gs, cam, workspace=Workspace.for_camera(cam, gs.num_lights))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream() for _ in range(2)]
    wss = [Workspace.for_camera(cam, gs.num_lights) for _ in range(2)]
    outs = [alloc_outputs(cam, gs.num_lights, torch.device("cuda")) for _ in range(2)]
    for rep in range(2):
        for k in range(2):
            render_stereo(gs, cam, workspace=wss[k], outputs=outs[k], stream=streams[k])
        torch.cuda.synchronize()
        for k in range(2):
            for name in ("radiance", "hit_t", "hit_prim"):
                assert torch.equal(outs[k][name], ref[name]), (rep, k, name)
    gs.close()


@pytest.mark.parametrize("accel", ["ploc", "karras"])
def test_corner_boxes_and_grid_ties(torch_cuda, accel):
    """Clusters whose merges tie exactly: a box B = [0,2]^3 (one triangle cutting its corner), tiny
    triangles at B's low and high corners and a distant triangle, in that Morton order, so that every
    merge with B or between the corners has B's area; copies at other places; a grid of equal quads.
    The clustering rounds must still merge (a partner rule that broke mutual pairs here once refused
    the scene)."""
    scene, cam = corners_scene()
    g, _, _ = check_parity(torch_cuda, scene, cam, accel=accel, allow_min_one=False)
    _, ob = render(torch_cuda, scene, cam, accel=accel, brute_force=True)
    b = gpu_flat(ob)
    for k in ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state"):
        assert np.array_equal(g[k], b[k]), k


def test_deep_clustering_tree_falls_back_to_karras(torch_cuda):
    """Nested triangles of growing size (boxes [0, 1.2^k]^3) make the clustering tree a chain as deep as
    the input is long, too deep for the traversal stack: the build rebuilds with the Karras tree, says so,
    and the render matches the oracle and the brute-force path."""
    from paper_1702_01530_amd.stereo import GpuScene
    scene, cam = nested_scene()
    gs = GpuScene(scene, accel="ploc")
    info = gs.info()
    gs.close()
    say(f"[nested] builder={info['builder_name']} depth={info['bvh_depth']}")
    assert info["builder_name"] == "karras" and 3 * info["bvh_depth"] < 128
    g, _, _ = check_parity(torch_cuda, scene, cam, accel="ploc", allow_min_one=False)
    _, ob = render(torch_cuda, scene, cam, accel="ploc", brute_force=True)
    b = gpu_flat(ob)
    for k in ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state"):
        assert np.array_equal(g[k], b[k]), k
