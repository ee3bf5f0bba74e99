"""The entry point that allocates nothing (rt_render_stereo_noalloc) against rt_render_stereo: two calls in a
row through the C ABI, the second with a smaller input, each bitwise equal to the workspace entry point."""
import sys

import pytest

import scenegen as sg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_01530_amd import rt
    rt.lib()
    return torch


def _noalloc(torch, gs, cam, path_ids, host=False):
    from paper_1702_01530_amd import rt
    from paper_1702_01530_amd.stereo import alloc_outputs, output_struct, stream_handle
    o = alloc_outputs(cam, gs.num_lights, gs.device, path_ids, host)
    for k in ("radiance", "hit_t"):
        o[k].fill_(-7.0)  # stale values must not survive
    flags = rt.RT_FLAG_PATH_IDS if path_ids else 0
    rt.rt_render_stereo_noalloc(gs.handle, rt.make_camera_struct(cam), output_struct(o), flags,
                                stream_handle(None), None)
    return o


def test_noalloc_equals_workspace_entry_point(torch_cuda):
    torch = torch_cuda
    from paper_1702_01530_amd import rt
    from paper_1702_01530_amd.stereo import GpuScene, render_stereo
    # first call: the 212k-triangle terrain at 1920x1080 per eye, depth 3, 2 lights -- far more paths than
    # one pass of the fixed scratch holds, so the frame takes several passes
    big_scene, big_cam = sg.make_terrain_1080p()
    # second call, right after: a smaller input (the tiny sphere scene, 256x256 per eye, 1 light)
    small_scene, small_cam = sg.make_spheres_scene()
    gb, gsm = GpuScene(big_scene), GpuScene(small_scene)
    for rep in range(2):
        for gs, cam, ids in ((gb, big_cam, rep == 0), (gsm, small_cam, True)):
            say(f"[noalloc] rep {rep}: {cam.width}x{cam.height} D={cam.max_depth} L={gs.num_lights} ids={ids}")
            got = _noalloc(torch, gs, cam, ids)
            ref = render_stereo(gs, cam, path_ids=ids)
            torch.cuda.synchronize()
            keys = ("radiance", "hit_t", "hit_prim") + (("path_prims", "shadow_state") if ids else ())
            for k in keys:
                assert torch.equal(got[k], ref[k]), (rep, cam.width, k)
    gb.close()
    gsm.close()


def test_noalloc_rejects_bad_arguments(torch_cuda):
    from paper_1702_01530_amd import rt
    from paper_1702_01530_amd.stereo import GpuScene, alloc_outputs, output_struct
    scene, cam = sg.make_spheres_scene()
    gs = GpuScene(scene)
    o = alloc_outputs(cam, gs.num_lights, gs.device)
    with pytest.raises(rt.RtError) as ei:
        rt.rt_render_stereo_noalloc(None, rt.make_camera_struct(cam), output_struct(o), 0, None, None)
    assert ei.value.status == rt.RT_ERR_INVALID_ARGUMENT
    with pytest.raises(rt.RtError) as ei:
        rt.rt_render_stereo_noalloc(gs.handle, rt.make_camera_struct(cam.with_(hfov_deg=200.0)), output_struct(o), 0,
                                    None, None)
    assert ei.value.status == rt.RT_ERR_INVALID_ARGUMENT
    with pytest.raises(rt.RtError) as ei:  # PATH_IDS without the signature outputs
        rt.rt_render_stereo_noalloc(gs.handle, rt.make_camera_struct(cam), output_struct(o), rt.RT_FLAG_PATH_IDS,
                                    None, None)
    assert ei.value.status == rt.RT_ERR_INVALID_ARGUMENT
    gs.close()


def test_noalloc_render_replays_in_a_graph(torch_cuda):
    """The use the entry point exists for: a render captured into a HIP graph (nothing is allocated while
    capturing) and replayed, with eager work and synchronisations between the replays; every replay gives the
    bytes of the eager render."""
    torch = torch_cuda
    from paper_1702_01530_amd import rt
    from paper_1702_01530_amd.stereo import GpuScene, alloc_outputs, output_struct, render_stereo
    scene, cam = sg.make_small_terrain(seed=5, grid=20, n_spheres=3, level=1, lights=2, depth=3)
    cam = cam.resized(96, 64)
    gs = GpuScene(scene)
    ref = render_stereo(gs, cam, path_ids=True)
    torch.cuda.synchronize()
    out = alloc_outputs(cam, gs.num_lights, gs.device, path_ids=True, counts=False)
    st, camst = output_struct(out), rt.make_camera_struct(cam)
    s = torch.cuda.Stream()
    # first call on the device outside the capture: it looks up the scratch and the launch grid
    rt.rt_render_stereo_noalloc(gs.handle, camst, st, rt.RT_FLAG_PATH_IDS, s.cuda_stream, None)
    s.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        rt.rt_render_stereo_noalloc(gs.handle, camst, st, rt.RT_FLAG_PATH_IDS, s.cuda_stream, None)
    other = sg.make_spheres_scene()
    g2 = GpuScene(other[0])
    for rep in range(3):
        for k in ("radiance", "hit_t"):
            out[k].fill_(-7.0)
        render_stereo(g2, other[1].resized(40, 24))  # eager work between replays
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        say(f"[noalloc graph] replay {rep}")
        for k in ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state"):
            assert torch.equal(out[k], ref[k]), (rep, k)
    del graph
    gs.close()
    g2.close()
