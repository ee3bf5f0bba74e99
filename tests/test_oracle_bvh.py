"""The oracle's hierarchy mode (accel="bvh") against its brute-force mode: the same radiance, primary hit,
ray-tree signature and shadow contributions, byte for byte, on scenes built to break a tree (coincident and
zero-area triangles, boxes of zero height with grazing and axis-parallel rays, exactly tied merges, a chain of
nested boxes, spheres and planes beside triangles) and on a sample of the 212k-triangle terrain frame."""
import numpy as np
import pytest

import oracle
import scenegen as sg
from tests.helpers import coincident_scene, corners_scene, flat_scene, make_scene, material, mono_camera, \
    nested_scene

KEYS = ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state", "shadow_contrib", "path_t", "hit_cos",
        "ray_counts")


def _same(scene, cam, samples=None):
    a = oracle.render(scene, cam, samples=samples)
    b = oracle.render(scene, cam, samples=samples, accel="bvh")
    for k in KEYS:
        assert np.array_equal(a[k], b[k], equal_nan=k == "hit_cos"), k
    # the hierarchy computes no margins: NaN for every decision taken, +inf where no ray was spawned
    spawned = a["path_prims"] != -2
    assert np.isnan(b["hit_margin"][spawned]).all() and np.isinf(b["hit_margin"][~spawned]).all()
    return a


@pytest.mark.parametrize("make", [coincident_scene, flat_scene, corners_scene, nested_scene],
                         ids=["coincident", "flat", "corners", "nested"])
def test_bvh_equals_brute_force_on_degenerate_scenes(make):
    scene, cam = make()
    a = _same(scene, cam)
    assert (a["path_prims"] >= 0).any()


def test_bvh_equals_brute_force_on_a_terrain_with_spheres_and_planes():
    scene, cam = sg.make_small_terrain(seed=9, grid=30, n_spheres=4, level=2, lights=4, depth=4)
    planes = np.array([[0.0, 1.0, 0.0, -0.8], [1.0, 0.0, 0.0, 9.0]], np.float32)
    scene = scene.__class__(**{**scene.__dict__, "planes": planes, "plane_material": np.zeros(2, np.uint32)})
    _same(scene, cam.resized(80, 48))


def test_bvh_equals_brute_force_on_random_triangles():
    rng = np.random.default_rng(11)
    c = rng.uniform(-3, 3, (400, 1, 3)) + [0, 1.5, 6]
    tris = c + rng.normal(0, 0.4, (400, 3, 3))
    tris[::7, 2] = tris[::7, 0]  # some degenerate (a repeated vertex)
    scene = make_scene(tris=tris, tri_mat=(np.arange(400) % 3 == 0).astype(np.uint32),
                       lights=[[2, 6, 0, 1, 1, 1], [-3, 3, 2, 0.6, 0.6, 0.6]],
                       materials=[material(kd=(0.6, 0.5, 0.4), ks=(0.3, 0.3, 0.3)),
                                  material(kd=(0.1, 0.1, 0.1), kr=(0.7, 0.7, 0.7))], ambient=(0.05,) * 3)
    # looking straight along +z: the centre column and row are axis-parallel in x and y
    _same(scene, mono_camera(center=(0, 1.5, 0), width=41, height=31, depth=3, baseline=0.065, convergence=6.0))


def test_bvh_equals_brute_force_on_a_terrain212k_sample():
    scene, cam = sg.make_terrain_1080p()
    _same(scene, cam, samples=sg.sample_paths(cam, 1500, seed=23))


def test_bvh_finds_a_nearer_hit_in_a_box_entered_later():
    """A grid of small triangles just in front of a large slanted one whose box the rays enter first: the
    tree visits the large triangle's leaf first and must still reach the small ones, 0.01% nearer, rather
    than prune them."""
    tris = [[[-3.0, -3.0, 4.9995], [3.0, -3.0, 4.9995], [0.0, 3.0, 5.0015]]]  # z = 5.0005 at y = 0
    for i in range(8):
        for j in range(8):
            x, y = -0.8 + 0.2 * i, -0.8 + 0.2 * j
            tris.append([[x, y, 5.0], [x + 0.2, y, 5.0], [x, y + 0.2, 5.0]])
    scene = make_scene(tris=tris, lights=[[0, 3, 0, 1, 1, 1]], materials=[material(kd=(0.5, 0.6, 0.7))])
    cam = mono_camera(center=(0, 0, 0), width=24, height=24, hfov=18.0, depth=0)
    a = _same(scene, cam)
    near = (a["hit_prim"] >= 1).sum()
    assert near > 200 and (a["hit_prim"] == 0).sum() > 50  # small ones win where they are hit


def test_full_frame_comparison_takes_margins_from_brute_force():
    """tests.parity.compare_full on a stand-in GPU frame written from the oracle itself: no ties; a path
    changed to another primitive becomes a tie whose margin comes from the brute-force mode (here far from
    certifiable, so the comparison fails)."""
    from tests.parity import compare_full
    scene, cam = sg.make_small_terrain(seed=3, grid=16, n_spheres=2, level=1, lights=2, depth=2)
    cam = cam.resized(32, 24)
    orc = oracle.render(scene, cam)
    g = {k: orc[k].astype(np.float32) if k in ("radiance", "hit_t") else orc[k].copy()
         for k in ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state")}
    res = compare_full(g, scene, cam, say=lambda *a: None)
    assert res["ties"] == 0 and res["passed"] and res["certified_by_brute_force"] == 0
    row = int(np.nonzero(orc["path_prims"][:, 0] >= 0)[0][5])
    g["path_prims"][row, 0] = (g["path_prims"][row, 0] + 7) % scene.num_triangles
    res = compare_full(g, scene, cam, say=lambda *a: None)
    assert res["ties"] == 1 and res["certified_by_brute_force"] == 1 and not res["passed"]
    assert res["uncertified"] == [(row, float(orc["hit_margin"][row, 0]))]
