"""The oracle's shifted render (hit points moved along their rays) and the two parity rules that use the scene:
the backward-error certificate for ties and the hit-distance check taken normal to the hit surface.

Pins: a mirror floor in front of a wall, where moving the floor hit point by s along the primary ray shortens
the mirror ray to the wall by exactly s (the mirror keeps the ray's z component, so the reflected ray meets the
plane z = Z after (Z - P.z - s d.z) / d.z); a wall made of two triangles meeting along a horizontal edge at a
height the test sets, so that the shift that moves the mirror ray's hit across the edge is known in closed
form, on either side of the certificate's bound."""
import numpy as np
import pytest

import oracle
from tests.helpers import make_scene, material, mono_camera
from tests.parity import T_TOL, assert_parity, certify_by_shift, compare, first_divergence, CONTRIB_MIN

KEYS = ("radiance", "hit_t", "hit_prim", "path_prims", "shadow_state", "shadow_contrib", "path_t")
WALL_Z = 10.0


def _mirror_room(wall_tris=None):
    mats = [material(kd=(0.1, 0.1, 0.1), kr=(0.9, 0.9, 0.9)), material(kd=(0.6, 0.5, 0.4), ks=(0.2, 0.2, 0.2))]
    lights = [[1.0, 4.0, 2.0, 0.8, 0.8, 0.8], [-2.0, 3.0, 8.0, 0.5, 0.5, 0.5]]
    if wall_tris is None:
        return make_scene(planes=[[0, 1, 0, 0], [0, 0, 1, WALL_Z]], plane_mat=[0, 1], materials=mats, lights=lights)
    return make_scene(tris=wall_tris, tri_mat=[1] * len(wall_tris), planes=[[0, 1, 0, 0]], plane_mat=[0],
                      materials=mats, lights=lights)


def _camera(forward=(0.0, -0.25, 1.0), width=16, height=12):
    return mono_camera(center=(0.0, 1.0, 0.0), forward=forward, width=width, height=height, depth=2, hfov=40.0)


def _floor_to_wall_closed_form(cam, pid):
    """Primary ray, floor hit, mirror ray and its hit on the plane z = WALL_Z, written out for the mirror y = 0."""
    HW = cam.width * cam.height
    eye, px = divmod(pid, HW)
    row, col = divmod(px, cam.width)
    O, d = oracle.primary_ray(cam, eye, col, row)
    t0 = -O[1] / d[1]
    P = O + t0 * d
    r = np.array([d[0], -d[1], d[2]])
    t1 = (WALL_Z - P[2]) / r[2]
    return O, d, t0, P, r, t1, P + t1 * r


def test_zero_shift_is_the_plain_render_and_path_t_is_the_hit_distance():
    scene, cam = _mirror_room(), _camera()
    n = 2 * cam.width * cam.height
    for accel in ("brute", "bvh"):
        a = oracle.render(scene, cam, accel=accel)
        b = oracle.render(scene, cam, accel=accel, t_shift=np.zeros((n, cam.max_depth + 1)))
        for k in KEYS:
            assert np.array_equal(a[k], b[k], equal_nan=True), (accel, k)
        if accel == "brute":
            assert np.array_equal(a["hit_margin"], b["hit_margin"]) and np.array_equal(a["shadow_margin"],
                                                                                       b["shadow_margin"])
        assert np.array_equal(a["path_t"][:, 0], a["hit_t"])
        assert np.isinf(a["path_t"][a["path_prims"] < 0]).all()
        assert np.isfinite(a["path_t"][a["path_prims"] >= 0]).all()


def test_shifting_the_floor_hit_shortens_the_mirror_ray_by_the_shift():
    scene, cam = _mirror_room(), _camera()
    a = oracle.render(scene, cam)
    floor_wall = np.nonzero((a["path_prims"][:, 0] == 0) & (a["path_prims"][:, 1] == 1))[0]
    assert len(floor_wall) > 20
    for pid in floor_wall[::7]:
        O, d, t0, P, r, t1, Q = _floor_to_wall_closed_form(cam, int(pid))
        assert a["path_t"][pid, 0] == pytest.approx(t0, rel=1e-13)
        assert a["path_t"][pid, 1] == pytest.approx(t1, rel=1e-12)
        shifts = np.array([-3e-3, -1e-5, 1e-5, 3e-3])
        tab = np.zeros((len(shifts), cam.max_depth + 1))
        tab[:, 0] = shifts
        b = oracle.render(scene, cam, samples=[pid] * len(shifts), t_shift=tab)
        assert (b["path_prims"][:, :2] == [0, 1]).all()
        assert np.allclose(b["path_t"][:, 1], t1 - shifts, rtol=0, atol=1e-12)
        assert (b["path_t"][:, 0] == a["path_t"][pid, 0]).all()  # the recorded distance is the unshifted one


def test_shift_table_is_checked():
    scene, cam = _mirror_room(), _camera()
    with pytest.raises(ValueError):
        oracle.render(scene, cam, samples=[0, 1], t_shift=np.zeros((2, cam.max_depth)))
    with pytest.raises(ValueError):
        oracle.render(scene, cam, samples=[0], t_shift=np.full((1, cam.max_depth + 1), np.nan))


def _edge_wall(cam, pid, offset):
    """Two wall triangles meeting along y = y_e, with the mirror ray of path pid hitting `offset` above the edge."""
    O, d, t0, P, r, t1, Q = _floor_to_wall_closed_form(cam, pid)
    y_e = float(np.float32(Q[1] - offset))
    x = float(Q[0])
    upper = [[x - 5, y_e, WALL_Z], [x + 5, y_e, WALL_Z], [x, y_e + 5, WALL_Z]]
    lower = [[x - 5, y_e, WALL_Z], [x, y_e - 5, WALL_Z], [x + 5, y_e, WALL_Z]]
    scene = _mirror_room([upper, lower])
    # the mirror ray's hit moves down by 2 |d.y| per unit of shift (Q' = Q + s (d - r))
    flip = (Q[1] - y_e) / (2 * abs(d[1]))
    return scene, t0, flip


def _stand_in(scene, cam, pid, shift):
    """A stand-in for GPU outputs: the oracle's render in FP32, with path pid's floor hit moved by `shift`."""
    n = 2 * cam.width * cam.height
    tab = np.zeros((n, cam.max_depth + 1))
    tab[pid, 0] = shift
    r = oracle.render(scene, cam, t_shift=tab)
    return {"radiance": r["radiance"].astype(np.float32), "hit_t": r["hit_t"].astype(np.float32),
            "hit_prim": r["hit_prim"], "path_prims": r["path_prims"].copy(), "shadow_state": r["shadow_state"]}


@pytest.mark.parametrize("within", [0.5, 2.0])
def test_backward_error_certificate_on_a_wall_edge(within):
    cam = _camera()
    pid = cam.width * (cam.height - 2) + cam.width // 2
    scene0 = _mirror_room()
    assert list(oracle.render(scene0, cam, samples=[pid])["path_prims"][0, :2]) == [0, 1]
    _, _, t0, *_ = _floor_to_wall_closed_form(cam, pid)
    bound = T_TOL * max(1.0, t0)
    scene, t0, flip = _edge_wall(cam, pid, offset=within * bound * 2 * abs(oracle.primary_ray(cam, 0, cam.width // 2,
                                                                                               cam.height - 2)[1][1]))
    assert flip == pytest.approx(within * bound, rel=5e-2)  # y_e is rounded to FP32
    orc = oracle.render(scene, cam)
    assert list(orc["path_prims"][pid, :2]) == [2, 0]   # the floor (a plane: ids after the triangles), then
    g = _stand_in(scene, cam, pid, shift=1.2 * flip)    # the upper triangle, just above the edge
    assert g["path_prims"][pid, 1] == 1                 # moved across the edge
    # the near-edge margin certifies this tie on its own; leave it open to test the certificate itself
    orc["hit_margin"][pid, 1] = np.inf
    res = compare(g, orc, scene=scene, cam=cam)
    assert res["ties"] == 1 and res["tie_ids"] == [pid]
    if within < 1.0:
        assert list(res["certified_by_shift"]) == [pid] and not res["uncertified"]
        e, s = res["certified_by_shift"][pid]
        # the smallest shift on the grid past the crossing
        assert e == 0 and flip < s <= flip + bound / 16
        assert_parity(res)
    else:
        assert res["uncertified"] == [(pid, np.inf)] and not res["certified_by_shift"]
    # without the scene, the open margin leaves the tie uncertified
    assert compare(g, orc)["uncertified"] == [(pid, np.inf)]


def test_backward_error_certificate_wants_the_gpu_choice():
    """A tie whose GPU choice no shift within the bound produces (here: a primitive the ray never meets)."""
    cam = _camera()
    pid = cam.width * (cam.height - 2) + cam.width // 2
    scene, t0, flip = _edge_wall(cam, pid, offset=1e-6)
    orc = oracle.render(scene, cam)
    g = _stand_in(scene, cam, pid, shift=0.0)
    g["path_prims"][pid, 1] = 2           # the floor again: excluded for the mirror ray at any shift
    orc["hit_margin"][pid, 1] = np.inf
    rows = np.nonzero((g["path_prims"] != orc["path_prims"]).any(axis=1))[0]
    assert list(rows) == [pid]
    prim = g["path_prims"][rows] != orc["path_prims"][rows]
    sh = (g["shadow_state"][rows] != orc["shadow_state"][rows]) & (orc["shadow_contrib"][rows] > CONTRIB_MIN)
    todo = [(pid, first_divergence(prim[0], sh[0]))]
    assert todo[0][1][:2] == ("hit", 1)
    assert certify_by_shift(g, orc, orc["samples"], todo, scene, cam) == {}
    # the same tie with the GPU's real choice across the edge is certified by a shift
    g2 = _stand_in(scene, cam, pid, shift=2 * flip + 1e-7)
    assert g2["path_prims"][pid, 1] == 1
    assert pid in certify_by_shift(g2, orc, orc["samples"], todo, scene, cam)


def test_hit_distance_is_held_normal_to_the_surface():
    # nearly level rays meet the floor at grazing incidence; steep ones head on
    cam = _camera(forward=(0.0, -0.1, 1.0), width=24, height=40)
    scene = make_scene(planes=[[0, 1, 0, 0]], materials=[material()])
    orc = oracle.render(scene, cam)
    floor = np.nonzero(orc["hit_prim"] == 0)[0]
    cosines = np.abs([_floor_to_wall_closed_form(cam, int(p))[1][1] for p in floor])
    # the oracle's cosine at the primary hit is |d.y| for the floor y = 0; NaN where the ray misses
    assert np.allclose(orc["hit_cos"][floor], cosines, rtol=1e-14, atol=0)
    assert np.isnan(orc["hit_cos"][orc["hit_prim"] < 0]).all() and (orc["hit_prim"] < 0).any()
    graze, steep = int(floor[np.argmin(cosines)]), int(floor[np.argmax(cosines)])
    assert cosines.min() < 0.05 and cosines.max() > 0.2
    g = _stand_in(scene, cam, 0, 0.0)
    g["hit_t"][graze] = np.float32(orc["hit_t"][graze] * (1 + 5e-5))
    res = compare(g, orc)
    assert res["max_rel_t_err"] > 4e-5 and res["max_t_offset"] <= T_TOL
    assert_parity(res)
    without = {k: v for k, v in orc.items() if k != "hit_cos"}   # along the ray only
    with pytest.raises(AssertionError):
        assert_parity(compare(g, without))
    g["hit_t"][steep] = np.float32(orc["hit_t"][steep] * (1 + 5e-5))
    res = compare(g, orc)
    assert res["max_t_offset"] > T_TOL and not res["passed"]
