"""Pins of the oracle's decision margins, shading terms and triangle normals.

The parity gate excuses a GPU/oracle disagreement only when the oracle's margin at the first
divergent decision is small, and ignores a shadow decision whose oracle contribution is small.  So
each margin and contribution is pinned here against a value reached by another route: signed
distances to a triangle's edge lines instead of Cramer's rule, the perpendicular distance of a
sphere's centre from the ray line, hand-computed Phong terms on rays whose geometry is exact, and a
plane equation in place of a cross product.  A dropped term, a wrong sign or index, or a transposed
operand in any of them fails one of these tests.
"""
import math

import numpy as np
import pytest

import oracle
from tests.helpers import f32, make_scene, material, mono_camera


def unit(v):
    v = np.asarray(v, np.float64)
    return v / np.linalg.norm(v)


# ---------------------------------------------------------------------------------------------
# Primitive margins
# ---------------------------------------------------------------------------------------------

def _edge_ratio(P, a, b, c, n):
    """Signed distance of P from the line through a and b (positive towards c), over the distance of c."""
    m = np.cross(n, b - a)
    m /= np.linalg.norm(m)
    if (c - a) @ m < 0:
        m = -m
    return ((P - a) @ m) / ((c - a) @ m)


def test_triangle_margin_is_edge_ratio_times_sine():
    """margin = min over edges of (distance of the hit point from the edge line / the opposite vertex's
    altitude) x |sin| of the ray's angle to the plane, for points inside and outside the triangle."""
    rng = np.random.default_rng(21)
    n_in = n_out = 0
    for _ in range(2000):
        v0, v1, v2 = rng.uniform(-2, 2, (3, 3))
        n = np.cross(v1 - v0, v2 - v0)
        if np.linalg.norm(n) < 0.2:
            continue
        n /= np.linalg.norm(n)
        w = rng.uniform(-0.3, 1.0, 3)
        w /= w.sum()
        P = w[0] * v0 + w[1] * v1 + w[2] * v2       # a point of the plane, inside or outside
        d = rng.normal(size=3) * rng.uniform(0.2, 3.0)  # not unit on purpose
        if abs(unit(d) @ n) < 0.05:
            continue
        O = P - rng.uniform(0.5, 4.0) * d
        ratios = [_edge_ratio(P, v1, v2, v0, n), _edge_ratio(P, v2, v0, v1, n), _edge_ratio(P, v0, v1, v2, n)]
        expect = min(ratios) * abs(unit(d) @ n)
        hit, t, u, v, m = oracle.intersect_triangle(O, d, v0, v1, v2, with_margin=True)
        assert m == pytest.approx(expect, rel=1e-8, abs=1e-12)
        assert hit == (min(ratios) >= 0)
        n_in += hit
        n_out += not hit
    assert n_in > 200 and n_out > 200


@pytest.mark.parametrize("delta", [0.02, 1e-3, 1e-6, -1e-6, -1e-3])
@pytest.mark.parametrize("theta_deg", [90.0, 30.0, 5.0])
def test_triangle_margin_near_an_edge(delta, theta_deg):
    """A ray at barycentric distance delta from an edge (unit altitude) at angle theta to the plane:
    margin = delta sin(theta)."""
    v0, v1, v2 = np.array([0.0, 0, 2]), np.array([1.0, 0, 2]), np.array([0.0, 1, 2])
    P = np.array([0.4, delta, 2.0])  # distance delta from the edge v0-v1 (y = 0), altitude 1
    th = math.radians(theta_deg)
    d = np.array([math.cos(th) * 0.6, math.cos(th) * 0.8, math.sin(th)])
    O = P - 5.0 * d
    hit, t, u, v, m = oracle.intersect_triangle(O, d, v0, v1, v2, with_margin=True)
    assert m == pytest.approx(delta * math.sin(th), rel=1e-9, abs=1e-15)
    assert hit == (delta >= 0)
    if hit:
        assert t == pytest.approx(5.0, rel=1e-12)


def test_sphere_margin_is_one_minus_h_over_r_squared():
    """disc / r^2 = 1 - (h/r)^2 with h the distance of the centre from the ray line; on a miss t is
    the closest approach."""
    rng = np.random.default_rng(22)
    for _ in range(500):
        c = rng.uniform(-3, 3, 3)
        r = rng.uniform(0.2, 2.0)
        d = unit(rng.normal(size=3))
        side = unit(np.cross(d, rng.normal(size=3)))
        h = r * rng.uniform(0.0, 2.0)
        s = rng.uniform(1.0, 8.0)
        O = c + h * side - s * d  # the ray passes the centre at distance h, s units ahead
        hit, t, m = oracle.intersect_sphere(O, d, c, r, with_margin=True)
        w = c - O
        h_line = np.linalg.norm(np.cross(w, d))  # the distance by a cross product
        assert h_line == pytest.approx(h, rel=1e-9, abs=1e-12)
        assert m == pytest.approx(1.0 - (h / r) ** 2, rel=1e-8, abs=1e-12)
        assert hit == (h <= r or np.linalg.norm(O - c) < r)
        if not hit:
            ok, t_any = oracle.intersect_sphere(O, d, c, r, tmax=np.inf)
            assert not ok
    # a near miss and a near hit at relative clearance 1e-3
    d = np.array([0.0, 0.0, 1.0])
    for h, expect_hit in ((1.001, False), (0.999, True)):
        hit, t, m = oracle.intersect_sphere([h * 0.5, 0, 0], d, [0, 0, 5], 0.5, with_margin=True)
        assert hit == expect_hit and m == pytest.approx(1 - h * h, rel=1e-9)


@pytest.mark.parametrize("theta_deg", [90.0, 45.0, 3.0, 0.01])
def test_plane_margin_is_sine_of_grazing_angle(theta_deg):
    th = math.radians(theta_deg)
    n = unit([1.0, 2.0, -2.0])
    e = unit(np.cross(n, [0.3, 1.0, 0.2]))  # in the plane
    d = 2.5 * (math.cos(th) * e - math.sin(th) * n)  # not unit
    O = 3.0 * n + np.array([0.1, 0.2, 0.3])
    hit, t, m = oracle.intersect_plane(O, d, n * 3.0, 0.0, with_margin=True)  # scaled normal: same plane
    assert m == pytest.approx(math.sin(th), rel=1e-9)
    assert hit


# ---------------------------------------------------------------------------------------------
# Closest-hit decision margins
# ---------------------------------------------------------------------------------------------

def _closest(scene, O, d, tmin=0.0, exclude=None):
    t, p, m = oracle.closest_hits(scene, np.asarray([O], float), np.asarray([d], float), tmin=tmin,
                                  exclude=None if exclude is None else [exclude])
    return float(t[0]), int(p[0]), float(m[0])


def test_closest_margin_relative_t_gap():
    """Two spheres on the ray at known depths: the winner's margin is (t2 - t1) / t1."""
    scene = make_scene(spheres=[[0, 0, 5, 1], [0, 0, 9, 2]])
    t, p, m = _closest(scene, [0, 0, 0], [0, 0, 1])
    assert (p, t) == (0, 4.0)
    assert m == pytest.approx((7.0 - 4.0) / 4.0, rel=1e-12)
    # swapping the ids does not change the margin; the nearer sphere still wins
    scene = make_scene(spheres=[[0, 0, 9, 2], [0, 0, 5, 1]])
    t, p, m = _closest(scene, [0, 0, 0], [0, 0, 1])
    assert (p, t) == (1, 4.0) and m == pytest.approx(0.75, rel=1e-12)


def test_closest_margin_near_missed_sphere_in_front():
    """A sphere the ray misses by a relative clearance of 1e-3, in front of the winner, sets the margin
    to |1 - (h/r)^2|; the same sphere behind the winner does not."""
    h = f32(0.5005)
    front = make_scene(spheres=[[0, 0, 5, 1], [0, 0, 9, 2], [0.5005, 0, 3.0, 0.5]])
    t, p, m = _closest(front, [0, 0, 0], [0, 0, 1])
    assert p == 0 and m == pytest.approx(abs(1 - (h / 0.5) ** 2), rel=1e-9)
    behind = make_scene(spheres=[[0, 0, 5, 1], [0, 0, 9, 2], [0.5005, 0, 4.5, 0.5]])
    t, p, m = _closest(behind, [0, 0, 0], [0, 0, 1])
    assert p == 0 and m == pytest.approx(0.75, rel=1e-12)
    # just inside: the small sphere is hit first, and its own inside margin is the decision's
    inside = make_scene(spheres=[[0, 0, 5, 1], [0, 0, 9, 2], [0.4995, 0, 3.0, 0.5]])
    t, p, m = _closest(inside, [0, 0, 0], [0, 0, 1])
    hi = f32(0.4995)
    assert p == 2 and m == pytest.approx(1 - (hi / 0.5) ** 2, rel=1e-9)


@pytest.mark.parametrize("delta", [2e-3, -2e-3])
def test_closest_margin_triangle_edge(delta):
    """The winner (delta > 0) or a near-missed triangle in front of a plane (delta < 0) passes at
    barycentric distance |delta| from an edge at 30 degrees to its plane: margin |delta| sin 30."""
    tri = [[0.0, 0, 2], [1.0, 0, 2], [0.0, 1, 2]]
    scene = make_scene(tris=[tri], planes=[[0, 0, 1, 6.0]])
    P = np.array([0.4, delta, 2.0])
    d = np.array([math.cos(math.pi / 6) * 0.6, math.cos(math.pi / 6) * 0.8, 0.5])
    t, p, m = _closest(scene, P - 1.0 * d, d)
    assert p == (0 if delta > 0 else 1)
    assert m == pytest.approx(abs(delta) * 0.5, rel=1e-6)


def test_closest_margin_near_tmin_and_exact_ties():
    """A secondary ray whose candidate lies just past tmin gets the relative distance to tmin (near-miss
    margins of 1e-2 and more are not recorded); two coincident triangles tie exactly (margin 0, smaller
    id wins, the excluded one gives way)."""
    dist = f32(1.0005e-4)
    scene = make_scene(planes=[[0, 0, 1, 1.0005e-4]])
    t, p, m = _closest(scene, [0, 0, 0], [0, 0, 1], tmin=1e-4)
    assert p == 0 and t == dist
    assert m == pytest.approx((dist - 1e-4) / 1e-4, rel=1e-9)
    scene = make_scene(planes=[[0, 0, 1, 1.05e-4]])  # 5% past tmin: above the recording threshold
    t, p, m = _closest(scene, [0, 0, 0], [0, 0, 1], tmin=1e-4)
    assert p == 0 and m == math.inf
    tri = [[-1, -1, 3], [1, -1, 3], [0, 1, 3]]
    scene = make_scene(tris=[tri, tri])
    t, p, m = _closest(scene, [0, 0, 0], [0, 0, 1])
    assert (p, t, m) == (0, 3.0, 0.0)
    t, p, m = _closest(scene, [0, 0, 0], [0, 0, 1], tmin=1e-4, exclude=0)
    assert p == 1 and t == 3.0
    # nothing near the ray: no decision can flip
    t, p, m = _closest(scene, [5, 5, 0], [0, 0, 1])
    assert p == -1 and m == math.inf


# ---------------------------------------------------------------------------------------------
# Occlusion decision margins
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("clear", [1.001, 0.999, 1.2, 0.5])
def test_occlusion_margin_sphere_clearance(clear):
    """A shadow segment passing a sphere's centre at distance h = clear * r: occluded iff h < r, with
    margin |1 - (h/r)^2|."""
    r = 0.5
    scene = make_scene(spheres=[[clear * r, 2.0, 5.5, r]])
    P = np.array([0.0, 0.0, 4.0])
    Lp = np.array([0.0, 4.0, 7.0])
    d = (Lp - P) / 5.0  # (0, 0.8, 0.6): the segment's midpoint (0, 2, 5.5) is the foot of the centre
    occ, m = oracle.occluded(scene, [P], [d], tmax=5.0)
    h = f32(clear * r)
    assert occ[0] == (h < r)
    assert m[0] == pytest.approx(abs(1 - (h / r) ** 2), rel=1e-8)


def test_occlusion_margin_near_segment_ends():
    """An occluder crossing the segment just past its end (light just in front of a surface) or just
    before it: the relative distance of its t from tmax.  A sphere whose closest approach lies inside
    the segment always counts, however far it is (h = 6 r: |1 - 36| = 35); nothing inside or near the
    segment: infinite margin."""
    for z, expect in ((5.0 * 1.003, False), (5.0 * 0.997, True)):
        scene = make_scene(planes=[[0, 0, 1, z]])
        occ, m = oracle.occluded(scene, [[0.0, 0.0, 0.0]], [[0.0, 0.0, 1.0]], tmax=5.0)
        assert occ[0] == expect
        assert m[0] == pytest.approx(abs(f32(z) - 5.0) / 5.0, rel=1e-6)
    scene = make_scene(planes=[[0, 0, 1, 50.0]], spheres=[[3, 0, 2, 0.5]])
    occ, m = oracle.occluded(scene, [[0.0, 0.0, 0.0]], [[0.0, 0.0, 1.0]], tmax=5.0)
    assert not occ[0] and m[0] == pytest.approx(35.0, rel=1e-12)
    scene = make_scene(planes=[[0, 0, 1, 50.0]], spheres=[[3, 0, -2, 0.5]])  # behind the origin
    occ, m = oracle.occluded(scene, [[0.0, 0.0, 0.0]], [[0.0, 0.0, 1.0]], tmax=5.0)
    assert not occ[0] and m[0] == math.inf


# ---------------------------------------------------------------------------------------------
# Shading terms, shadow contributions and margins in a render (1x1 cameras: the ray is the axis)
# ---------------------------------------------------------------------------------------------
#
# Camera at (0, 3, 0) looking along (0, -3, 4)/5 = (0, -0.6, 0.8) hits the floor y = 0 at (0, 0, 4)
# (t = 5).  There N = (0, 1, 0) and V = (0, 0.6, -0.8).
#   light A at (0, 4, 7):  L = (0, 0.8, 0.6), N.L = 0.8, R = (0, 0.8, -0.6), R.V = 0.96
#   light B at (0, -4, 7): L = (0, -0.8, 0.6), N.L = -0.8 (behind the surface: no shadow ray);
#                          at N.L = 0 the reflected light direction is -L and -L.V = 0.96
# Material kd = (0.5, 0.25, 0.125), ks = (0.25, 0.5, 0.75), n = 2; I_A = (1, 0.5, 0.25), I_B = 0.5.
#   light A's term: I_A (kd 0.8 + ks 0.9216) = (0.6304, 0.3304, 0.1978)
#   light B's worth: I_B ks 0.9216 = (0.1152, 0.2304, 0.3456)

KD = (0.5, 0.25, 0.125)
KS = (0.25, 0.5, 0.75)


def _axis_camera(depth=0):
    return mono_camera(center=(0, 3, 0), forward=(0, -3, 4), width=1, height=1, depth=depth)


@pytest.mark.parametrize("clear", [1.001, 0.999])
def test_render_shadow_contrib_and_margins(clear):
    sphere = [clear * 0.5, 2.0, 5.5, 0.5]  # passes light A's shadow segment at clearance clear * r
    scene = make_scene(planes=[[0, 1, 0, 0]], spheres=[sphere], plane_mat=[0], sphere_mat=[1],
                       materials=[material(kd=KD, ks=KS, n=2.0), material()],
                       lights=[[0, 4, 7, 1, 0.5, 0.25], [0, -4, 7, 0.5, 0.5, 0.5]])
    r = oracle.render(scene, _axis_camera())
    assert r["hit_prim"][0] == 1 and r["hit_t"][0] == pytest.approx(5.0, rel=1e-12)
    assert r["hit_margin"][0, 0] == math.inf  # the floor alone: nothing near, no runner-up
    h = f32(clear * 0.5)
    occluded = h < 0.5
    assert r["shadow_state"][0, 0, 0] == (1 if occluded else 2)
    assert r["shadow_contrib"][0, 0, 0] == pytest.approx(0.6304, rel=1e-12)
    assert r["shadow_margin"][0, 0, 0] == pytest.approx(abs(1 - (h / 0.5) ** 2), rel=1e-8)  # below N.L = 0.8
    assert r["shadow_state"][0, 0, 1] == 0
    assert r["shadow_contrib"][0, 0, 1] == pytest.approx(0.3456, rel=1e-12)
    assert r["shadow_margin"][0, 0, 1] == pytest.approx(0.8, rel=1e-12)
    expect = np.zeros(3) if occluded else np.array([0.6304, 0.3304, 0.1978])
    np.testing.assert_allclose(r["radiance"][0], expect, rtol=1e-12, atol=1e-15)


def test_render_shadow_margin_is_cast_margin_when_nothing_occludes():
    scene = make_scene(planes=[[0, 1, 0, 0]], materials=[material(kd=KD, ks=KS, n=2.0)],
                       lights=[[0, 4, 7, 1, 0.5, 0.25]])
    r = oracle.render(scene, _axis_camera())
    assert r["shadow_state"][0, 0, 0] == 2
    assert r["shadow_margin"][0, 0, 0] == pytest.approx(0.8, rel=1e-12)


def test_render_contrib_carries_the_throughput():
    """A mirror floor (kr 0.5) reflects the axis ray to (0, 0.6, 0.8), which meets the wall z = 10 at
    (0, 4.5, 10) with N = (0, 0, -1) and V = (0, -0.6, -0.8).  Light at (0, 7.5, 6): L = (0, 0.6, -0.8),
    N.L = 0.8, R = (0, -0.6, -0.8), R.V = 1.  Term I (kd 0.8 + ks) = (0.65, 0.35, 0.2125); at the pixel
    it is worth 0.5 x 0.65 = 0.325, and the pixel's radiance is 0.5 x the term."""
    scene = make_scene(planes=[[0, 1, 0, 0], [0, 0, 1, 10]], plane_mat=[0, 1],
                       materials=[material(kd=(0, 0, 0), ks=(0, 0, 0), kr=(0.5, 0.5, 0.5)),
                                  material(kd=KD, ks=KS, n=2.0)],
                       lights=[[0, 7.5, 6, 1, 0.5, 0.25]])
    r = oracle.render(scene, _axis_camera(depth=1))
    assert list(r["path_prims"][0]) == [0, 1]
    assert r["shadow_state"][0, 0, 0] == 2 and r["shadow_contrib"][0, 0, 0] == 0.0  # black mirror
    assert r["shadow_state"][0, 1, 0] == 2
    assert r["shadow_contrib"][0, 1, 0] == pytest.approx(0.325, rel=1e-12)
    assert r["shadow_margin"][0, 1, 0] == pytest.approx(0.8, rel=1e-12)
    assert r["hit_margin"][0, 1] == math.inf
    np.testing.assert_allclose(r["radiance"][0], [0.325, 0.175, 0.10625], rtol=1e-12)


# ---------------------------------------------------------------------------------------------
# Triangle shading: the normal from the plane equation, not from a cross product
# ---------------------------------------------------------------------------------------------

@pytest.mark.parametrize("light,lit", [((2.0, 2.0, 3.0), True), ((-1.0, -1.0, 0.0), False)])
def test_lit_triangle_quad_lambert(light, lit):
    """The quad (s, t, 4 - 2s - 2t), s, t in [0, 1], lies exactly on the plane 2x + 2y + z = 4, so its
    unit normal is (2, 2, 1)/3.  Split into two triangles of opposite winding, lit by a point light:
    radiance = rho I max(0, n.L) at every pixel that sees it (ks = 0, no ambient), the hit point coming
    from the plane equation, and the id from which side of the diagonal s = t the point lies."""
    quad = [[0, 0, 4], [1, 0, 2], [1, 1, 0], [0, 1, 2]]
    tris = [[quad[0], quad[1], quad[2]], [quad[0], quad[3], quad[2]]]  # the second wound the other way
    rho = np.array([0.8, 0.5, 0.3])
    I = np.array([0.9, 0.7, 1.1])
    scene = make_scene(tris=tris, materials=[material(kd=rho)], lights=[list(light) + list(I)],
                       background=(0.1, 0.2, 0.3))
    C = np.array([3.0, 3.0, 6.0])
    cam = mono_camera(center=C, forward=np.array([0.5, 0.5, 2.0]) - C, width=40, height=40, hfov=30.0)
    res = oracle.render(scene, cam)
    n = np.array([2.0, 2.0, 1.0])
    nhat = n / 3.0
    Lf, If, rf = f32(light), f32(I), f32(rho)
    seen = 0
    for k in range(40 * 40):
        j, i = divmod(k, 40)
        O, d = oracle.primary_ray(cam, 0, i, j)
        t = (4.0 - n @ O) / (n @ d)
        P = O + t * d
        s_, t_ = P[0], P[1]
        inside = min(s_, t_, 1 - s_, 1 - t_, abs(s_ - t_)) > 1e-6
        if not inside:
            continue
        seen += 1
        assert res["hit_prim"][k] == (0 if s_ > t_ else 1)
        assert res["hit_t"][k] == pytest.approx(t, rel=1e-12)
        L = (Lf - P) / np.linalg.norm(Lf - P)
        N = nhat if (nhat @ d) < 0 else -nhat
        expect = rf * If * max(0.0, N @ L)
        np.testing.assert_allclose(res["radiance"][k], expect, rtol=1e-10, atol=1e-14)
        assert res["shadow_state"][k, 0, 0] == (2 if lit else 0)
    assert seen > 300
