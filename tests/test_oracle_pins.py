"""Pins of the FP64 oracle to closed forms, geometric identities and invariants.

None of these re-type the oracle's own formulas: each expected value comes from
a different route (textbook quadratic roots, a linear solve, projective
geometry, a mirrored camera, superposition), so that a dropped term, a wrong
sign or index, or a transposed operand in the oracle fails one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import scenegen as sg
from tests.helpers import make_scene, material, mono_camera, f32

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------------------------
# Ray-primitive tests
# ---------------------------------------------------------------------------------------------

def _textbook_sphere(O, d, c, r):
    """Roots of |O + t d - c|^2 = r^2 with the schoolbook formula (-b +- sqrt(b^2 - 4ac)) / 2a."""
    oc = O - c
    a = d @ d
    b = 2 * d @ oc
    cc = oc @ oc - r * r
    disc = b * b - 4 * a * cc
    if disc < 0:
        return []
    s = math.sqrt(disc)
    return sorted([(-b - s) / (2 * a), (-b + s) / (2 * a)])


def test_sphere_matches_textbook_roots():
    rng = np.random.default_rng(5)
    n_hit = n_miss = n_inside = 0
    for _ in range(2000):
        c = rng.uniform(-3, 3, 3)
        r = rng.uniform(0.1, 2.0)
        O = rng.uniform(-6, 6, 3) if rng.random() > 0.1 else c + rng.uniform(-0.5, 0.5, 3) * r
        d = (c - O) * rng.choice([1.0, -1.0], p=[0.8, 0.2]) + rng.normal(size=3) * r
        d /= np.linalg.norm(d)
        roots = [t for t in _textbook_sphere(O, d, c, r) if t > 0]
        hit, t = oracle.intersect_sphere(O, d, c, r)
        if roots:
            assert hit
            assert t == pytest.approx(roots[0], rel=1e-9, abs=1e-9)
            n_hit += 1
            n_inside += np.linalg.norm(O - c) < r
        else:
            assert not hit
            n_miss += 1
    assert n_hit > 100 and n_miss > 100 and n_inside > 10


def test_sphere_special_cases():
    c = np.array([0.0, 0.0, 5.0])
    d = np.array([0.0, 0.0, 1.0])
    # straight through: near root at 4
    assert oracle.intersect_sphere([0, 0, 0], d, c, 1.0) == (True, pytest.approx(4.0))
    # origin inside: far root
    assert oracle.intersect_sphere([0, 0, 5.5], d, c, 1.0) == (True, pytest.approx(0.5))
    # sphere behind the ray: miss
    assert not oracle.intersect_sphere([0, 0, 10], d, c, 1.0)[0]
    # tangent ray: one double root at the closest approach
    hit, t = oracle.intersect_sphere([1.0, 0, 0], d, c, 1.0)
    assert hit and t == pytest.approx(5.0)
    # passing just outside: miss
    assert not oracle.intersect_sphere([1.0 + 1e-9, 0, 0], d, c, 1.0)[0]
    # tmax cuts the root off
    assert not oracle.intersect_sphere([0, 0, 0], d, c, 1.0, tmax=3.9)[0]


def test_triangle_recovers_constructed_barycentrics():
    rng = np.random.default_rng(7)
    for _ in range(1000):
        v0, v1, v2 = rng.uniform(-2, 2, (3, 3))
        u, v = rng.uniform(0, 1, 2)
        if u + v > 1:
            u, v = 1 - u, 1 - v
        P = (1 - u - v) * v0 + u * v1 + v * v2
        O = rng.uniform(-5, 5, 3)
        d = P - O  # not unit: the hit is at t = 1
        hit, t, uu, vv = oracle.intersect_triangle(O, d, v0, v1, v2)
        assert hit
        assert t == pytest.approx(1.0, abs=1e-9)
        assert uu == pytest.approx(u, abs=1e-9) and vv == pytest.approx(v, abs=1e-9)


def test_triangle_decision_matches_linear_solve():
    """O + t d = v0 + u (v1 - v0) + v (v2 - v0) solved by LU (numpy) decides hit/miss the same way."""
    rng = np.random.default_rng(8)
    hits = misses = 0
    for _ in range(3000):
        v0, v1, v2 = rng.uniform(-1, 1, (3, 3))
        O = rng.uniform(-3, 3, 3)
        d = ((v0 + v1 + v2) / 3 - O) * rng.choice([1.0, -1.0], p=[0.9, 0.1]) + rng.normal(size=3) * 0.5
        A = np.stack([d, -(v1 - v0), -(v2 - v0)], axis=1)
        if abs(np.linalg.det(A)) < 1e-6:
            continue
        t, u, v = np.linalg.solve(A, v0 - O)
        m = min(u, v, 1 - u - v, t)
        if abs(m) < 1e-9:
            continue
        expect = m > 0
        hit, tt, uu, vv = oracle.intersect_triangle(O, d, v0, v1, v2)
        assert hit == expect
        if hit:
            hits += 1
            assert tt == pytest.approx(t, rel=1e-9, abs=1e-12)
        else:
            misses += 1
    assert hits > 100 and misses > 100


def test_triangle_edges_inclusive_and_parallel_rejected():
    v0, v1, v2 = np.array([0.0, 0, 0]), np.array([1.0, 0, 0]), np.array([0.0, 1, 0])
    d = np.array([0.0, 0, 1])
    # exactly on the hypotenuse u + v = 1 and on the vertices: closed triangle
    for p in ([0.5, 0.5], [0.0, 0.0], [1.0, 0.0], [0.0, 1.0], [0.25, 0.0]):
        assert oracle.intersect_triangle([p[0], p[1], -1], d, v0, v1, v2)[0]
    assert not oracle.intersect_triangle([0.5 + 1e-12, 0.5, -1], d, v0, v1, v2)[0]
    # ray in the triangle's plane: det = 0, rejected
    assert not oracle.intersect_triangle([-1, 0.2, 0], [1, 0, 0], v0, v1, v2)[0]
    # behind the origin
    assert not oracle.intersect_triangle([0.2, 0.2, 1], d, v0, v1, v2)[0]


def test_plane_hits_constructed_point():
    rng = np.random.default_rng(9)
    for _ in range(500):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        dist = rng.uniform(-3, 3)
        Q = dist * n + np.cross(n, rng.normal(size=3))  # a point with n.Q = dist
        d = rng.normal(size=3)
        if abs(n @ d) < 1e-3:
            continue
        t0 = rng.uniform(0.1, 10)
        O = Q - t0 * d
        hit, t = oracle.intersect_plane(O, d, n, dist)
        assert hit and t == pytest.approx(t0, rel=1e-9)
        assert not oracle.intersect_plane(Q + t0 * d, d, n, dist)[0]  # plane behind
    assert not oracle.intersect_plane([0, 1, 0], [1, 0, 0], [0, 1, 0], 0.0)[0]  # parallel


# ---------------------------------------------------------------------------------------------
# Stereo camera
# ---------------------------------------------------------------------------------------------

def _rays(cam, eye):
    W, H = cam.width, cam.height
    O = np.zeros((H, W, 3))
    D = np.zeros((H, W, 3))
    for j in range(H):
        for i in range(W):
            O[j, i], D[j, i] = oracle.primary_ray(cam, eye, i, j)
    return O, D


def test_eye_positions_and_basis():
    cam = sg.make_camera((0.5, 1, -2), forward=(0, 0, 3), baseline=0.065, convergence=5.0, width=33, height=21)
    B = f32(0.065)
    OL, dL = oracle.primary_ray(cam, 0, 0, 0)
    OR, dR = oracle.primary_ray(cam, 1, 0, 0)
    # forward +z, up +y: right = +x, so the left eye sits at -B/2 along x
    np.testing.assert_allclose(OL, [0.5 - B / 2, 1, -2], atol=1e-15)
    np.testing.assert_allclose(OR, [0.5 + B / 2, 1, -2], atol=1e-15)
    # pixel (0, 0) is the top-left corner: it looks left (-x) and up (+y)
    assert dL[0] < 0 and dL[1] > 0
    for eye in (0, 1):
        _, d = oracle.primary_ray(cam, eye, 7, 3)
        assert np.linalg.norm(d) == pytest.approx(1.0, abs=1e-15)


def _point_on_ray_distance(X, O, d):
    w = X - O
    return np.linalg.norm(w - (w @ d) * d)


def test_centre_rays_converge_at_z0():
    for Z0 in (2.0, 5.0, 13.0):
        cam = sg.make_camera((0.3, 1.2, -1), forward=(0.2, -0.1, 1), baseline=0.1, convergence=Z0, width=41, height=31)
        f = f32(cam.forward) / np.linalg.norm(f32(cam.forward))
        X = f32(cam.center) + f32(Z0) * f
        for eye in (0, 1):
            O, d = oracle.primary_ray(cam, eye, 20, 15)  # centre pixel of an odd-sized image
            assert _point_on_ray_distance(X, O, d) < 1e-12


def test_field_of_view_and_pinhole_linearity():
    for hfov in (40.0, 60.0, 90.0):
        cam = mono_camera(width=50, height=30, hfov=hfov)
        tans = []
        for i in range(cam.width):
            _, d = oracle.primary_ray(cam, 0, i, 10)
            tans.append(d[0] / d[2])
        tans = np.array(tans)
        steps = np.diff(tans)
        np.testing.assert_allclose(steps, steps.mean(), rtol=1e-9)  # a pinhole is affine in tan space
        left = tans[0] - steps.mean() / 2
        right = tans[-1] + steps.mean() / 2
        assert math.degrees(math.atan(right) - math.atan(left)) == pytest.approx(hfov, rel=1e-9)
        # square pixels: vertical tan steps equal horizontal ones, row 0 at the top
        tv = [oracle.primary_ray(cam, 0, 25, j)[1] for j in (0, 1)]
        assert tv[0][1] / tv[0][2] - tv[1][1] / tv[1][2] == pytest.approx(steps.mean(), rel=1e-9)


@pytest.mark.parametrize("Z0", [0.0, 5.0, 12.0])
def test_disparity_closed_form(Z0):
    """A point on the axis at depth Z lands u_L - u_R = f_px B (1/Z - 1/Z0) pixels apart (f_px B / Z if parallel)."""
    W, H, hfov, B = 256, 256, 60.0, 0.065
    cam = sg.make_camera((0, 1, 0), forward=(0, 0, 1), baseline=B, convergence=Z0, width=W, height=H, hfov_deg=hfov)
    fpx = (W / 2) / math.tan(math.radians(hfov) / 2)
    assert fpx == pytest.approx(221.70, abs=0.01)
    Bf = f32(B)
    for Z in (2.0, 5.0, 9.0, 40.0):
        X = np.array([0.0, 1.0, Z])
        cols = []
        for eye in (0, 1):
            O0, d0 = oracle.primary_ray(cam, eye, 0, 128)
            O1, d1 = oracle.primary_ray(cam, eye, 1, 128)
            t0, t1 = d0[0] / d0[2], d1[0] / d1[2]
            tx = (X[0] - O0[0]) / (X[2] - O0[2])
            cols.append((tx - t0) / (t1 - t0))  # sub-pixel column index where the eye sees X
        disparity = cols[0] - cols[1]
        expect = fpx * Bf * (1 / Z - (1 / Z0 if Z0 > 0 else 0.0))
        assert disparity == pytest.approx(expect, rel=1e-9, abs=1e-9)
    if Z0 == 0.0:  # the parallel-axis value quoted for the tiny sphere scene at Z = 5
        assert fpx * Bf / 5.0 == pytest.approx(2.882, abs=1e-3)


def test_zero_baseline_gives_identical_eyes():
    scene, cam = sg.make_spheres_scene()
    cam = cam.resized(48, 40).with_(baseline=0.0)
    r = oracle.render(scene, cam)
    n = cam.width * cam.height
    assert np.array_equal(r["radiance"][:n], r["radiance"][n:])
    assert np.array_equal(r["path_prims"][:n], r["path_prims"][n:])


# ---------------------------------------------------------------------------------------------
# Shading
# ---------------------------------------------------------------------------------------------

def test_headlight_lambert_closed_form():
    """One diffuse sphere lit from the eye: radiance = rho I sqrt(1 - (h/r)^2), h = centre-to-ray distance."""
    c = np.array([0.3, 0.9, 6.0])
    r = 1.3
    rho = np.array([0.7, 0.4, 0.2])
    I = np.array([0.9, 1.1, 0.5])
    eye = np.array([0.0, 1.0, 0.0])
    scene = make_scene(spheres=[list(c) + [r]], materials=[material(kd=rho, ks=(0.5, 0.5, 0.5))],
                       lights=[list(eye) + list(I)], background=(0.1, 0.2, 0.3))
    # ks != 0 on purpose: with the light at the eye L = V, so R.V = 2 cos^2(theta) - 1 = 1 - 2 (h/r)^2
    # with cos(theta) = sqrt(1 - (h/r)^2) the incidence cosine.
    cam = mono_camera(center=eye, width=40, height=40, hfov=30.0)
    res = oracle.render(scene, cam)
    L = res["radiance"][: 40 * 40].reshape(40, 40, 3)
    cf, rf, rhof, If = f32(c), f32(r), f32(rho), f32(I)
    checked = 0
    for j in range(40):
        for i in range(40):
            O, d = oracle.primary_ray(cam, 0, i, j)
            w = cf - O
            h = np.linalg.norm(w - (w @ d) * d)
            if abs(h - rf) < 1e-6:
                continue
            if h < rf:
                q = (h / rf) ** 2
                expect = rhof * If * math.sqrt(1 - q) + 0.5 * If * max(0.0, 1 - 2 * q) ** 32
                np.testing.assert_allclose(L[j, i], expect, rtol=1e-9, atol=1e-12)
                checked += 1
            else:
                np.testing.assert_allclose(L[j, i], [0.1, 0.2, 0.3], atol=1e-7)
    assert checked > 300


def test_phong_on_plane_closed_form():
    """Diffuse + specular on the plane y = 0 from a point light: the mirror of R.V through the plane is the
    angle between the light direction and the line from the eye's mirror image (C_x, -C_y, C_z) through P."""
    C = np.array([0.4, 2.0, -1.0])
    Lp = np.array([-1.5, 3.0, 6.0])
    I = np.array([0.8, 0.6, 1.0])
    kd, ks, n = np.array([0.3, 0.2, 0.1]), np.array([0.6, 0.7, 0.5]), 32.0
    scene = make_scene(planes=[[0, 1, 0, 0]], materials=[material(kd=kd, ks=ks, n=n)], lights=[list(Lp) + list(I)],
                       ambient=(0.0, 0.0, 0.0))
    cam = mono_camera(center=C, forward=(0, -0.6, 1), width=64, height=48, hfov=70.0)
    res = oracle.render(scene, cam)
    Lr = res["radiance"][: 64 * 48].reshape(48, 64, 3)
    Cf, Lf, If, kdf, ksf = f32(C), f32(Lp), f32(I), f32(kd), f32(ks)
    Cm = Cf * np.array([1, -1, 1])
    best = (-1.0, None)
    count = 0
    for j in range(48):
        for i in range(64):
            O, d = oracle.primary_ray(cam, 0, i, j)
            if d[1] >= 0:
                continue
            P = O + (-O[1] / d[1]) * d  # the plane y = 0 by direct substitution
            ldir = (Lf - P) / np.linalg.norm(Lf - P)
            view_m = (P - Cm) / np.linalg.norm(P - Cm)
            spec = max(0.0, ldir @ view_m) ** n
            expect = If * (kdf * ldir[1] + ksf * spec)
            np.testing.assert_allclose(Lr[j, i], expect, rtol=1e-9, atol=1e-12)
            count += 1
            if spec > best[0]:
                best = (spec, P)
    assert count > 1000
    # the highlight peak sits where the eye's mirror image, P and the light are collinear
    hc, hl = Cf[1], Lf[1]
    X = (hl * Cf[[0, 2]] + hc * Lf[[0, 2]]) / (hl + hc)
    assert np.linalg.norm(best[1][[0, 2]] - X) < 0.15


def test_shadow_mask_matches_segment_distance():
    """A point on the plane is shadowed iff the segment from it to the light passes within r of the sphere centre."""
    c = np.array([0.2, 1.0, 5.0])
    r = 0.6
    Lp = np.array([-0.5, 4.0, 4.0])
    scene = make_scene(spheres=[list(c) + [r]], planes=[[0, 1, 0, 0]], sphere_mat=[0], plane_mat=[1],
                       materials=[material(), material(kd=(0.5, 0.5, 0.5))], lights=[list(Lp) + [1, 1, 1]])
    cam = mono_camera(center=(0, 2.0, 0), forward=(0, -0.45, 1), width=80, height=60, hfov=60.0)
    res = oracle.render(scene, cam)
    cf, rf, Lf = f32(c), f32(r), f32(Lp)
    n_shadow = n_lit = 0
    for k in range(80 * 60):
        if res["hit_prim"][k] != 1:  # plane pixels only
            continue
        j, i = divmod(k, 80)
        O, d = oracle.primary_ray(cam, 0, i, j)
        P = O + (-O[1] / d[1]) * d
        seg = Lf - P
        s = np.clip((cf - P) @ seg / (seg @ seg), 0, 1)
        dist = np.linalg.norm(P + s * seg - cf)
        if abs(dist - rf) < 1e-6:
            continue
        state = res["shadow_state"][k, 0, 0]
        if dist < rf:
            assert state == 1
            n_shadow += 1
        else:
            assert state == 2
            n_lit += 1
    assert n_shadow > 50 and n_lit > 500


def test_mirror_plane_equals_mirrored_camera():
    """Bounce-1 off a perfect mirror y = 0 sees what a camera mirrored through the plane sees directly
    (with image columns flipped, since a mirror reverses handedness)."""
    spheres = [[-0.8, 0.7, 4.0, 0.5], [0.6, 1.2, 5.0, 0.7], [0.1, 0.4, 3.0, 0.3]]
    mats = [material(kd=(0.8, 0.2, 0.2), ks=(0.4, 0.4, 0.4)), material(kd=(0.2, 0.8, 0.3), ks=(0.2, 0.2, 0.2)),
            material(kd=(0.3, 0.3, 0.9)), material(kd=(0, 0, 0), ks=(0, 0, 0), kr=(1, 1, 1))]
    lights = [[-2, 5, 1, 1, 1, 1], [3, 4, 8, 0.5, 0.4, 0.3]]
    full = make_scene(spheres=spheres, sphere_mat=[0, 1, 2], planes=[[0, 1, 0, 0]], plane_mat=[3], materials=mats,
                      lights=lights, ambient=(0.05, 0.05, 0.05))
    no_plane = make_scene(spheres=spheres, sphere_mat=[0, 1, 2], materials=mats, lights=lights,
                          ambient=(0.05, 0.05, 0.05))
    W, H = 48, 40
    cam = mono_camera(center=(0.1, 1.5, 0), forward=(0, -0.3, 1), up=(0, 1, 0), width=W, height=H, depth=1)
    mcam = mono_camera(center=(0.1, -1.5, 0), forward=(0, 0.3, 1), up=(0, -1, 0), width=W, height=H, depth=1)
    a = oracle.render(full, cam)
    b = oracle.render(no_plane, mcam)
    plane_id = 3
    checked = 0
    for k in range(W * H):
        if a["path_prims"][k, 0] != plane_id:
            continue
        j, i = divmod(k, W)
        km = j * W + (W - 1 - i)
        if min(a["hit_margin"][k, 1], b["hit_margin"][km, 0]) < 1e-7:
            continue
        assert a["path_prims"][k, 1] == b["path_prims"][km, 0]
        np.testing.assert_allclose(a["radiance"][k], b["radiance"][km], rtol=1e-9, atol=1e-12)
        checked += 1
    assert checked > 200
    assert np.any(a["path_prims"][:, 1] >= 0)


def test_light_superposition():
    """Radiance is linear in the lights: L({A,B}) = L({A}) + L({B}) - L({})."""
    scene, cam = sg.make_spheres_scene()
    cam = cam.resized(40, 32)
    A = [-2, 5, 2, 1, 0.8, 0.6]
    Bl = [3, 4, 1, 0.3, 0.5, 0.7]
    rab = oracle.render(scene.with_lights([A, Bl]), cam)["radiance"]
    ra = oracle.render(scene.with_lights([A]), cam)["radiance"]
    rb = oracle.render(scene.with_lights([Bl]), cam)["radiance"]
    r0 = oracle.render(scene.with_lights(np.zeros((0, 6))), cam)["radiance"]
    np.testing.assert_allclose(rab, ra + rb - r0, atol=1e-12)


def test_reflection_depth_geometric_series():
    """Camera between two facing mirrors: ids alternate per bounce and radiance is a finite geometric sum."""
    # plane 0: z = 0 (seen facing +z), plane 1: z = 10
    planes = [[0, 0, 1, 0.0], [0, 0, 1, 10.0]]
    a = np.array([0.2, 0.4, 0.6])
    b = np.array([0.5, 0.1, 0.3])
    kr = 0.5
    mats = [material(kd=a, kr=(kr,) * 3), material(kd=b, kr=(kr,) * 3)]
    amb = np.array([1.0, 1.0, 1.0])
    scene = make_scene(planes=planes, plane_mat=[0, 1], materials=mats, ambient=amb)
    for D in (0, 1, 3, 5):
        cam = mono_camera(center=(0, 0, 5), forward=(0.05, 0.02, 1), width=3, height=3, depth=D)
        res = oracle.render(scene, cam)
        pp = res["path_prims"][4]  # centre pixel, left eye
        expect_ids = [1 if k % 2 == 0 else 0 for k in range(D + 1)]
        assert list(pp) == expect_ids
        kd_seq = [f32(b) if k % 2 == 0 else f32(a) for k in range(D + 1)]
        expect = sum((f32(kr) ** k) * kd_seq[k] for k in range(D + 1))
        np.testing.assert_allclose(res["radiance"][4], expect, rtol=1e-12)


def test_no_reflectance_makes_depth_irrelevant():
    scene, cam = sg.make_paper5_scene()
    scene.materials[:, 6:9] = 0.0
    cam = cam.resized(40, 40)
    r0 = oracle.render(scene, cam.with_(max_depth=0))
    r4 = oracle.render(scene, cam.with_(max_depth=4))
    assert np.array_equal(r0["radiance"], r4["radiance"])
    assert r4["ray_counts"][1] == 0


def test_stereo_mirror_symmetry():
    """A scene symmetric about the plane x = C_x gives a left image equal to the flipped right image."""
    spheres = [[-0.9, 0.6, 4.0, 0.4], [0.9, 0.6, 4.0, 0.4], [0.0, 1.1, 6.0, 0.7]]
    mats = [material(kd=(0.7, 0.3, 0.3), ks=(0.3,) * 3, kr=(0.3,) * 3), material(kd=(0.3, 0.3, 0.3))]
    scene = make_scene(spheres=spheres, sphere_mat=[0, 0, 0], planes=[[0, 1, 0, 0]], plane_mat=[1], materials=mats,
                       lights=[[0, 5, 2, 1, 1, 1]], ambient=(0.05,) * 3)
    W, H = 40, 30
    for Z0 in (0.0, 5.0):
        cam = sg.make_camera((0, 1, 0), forward=(0, -0.1, 1), baseline=0.2, convergence=Z0, width=W, height=H,
                             max_depth=2)
        res = oracle.render(scene, cam)
        left = res["radiance"][: W * H].reshape(H, W, 3)
        right = res["radiance"][W * H:].reshape(H, W, 3)
        np.testing.assert_allclose(left, right[:, ::-1], atol=1e-12)


def test_secondary_rays_skip_origin_and_count():
    scene, cam = sg.make_spheres_scene()
    cam = cam.resized(64, 64)
    res = oracle.render(scene, cam)
    pp = res["path_prims"]
    # a reflection off a convex sphere never re-hits it
    sph = (pp[:, 0] >= 0) & (pp[:, 0] < 8)
    assert np.all(pp[sph, 1] != pp[sph, 0])
    assert res["ray_counts"][0] == 2 * 64 * 64
    assert res["ray_counts"][1] == np.count_nonzero(pp[:, 1] != -2)
    assert res["ray_counts"][2] == np.count_nonzero(res["shadow_state"] != 0)


def test_paper5_fixture_matches_paper_counts():
    g = json.load(open(os.path.join(GOLDEN, "paper5_objects.json")))
    scene, _ = sg.make_paper5_scene()
    assert [list(x) for x in scene.info["solids"]] == g["objects"]
    assert scene.num_triangles == g["total_polygons"]


# ---------------------------------------------------------------------------------------------
# Stereo-pair building
# ---------------------------------------------------------------------------------------------

def test_display_encoding_closed_forms():
    x = np.array([0.0, 1.0, 0.25, 4.0, -1.0, 1.0 / 255.0 ** 2, 0.5], np.float32)
    codes = oracle.encode8(x)
    assert codes[0] == 0 and codes[1] == 255 and codes[3] == 255 and codes[4] == 0
    assert codes[2] == 128  # sqrt(0.25) = 0.5 -> 127.5 + 0.5 -> 128
    assert codes[5] == 1  # sqrt(1/255^2) = 1/255 -> 1.5 -> 1
    assert codes[6] == 180  # 255 * 0.70710677 = 180.31 -> 180
    assert oracle.encode8(np.float32(0.25), exposure=4.0) == 255
    # monotone and onto 0..255 over [0, 1]
    ramp = oracle.encode8(np.linspace(0, 1, 200001, dtype=np.float32))
    assert np.all(np.diff(ramp.astype(int)) >= 0) and set(ramp) == set(range(256))


def test_anaglyph_and_side_by_side_layout():
    rng = np.random.default_rng(3)
    L = rng.uniform(0, 1.2, (5, 7, 3)).astype(np.float32)
    R = rng.uniform(0, 1.2, (5, 7, 3)).astype(np.float32)
    a = oracle.compose_stereo(L, R, "anaglyph")
    assert a.shape == (5, 7, 4) and np.all(a[..., 3] == 255)
    assert np.array_equal(a[..., 0], oracle.encode8(L[..., 0]))
    assert np.array_equal(a[..., 1], oracle.encode8(R[..., 1]))
    assert np.array_equal(a[..., 2], oracle.encode8(R[..., 2]))
    sbs = oracle.compose_stereo(L, R, "side_by_side")
    assert sbs.shape == (5, 14, 4)
    assert np.array_equal(sbs[:, :7, :3], oracle.encode8(L)) and np.array_equal(sbs[:, 7:, :3], oracle.encode8(R))
