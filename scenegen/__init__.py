"""Seeded synthetic stereo scenes and cameras.

This module is test and benchmark input only: it produces the FP32 arrays that
both the GPU library and the FP64 oracle consume.  It holds none of the ray
tracing arithmetic (no ray generation, intersection, shading or traversal).

The paper (Section 4, Figs 3-8) measures scenes of a few polyhedra lit by one
light; the throughput workloads here are larger procedural scenes of the same
kind (triangle soups lit by point lights, viewed by two eye cameras), built
from seeded value-noise height fields and icosphere instances.  Every array is
generated in float64 and rounded once to float32, so both consumers see the
identical vertices.

RNG: ``numpy.random.Generator(PCG64)`` streams spawned from
``SeedSequence(seed)`` in the fixed order [geometry, materials, mirror flags,
lights, camera].
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
import math

import numpy as np

MATERIAL_FIELDS = 10  # kd rgb, ks rgb, kr rgb, shininess
LIGHT_FIELDS = 6  # position xyz, intensity rgb


@dataclass
class Scene:
    """A scene as the flat FP32 arrays the C ABI takes.

    triangles [T,3,3] vertex positions; spheres [S,4] centre xyz + radius;
    planes [P,4] unit normal xyz + offset d (points x with n.x = d);
    materials [M,10] (kd, ks, kr, shininess); lights [L,6] (position, rgb).
    Primitive ids are the input order: triangles, then spheres, then planes.
    """

    name: str
    seed: int
    triangles: np.ndarray
    tri_material: np.ndarray
    spheres: np.ndarray
    sphere_material: np.ndarray
    planes: np.ndarray
    plane_material: np.ndarray
    materials: np.ndarray
    lights: np.ndarray
    ambient: np.ndarray
    background: np.ndarray
    info: dict = field(default_factory=dict)

    @property
    def num_triangles(self) -> int:
        return int(self.triangles.shape[0])

    @property
    def num_spheres(self) -> int:
        return int(self.spheres.shape[0])

    @property
    def num_planes(self) -> int:
        return int(self.planes.shape[0])

    @property
    def num_prims(self) -> int:
        return self.num_triangles + self.num_spheres + self.num_planes

    @property
    def num_lights(self) -> int:
        return int(self.lights.shape[0])

    def with_lights(self, lights) -> "Scene":
        return replace(self, lights=np.ascontiguousarray(np.asarray(lights, np.float32).reshape(-1, LIGHT_FIELDS)))


@dataclass
class StereoCamera:
    """Cyclopean eye pose plus the stereo and image parameters (all FP32).

    convergence <= 0 selects parallel optical axes; otherwise the two image
    centres converge at distance ``convergence`` along ``forward``.
    """

    center: np.ndarray
    forward: np.ndarray
    up: np.ndarray
    hfov_deg: float
    baseline: float
    convergence: float
    width: int
    height: int
    max_depth: int

    def resized(self, width: int, height: int) -> "StereoCamera":
        return replace(self, width=int(width), height=int(height))

    def with_(self, **kw) -> "StereoCamera":
        return replace(self, **kw)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _streams(seed: int):
    ss = np.random.SeedSequence(seed).spawn(5)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss]


def make_camera(center, target=None, forward=None, up=(0.0, 1.0, 0.0), hfov_deg=60.0, baseline=0.065,
                convergence=None, width=256, height=256, max_depth=1) -> StereoCamera:
    center = np.asarray(center, np.float64)
    if forward is None:
        forward = np.asarray(target, np.float64) - center
    forward = np.asarray(forward, np.float64)
    if convergence is None:
        convergence = float(np.linalg.norm(forward)) if target is not None else 0.0
    return StereoCamera(center=_f32(center), forward=_f32(forward), up=_f32(up), hfov_deg=float(np.float32(hfov_deg)),
                        baseline=float(np.float32(baseline)), convergence=float(np.float32(convergence)),
                        width=int(width), height=int(height), max_depth=int(max_depth))


# ---------------------------------------------------------------------------------------------
# Polyhedra (vertex sets generated from their definitions, faces found from adjacency)
# ---------------------------------------------------------------------------------------------

PHI = (1.0 + math.sqrt(5.0)) / 2.0


def _orient_outward(verts: np.ndarray, faces: list) -> np.ndarray:
    out = []
    c = verts.mean(axis=0)
    for f in faces:
        a, b, cc = verts[f[0]], verts[f[1]], verts[f[2]]
        n = np.cross(b - a, cc - a)
        if np.dot(n, (a + b + cc) / 3.0 - c) < 0:
            f = (f[0], f[2], f[1])
        out.append(f)
    return np.asarray(out, np.int64)


def icosahedron():
    """12 vertices (0,+-1,+-phi) and cyclic permutations; 20 faces = mutually adjacent triples."""
    v = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            v += [(0.0, s1, s2 * PHI), (s1, s2 * PHI, 0.0), (s2 * PHI, 0.0, s1)]
    v = np.asarray(v, np.float64)
    d = np.linalg.norm(v[:, None, :] - v[None, :, :], axis=-1)
    adj = np.isclose(d, 2.0)
    faces = [(i, j, k) for i in range(12) for j in range(i + 1, 12) for k in range(j + 1, 12)
             if adj[i, j] and adj[j, k] and adj[i, k]]
    assert len(faces) == 20
    return v, _orient_outward(v, faces)


def cube():
    """8 vertices (+-1)^3; each of the 6 faces split into two triangles."""
    v = np.asarray([(x, y, z) for x in (-1.0, 1.0) for y in (-1.0, 1.0) for z in (-1.0, 1.0)], np.float64)
    faces = []
    for axis in range(3):
        for s in (-1.0, 1.0):
            idx = [i for i in range(8) if v[i, axis] == s]
            n = np.zeros(3)
            n[axis] = s
            faces += _fan(v, idx, n)
    return v, _orient_outward(v, faces)


def dodecahedron():
    """20 vertices; its 12 pentagonal faces are the vertex sets that reach the maximum along a face
    normal (the vertex directions of the dual icosahedron, in the orientation for which exactly five
    vertices are extreme); each pentagon is fan-split into three triangles."""
    v = [(x, y, z) for x in (-1.0, 1.0) for y in (-1.0, 1.0) for z in (-1.0, 1.0)]
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            v += [(0.0, s1 / PHI, s2 * PHI), (s1 / PHI, s2 * PHI, 0.0), (s2 * PHI, 0.0, s1 / PHI)]
    v = np.asarray(v, np.float64)
    candidates = []
    for s1 in (-1.0, 1.0):
        for s2 in (-1.0, 1.0):
            candidates += [(0.0, s1 * PHI, s2), (s1 * PHI, s2, 0.0), (s2, 0.0, s1 * PHI),
                           (0.0, s1, s2 * PHI), (s1, s2 * PHI, 0.0), (s2 * PHI, 0.0, s1)]
    faces = []
    for n in np.asarray(candidates):
        n = n / np.linalg.norm(n)
        dots = v @ n
        top = np.nonzero(dots > dots.max() - 1e-9)[0]
        if len(top) == 5:
            faces += _fan(v, list(top), n)
    assert len(faces) == 36
    return v, _orient_outward(v, faces)


def _fan(v, idx, n):
    """Order a planar convex polygon's vertices around normal n and fan-triangulate from the first."""
    pts = v[idx]
    c = pts.mean(axis=0)
    a0 = pts[0] - c
    a0 /= np.linalg.norm(a0)
    b0 = np.cross(n, a0)
    ang = np.arctan2((pts - c) @ b0, (pts - c) @ a0)
    order = [idx[k] for k in np.argsort(ang, kind="stable")]
    return [(order[0], order[k], order[k + 1]) for k in range(1, len(order) - 1)]


def icosphere(level: int):
    """Unit icosahedron after ``level`` rounds of 4-way midpoint subdivision, re-projected to the sphere.

    20*4^L triangles, 10*4^L + 2 vertices."""
    v, f = icosahedron()
    verts = [p / np.linalg.norm(p) for p in v]
    faces = [tuple(x) for x in f]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    return np.asarray(verts, np.float64), np.asarray(faces, np.int64)


def random_rotation(rng) -> np.ndarray:
    """Uniform random rotation from a uniform unit quaternion (Shoemake 1992)."""
    u1, u2, u3 = rng.random(3)
    q = np.array([math.sqrt(1 - u1) * math.sin(2 * math.pi * u2), math.sqrt(1 - u1) * math.cos(2 * math.pi * u2),
                  math.sqrt(u1) * math.sin(2 * math.pi * u3), math.sqrt(u1) * math.cos(2 * math.pi * u3)])
    x, y, z, w = q
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
                     [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
                     [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)]])


# ---------------------------------------------------------------------------------------------
# Value-noise fBm height field
# ---------------------------------------------------------------------------------------------

class FBm:
    """Value noise on a seeded 256x256 lattice of U[-1,1] values, quintic fade, wrap-around,
    summed over octaves (frequency x lacunarity, amplitude x gain) and normalised by the amplitude sum
    so that |h| <= amplitude."""

    def __init__(self, rng, octaves, base_freq, lacunarity=2.0, gain=0.5, amplitude=1.0, size=256):
        self.lattice = rng.uniform(-1.0, 1.0, size=(size, size))
        self.offsets = rng.uniform(0.0, float(size), size=(octaves, 2))
        self.octaves, self.base_freq, self.lac, self.gain, self.amp, self.size = (
            octaves, base_freq, lacunarity, gain, amplitude, size)

    def _noise(self, x, z):
        x0 = np.floor(x)
        z0 = np.floor(z)
        fx, fz = x - x0, z - z0
        wx = fx * fx * fx * (fx * (fx * 6.0 - 15.0) + 10.0)
        wz = fz * fz * fz * (fz * (fz * 6.0 - 15.0) + 10.0)
        i0 = np.mod(x0.astype(np.int64), self.size)
        j0 = np.mod(z0.astype(np.int64), self.size)
        i1 = (i0 + 1) % self.size
        j1 = (j0 + 1) % self.size
        L = self.lattice
        a = L[i0, j0] * (1 - wx) + L[i1, j0] * wx
        b = L[i0, j1] * (1 - wx) + L[i1, j1] * wx
        return a * (1 - wz) + b * wz

    def __call__(self, x, z):
        x = np.asarray(x, np.float64)
        z = np.asarray(z, np.float64)
        total = np.zeros(np.broadcast(x, z).shape)
        norm = 0.0
        freq, amp = self.base_freq, 1.0
        for o in range(self.octaves):
            total = total + amp * self._noise(x * freq + self.offsets[o, 0], z * freq + self.offsets[o, 1])
            norm += amp
            freq *= self.lac
            amp *= self.gain
        return self.amp * total / norm


def heightfield_triangles(h: FBm, n: int, x0, x1, z0, z1) -> np.ndarray:
    """n x n vertex grid; each cell (i,j) split along the (i,j)-(i+1,j+1) diagonal, wound so e1 x e2 is +y."""
    xs = np.linspace(x0, x1, n)
    zs = np.linspace(z0, z1, n)
    X, Z = np.meshgrid(xs, zs, indexing="ij")  # [i (x), j (z)]
    Y = h(X, Z)
    P = np.stack([X, Y, Z], axis=-1)
    a = P[:-1, :-1]
    b = P[1:, :-1]
    c = P[1:, 1:]
    d = P[:-1, 1:]
    t1 = np.stack([a, c, b], axis=-2).reshape(-1, 3, 3)
    t2 = np.stack([a, d, c], axis=-2).reshape(-1, 3, 3)
    tris = np.stack([t1, t2], axis=1).reshape(-1, 3, 3)
    return tris


def _material(kd, ks, kr, n):
    return np.concatenate([np.asarray(kd, np.float64), np.asarray(ks, np.float64), np.asarray(kr, np.float64),
                           [float(n)]])


# ---------------------------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------------------------

def make_spheres_scene(seed: int = 1, num_spheres: int = 8):
    """Tiny plain stereo pair: spheres over a ground plane, one light (brute-force workload)."""
    g, m, _mir, _li, _cam = _streams(seed)
    centres = np.stack([g.uniform(-2, 2, num_spheres), g.uniform(0, 2, num_spheres), g.uniform(3, 7, num_spheres)], 1)
    radii = g.uniform(0.2, 0.6, num_spheres)
    mats = []
    for _ in range(num_spheres):
        kd = m.uniform(0.1, 0.9, 3)
        ks = m.uniform(0.0, 0.6, 3)
        mats.append(_material(kd, ks, ks, 32.0))
    mats.append(_material([0.5, 0.5, 0.5], [0, 0, 0], [0, 0, 0], 32.0))
    scene = Scene(
        name=f"spheres{num_spheres}", seed=seed,
        triangles=np.zeros((0, 3, 3), np.float32), tri_material=np.zeros(0, np.uint32),
        spheres=_f32(np.concatenate([centres, radii[:, None]], 1)),
        sphere_material=np.arange(num_spheres, dtype=np.uint32),
        planes=_f32([[0.0, 1.0, 0.0, 0.0]]), plane_material=np.asarray([num_spheres], np.uint32),
        materials=_f32(mats), lights=_f32([[-2.0, 5.0, 2.0, 1.0, 1.0, 1.0]]),
        ambient=_f32([0.05, 0.05, 0.05]), background=_f32([0.2, 0.3, 0.5]))
    cam = make_camera((0, 1, 0), forward=(0, 0, 1), convergence=5.0, width=256, height=256, max_depth=1)
    return scene, cam


def make_paper5_scene(seed: int = 6):
    """The five polyhedra of the paper's Fig. 6 experiment (Section 4): two cubes (8 vertices, 12 polygons),
    two icosahedra (12, 20) and one triangulated dodecahedron (20, 36) -- 100 triangles -- one light."""
    g, m, _mir, li, _cam = _streams(seed)
    solids = [cube(), cube(), icosahedron(), icosahedron(), dodecahedron()]
    tris, mat_ids, mats = [], [], []
    for k, (v, f) in enumerate(solids):
        R = random_rotation(g)
        s = g.uniform(0.3, 0.6)
        c = np.array([g.uniform(-2, 2), g.uniform(0.5, 2), g.uniform(3, 7)])
        w = (v / np.linalg.norm(v, axis=1).max()) @ R.T * s + c
        tris.append(w[f])
        mat_ids.append(np.full(len(f), k, np.uint32))
        mats.append(_material(m.uniform(0.1, 0.9, 3), m.uniform(0.0, 0.5, 3), m.uniform(0.0, 0.5, 3), 32.0))
    light = [li.uniform(-3, 3), li.uniform(4, 6), li.uniform(0, 2), 1.0, 1.0, 1.0]
    scene = Scene(
        name="paper5", seed=seed, triangles=_f32(np.concatenate(tris)), tri_material=np.concatenate(mat_ids),
        spheres=np.zeros((0, 4), np.float32), sphere_material=np.zeros(0, np.uint32),
        planes=np.zeros((0, 4), np.float32), plane_material=np.zeros(0, np.uint32),
        materials=_f32(mats), lights=_f32([light]), ambient=_f32([0.05] * 3), background=_f32([0.2, 0.3, 0.5]),
        info={"solids": [(len(v), len(f)) for v, f in solids]})
    cam = make_camera((0, 1, 0), forward=(0, 0, 1), convergence=5.0, width=256, height=256, max_depth=1)
    return scene, cam


def make_terrain_scene(seed, grid, extent, octaves, base_freq, n_spheres, level, radius, lights,
                       rotate=False, mirror_p=0.3, name="terrain"):
    """fBm height field over [-extent/2, extent/2] x [0, extent] plus icosphere instances.

    Materials: terrain (0.45, 0.5, 0.35) and one seeded albedo per instance, each in a plain and a
    mirror-flagged variant (kr = 0.8 grey); ks = 0.3 grey, shininess 32.  Every triangle is flagged
    mirror-like with probability ``mirror_p`` (Bernoulli, its own stream)."""
    g, m, mir, _li, _cam = _streams(seed)
    h = FBm(g, octaves=octaves, base_freq=base_freq)
    hf = heightfield_triangles(h, grid, -extent / 2, extent / 2, 0.0, float(extent))
    sv, sf = icosphere(level)
    sph = []
    margin = 1.0
    for _ in range(n_spheres):
        r = g.uniform(radius[0], radius[1])
        cx = g.uniform(-extent / 2 + margin, extent / 2 - margin)
        cz = g.uniform(margin, extent - margin)
        cy = float(h(cx, cz)) + r * g.uniform(0.2, 1.2)
        R = random_rotation(g) if rotate else np.eye(3)
        sph.append((sv @ R.T) * r + np.array([cx, cy, cz]))
    tris = [hf] + [w[sf] for w in sph]
    inst = np.concatenate([np.full(len(hf), 0, np.uint32)] + [np.full(len(sf), k + 1, np.uint32)
                                                               for k in range(n_spheres)])
    base_mats = [_material([0.45, 0.5, 0.35], [0.3] * 3, [0.0] * 3, 32.0)]
    for _ in range(n_spheres):
        base_mats.append(_material(m.uniform(0.1, 0.9, 3), [0.3] * 3, [0.0] * 3, 32.0))
    mats = []
    for bm in base_mats:
        mats.append(bm)
        mm = bm.copy()
        mm[6:9] = 0.8
        mats.append(mm)
    mirror = (mir.random(len(inst)) < mirror_p).astype(np.uint32)
    scene = Scene(
        name=name, seed=seed, triangles=_f32(np.concatenate(tris)), tri_material=(inst * 2 + mirror).astype(np.uint32),
        spheres=np.zeros((0, 4), np.float32), sphere_material=np.zeros(0, np.uint32),
        planes=np.zeros((0, 4), np.float32), plane_material=np.zeros(0, np.uint32),
        materials=_f32(mats), lights=_f32(lights), ambient=_f32([0.05] * 3), background=_f32([0.2, 0.3, 0.5]),
        info={"heightfield_tris": int(len(hf)), "instance_tris": int(len(sf) * n_spheres)})
    return scene


def make_terrain_1080p(seed: int = 2):
    """~212k triangles: 256^2-vertex fBm height field + 64 level-3 icospheres, 2 lights, depth 3, 1080p."""
    scene = make_terrain_scene(seed, grid=256, extent=16.0, octaves=6, base_freq=0.25, n_spheres=64, level=3,
                               radius=(0.3, 0.8), lights=[[-6, 8, 2, 0.7, 0.7, 0.7], [6, 6, 12, 0.7, 0.7, 0.7]],
                               name="terrain212k")
    cam = make_camera((0, 2.5, -4), target=(0, 0, 8), width=1920, height=1080, max_depth=3)
    return scene, cam


def make_terrain_3m(seed: int = 3):
    """~3.4M triangles: 1024^2-vertex fBm height field + 256 rotated level-4 icospheres, 4 lights, depth 4.

    The camera is returned at 1920x1080 per eye; ``cam.resized(3840, 2160)`` gives the 4K shape."""
    L = [[-10, 10, 6], [10, 10, 6], [-10, 8, 26], [10, 8, 26]]
    scene = make_terrain_scene(seed, grid=1024, extent=32.0, octaves=8, base_freq=0.125, n_spheres=256, level=4,
                               radius=(0.3, 1.0), lights=[p + [0.4, 0.4, 0.4] for p in L], rotate=True,
                               name="terrain3.4M")
    cam = make_camera((0, 4, -8), target=(0, 0, 16), width=1920, height=1080, max_depth=4)
    return scene, cam


def make_small_terrain(seed: int = 11, grid: int = 24, n_spheres: int = 4, level: int = 1, lights=2, depth=3):
    """A small terrain scene (about 1-2k triangles) with the large workloads' structure, for parity tests."""
    Ls = [[-6, 8, 2, 0.7, 0.7, 0.7], [6, 6, 12, 0.7, 0.7, 0.7], [-10, 8, 26, 0.4, 0.4, 0.4],
          [10, 10, 6, 0.4, 0.4, 0.4]][:lights]
    scene = make_terrain_scene(seed, grid=grid, extent=16.0, octaves=4, base_freq=0.25, n_spheres=n_spheres,
                               level=level, radius=(0.5, 1.2), lights=Ls, rotate=True, name=f"terrain_small{grid}")
    cam = make_camera((0, 2.5, -4), target=(0, 0, 8), width=96, height=64, max_depth=depth)
    return scene, cam


def make_batch_workload(seed: int = 4, n_pairs: int = 64, n_scenes: int = 8, t_min=1_000, t_max=500_000):
    """Batched rendering: n_pairs stereo pairs over n_scenes resident scenes whose triangle counts are
    log-uniform in [t_min, t_max] (terrain + icosphere scenes like the 212k workload), resolutions
    drawn from {320x240, 640x480, 1280x720, 1920x1080}, baselines U[0.03, 0.1], camera poses on seeded
    orbits around each scene, reflection depth 1-3, 2 lights.  Returns (scenes, [(scene index, camera)])."""
    g, _m, _mir, _li, cam_rng = _streams(seed)
    targets = np.exp(np.linspace(np.log(t_min), np.log(t_max), n_scenes))
    scenes = []
    for k, tgt in enumerate(targets):
        level = 1 if tgt < 5_000 else (2 if tgt < 50_000 else 3)
        per_sphere = 20 * 4 ** level
        n_sph = int(max(2, min(64, round(0.35 * tgt / per_sphere))))
        grid = int(max(6, round(np.sqrt(max(tgt - n_sph * per_sphere, 50) / 2.0)) + 1))
        sc = make_terrain_scene(seed * 100 + k, grid=grid, extent=16.0, octaves=6, base_freq=0.25,
                                n_spheres=n_sph, level=level, radius=(0.3, 0.8),
                                lights=[[-6, 8, 2, 0.7, 0.7, 0.7], [6, 6, 12, 0.7, 0.7, 0.7]], name=f"batch{k}")
        scenes.append(sc)
    sizes = [(320, 240), (640, 480), (1280, 720), (1920, 1080)]
    pairs = []
    for i in range(n_pairs):
        k = int(cam_rng.integers(n_scenes))
        w, h = sizes[int(cam_rng.integers(len(sizes)))]
        ang = cam_rng.uniform(0, 2 * np.pi)
        rad = cam_rng.uniform(7.0, 11.0)
        centre = np.array([0.0, 0.0, 8.0])
        eye = centre + np.array([rad * np.sin(ang), cam_rng.uniform(2.0, 4.0), -rad * np.cos(ang)])
        cam = make_camera(eye, target=centre, baseline=cam_rng.uniform(0.03, 0.1), width=w, height=h,
                          max_depth=int(cam_rng.integers(1, 4)))
        pairs.append((k, cam))
    return scenes, pairs


def make_serving_workload(seed: int = 5, n_requests: int = 200, rate_hz: float = 100.0, n_scenes: int = 8,
                          t_min=10_000, t_max=2_000_000, sizes=((640, 480), (1280, 720), (1920, 1080), (3840, 2160))):
    """Serving: Poisson arrivals at `rate_hz` of requests (scene id, stereo camera) over n_scenes resident
    scenes of log-uniform triangle counts in [t_min, t_max]; resolution drawn from `sizes`, baseline
    U[0.03, 0.1], reflection depth 1-4, pose on a seeded orbit.  Returns (scenes, [(arrival s, scene, cam)])."""
    scenes, _ = make_batch_workload(seed=seed, n_pairs=0, n_scenes=n_scenes, t_min=t_min, t_max=t_max)
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed).spawn(6)[5]))
    t = 0.0
    reqs = []
    for _ in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        k = int(rng.integers(n_scenes))
        w, h = sizes[int(rng.integers(len(sizes)))]
        ang = rng.uniform(0, 2 * np.pi)
        rad = rng.uniform(7.0, 11.0)
        centre = np.array([0.0, 0.0, 8.0])
        eye = centre + np.array([rad * np.sin(ang), rng.uniform(2.0, 4.0), -rad * np.cos(ang)])
        cam = make_camera(eye, target=centre, baseline=rng.uniform(0.03, 0.1), width=w, height=h,
                          max_depth=int(rng.integers(1, 5)))
        reqs.append((t, k, cam))
    return scenes, reqs


WORKLOADS = {
    "spheres8_256": make_spheres_scene,
    "paper5": make_paper5_scene,
    "terrain212k_1080p": make_terrain_1080p,
    "terrain3.4M_1080p": make_terrain_3m,
}


def sample_paths(cam: StereoCamera, n: int, seed: int) -> np.ndarray:
    """Seeded uniform sample (without replacement) of path ids eye*H*W + y*W + x over both eyes."""
    total = 2 * cam.width * cam.height
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    n = min(int(n), total)
    return np.sort(rng.choice(total, size=n, replace=False)).astype(np.int64)


def digest(scene: Scene, cam: StereoCamera) -> str:
    """SHA-256 over a scene's arrays and a camera's fields: two runs (or two machines) that report the same
    digest rendered the same input."""
    import hashlib
    h = hashlib.sha256()
    for a in (scene.triangles, scene.tri_material, scene.spheres, scene.sphere_material, scene.planes,
              scene.plane_material, scene.materials, scene.lights, scene.ambient, scene.background):
        h.update(np.ascontiguousarray(a).tobytes())
    for v in (cam.center, cam.forward, cam.up):
        h.update(np.asarray(v, np.float32).tobytes())
    h.update(np.asarray([cam.hfov_deg, cam.baseline, cam.convergence], np.float32).tobytes())
    h.update(np.asarray([cam.width, cam.height, cam.max_depth], np.int64).tobytes())
    return h.hexdigest()
