"""Small hand-built scenes for tests (test inputs only, no ray-tracing arithmetic)."""
import numpy as np

from scenegen import Scene, make_camera


def material(kd=(0.5, 0.5, 0.5), ks=(0.0, 0.0, 0.0), kr=(0.0, 0.0, 0.0), n=32.0):
    return list(kd) + list(ks) + list(kr) + [n]


def make_scene(tris=None, tri_mat=None, spheres=None, sphere_mat=None, planes=None, plane_mat=None, materials=None,
               lights=None, ambient=(0.0, 0.0, 0.0), background=(0.2, 0.3, 0.5), name="custom"):
    tris = np.zeros((0, 3, 3)) if tris is None else np.asarray(tris, np.float64).reshape(-1, 3, 3)
    spheres = np.zeros((0, 4)) if spheres is None else np.asarray(spheres, np.float64).reshape(-1, 4)
    planes = np.zeros((0, 4)) if planes is None else np.asarray(planes, np.float64).reshape(-1, 4)
    if tri_mat is None:
        tri_mat = np.zeros(len(tris))
    if sphere_mat is None:
        sphere_mat = np.zeros(len(spheres))
    if plane_mat is None:
        plane_mat = np.zeros(len(planes))
    if materials is None:
        materials = [material()]
    if lights is None:
        lights = np.zeros((0, 6))
    return Scene(
        name=name, seed=0, triangles=np.ascontiguousarray(tris, np.float32),
        tri_material=np.ascontiguousarray(tri_mat, np.uint32),
        spheres=np.ascontiguousarray(spheres, np.float32), sphere_material=np.ascontiguousarray(sphere_mat, np.uint32),
        planes=np.ascontiguousarray(planes, np.float32), plane_material=np.ascontiguousarray(plane_mat, np.uint32),
        materials=np.ascontiguousarray(np.asarray(materials, np.float64).reshape(-1, 10), np.float32),
        lights=np.ascontiguousarray(np.asarray(lights, np.float64).reshape(-1, 6), np.float32),
        ambient=np.asarray(ambient, np.float32), background=np.asarray(background, np.float32))


def mono_camera(center=(0, 1, 0), forward=(0, 0, 1), up=(0, 1, 0), width=64, height=48, depth=1, hfov=60.0,
                baseline=0.0, convergence=0.0):
    return make_camera(center, forward=forward, up=up, hfov_deg=hfov, baseline=baseline, convergence=convergence,
                       width=width, height=height, max_depth=depth)


def f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def oracle_sampled(scene, cam, samples, chunk=2048, say=print):
    """The oracle on a large sample of paths, in chunks with a progress line after each (a long oracle run
    stays visibly alive); the result equals one call over the whole sample."""
    import oracle
    samples = np.asarray(samples, np.int64)
    parts = []
    for lo in range(0, len(samples), chunk):
        parts.append(oracle.render(scene, cam, samples=samples[lo:lo + chunk]))
        say(f"[oracle] {min(lo + chunk, len(samples))}/{len(samples)} paths")
    out = {k: np.concatenate([p[k] for p in parts]) for k in parts[0] if k not in ("ray_counts", "seconds")}
    out["ray_counts"] = sum(p["ray_counts"] for p in parts)
    out["seconds"] = {k: sum(p["seconds"][k] for p in parts) for k in parts[0]["seconds"]}
    return out


def coincident_scene():
    """Hundreds of copies of one triangle (equal boxes, exact ties in t decided by the smaller id), zero-area
    triangles (collinear with integer coordinates, and point-like: never hit) and a mirror floor."""
    rng = np.random.default_rng(7)
    front = [[-1.0, 0.0, 4.0], [1.0, 0.0, 4.0], [0.0, 2.0, 4.0]]
    tris = [front] * 300
    for _ in range(60):
        a = rng.integers(-3, 4, 3).astype(np.float64) + [0, 1, 5]
        axis = np.eye(3)[rng.integers(0, 3)]
        tris.append([list(a), list(a + axis), list(a + 2 * axis)])
        tris.append([list(a)] * 3)
    tris.append([[-8, -0.5, 0], [8, -0.5, 0], [0, -0.5, 16]])
    mats = [0] * 300 + [0] * 120 + [1]
    scene = make_scene(tris=tris, tri_mat=mats, lights=[[0, 6, 1, 1, 1, 1], [3, 4, 2, 0.5, 0.5, 0.5]],
                       materials=[material(), material(kd=(0.2, 0.2, 0.2), kr=(0.6, 0.6, 0.6))],
                       ambient=(0.05,) * 3, name="coincident")
    cam = mono_camera(center=(0, 1, 0), width=48, height=32, depth=3, baseline=0.065, convergence=4.0)
    return scene, cam


def flat_scene():
    """Every triangle in the plane y = 0 (boxes of zero height), a mirror stripe, grazing rays from an eye
    0.25 over the plane, and an axis-parallel centre column (odd width)."""
    n = 24
    tris, mats = [], []
    for i in range(n):
        for j in range(n):
            x0, z0 = -6.0 + 0.5 * i, 0.5 * j
            q = [[x0, 0.0, z0], [x0 + 0.5, 0.0, z0], [x0 + 0.5, 0.0, z0 + 0.5], [x0, 0.0, z0 + 0.5]]
            tris += [[q[0], q[1], q[2]], [q[0], q[2], q[3]]]
            mats += [1 if i % 6 == 0 else 0] * 2
    scene = make_scene(tris=tris, tri_mat=mats, lights=[[0, 3, 4, 1, 1, 1], [-4, 0.5, 8, 0.6, 0.6, 0.6]],
                       materials=[material(kd=(0.7, 0.6, 0.5), ks=(0.3, 0.3, 0.3), n=16),
                                  material(kd=(0.1, 0.1, 0.1), kr=(0.8, 0.8, 0.8))],
                       ambient=(0.05,) * 3, name="flat")
    cam = mono_camera(center=(0, 0.25, -1), width=41, height=21, depth=2, baseline=0.065, convergence=3.0)
    return scene, cam


def corners_scene():
    """Boxes whose clustering merges tie exactly: a box B = [0,2]^3 (one triangle cutting its corner), tiny
    triangles at B's low and high corners and a distant triangle, copies at other places, a grid of equal
    mirror quads."""
    base = [[[2, 0, 0], [0, 2, 0], [0, 0, 2]],
            [[0, 0, 0], [0.01, 0, 0], [0, 0.01, 0.01]],
            [[2, 2, 2], [1.99, 2, 2], [2, 1.99, 1.99]]]
    tris = [[[-50, -50, -50], [-49, -50, -50], [-50, -49, -49]]]
    for off in ((0, 0, 0), (4, 0, 1), (-4, 1, 3), (2, 3, 6)):
        tris += [[[v[0] + off[0], v[1] + off[1], v[2] + off[2]] for v in t] for t in base]
    for i in range(12):
        for j in range(6):
            x, z = -6.0 + i, 8.0 + j
            tris += [[[x, -0.5, z], [x + 1, -0.5, z], [x + 1, -0.5, z + 1]], [[x, -0.5, z], [x + 1, -0.5, z + 1],
                                                                            [x, -0.5, z + 1]]]
    mats = [0] * (1 + 12) + [1] * (2 * 72)
    scene = make_scene(tris=tris, tri_mat=mats, lights=[[1, 6, -2, 1, 1, 1], [-3, 4, 3, 0.5, 0.5, 0.5]],
                       materials=[material(kd=(0.7, 0.5, 0.3), ks=(0.3, 0.3, 0.3)),
                                  material(kd=(0.2, 0.3, 0.2), kr=(0.5, 0.5, 0.5))],
                       ambient=(0.05,) * 3, name="corners")
    cam = mono_camera(center=(1, 2.5, -6), forward=(0, -0.2, 1), width=64, height=40, depth=2, baseline=0.065,
                      convergence=8.0)
    return scene, cam


def nested_scene():
    """150 nested triangles of growing size (boxes [0, 1.2^k]^3, the largest within the 1e12 coordinate
    limit): a tree over them is a chain."""
    tris, s = [], 1.0
    for _ in range(150):
        tris.append([[s, 0, 0], [0, s, 0], [0, 0, s]])
        s *= 1.2
    scene = make_scene(tris=tris, lights=[[3, 4, -2, 1, 1, 1]], materials=[material(kd=(0.6, 0.5, 0.4))],
                       ambient=(0.05,) * 3, name="nested")
    cam = mono_camera(center=(2, 2, -3), forward=(-0.1, -0.2, 1), width=48, height=32, depth=1)
    return scene, cam
