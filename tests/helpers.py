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
    out = {k: np.concatenate([p[k] for p in parts]) for k in parts[0] if k != "ray_counts"}
    out["ray_counts"] = sum(p["ray_counts"] for p in parts)
    return out
