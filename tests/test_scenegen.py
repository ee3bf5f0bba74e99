"""The seeded scene generator: determinism, the counts the workloads are defined by, and
well-formed solids (test input quality, not ray-tracing arithmetic)."""
from collections import Counter

import numpy as np
import pytest

import scenegen as sg


def _closed_and_planar(v, f, faces_per_polygon=1):
    edges = Counter()
    for a, b, c in f:
        for e in ((a, b), (b, c), (c, a)):
            edges[tuple(sorted(e))] += 1
    assert set(edges.values()) == {2}, "every edge is shared by exactly two triangles"
    # outward orientation and positive area
    cen = v.mean(0)
    for a, b, c in f:
        n = np.cross(v[b] - v[a], v[c] - v[a])
        assert np.linalg.norm(n) > 1e-9
        assert n @ ((v[a] + v[b] + v[c]) / 3 - cen) > 0
    # Euler characteristic of a sphere: V - E + F = 2
    assert len(v) - len(edges) + len(f) == 2


@pytest.mark.parametrize("solid,counts", [(sg.cube, (8, 12)), (sg.icosahedron, (12, 20)),
                                          (sg.dodecahedron, (20, 36))])
def test_platonic_solids(solid, counts):
    v, f = solid()
    assert (len(v), len(f)) == counts
    _closed_and_planar(v, f)
    # polygons are planar: triangles of one polygon share a normal; the number of distinct
    # normals is the number of faces of the solid (6, 20, 12)
    normals = {tuple(np.round(np.cross(v[b] - v[a], v[c] - v[a]) / np.linalg.norm(np.cross(v[b] - v[a], v[c] - v[a])),
                              9)) for a, b, c in f}
    assert len(normals) == {12: 6, 20: 20, 36: 12}[len(f)]


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_icosphere_counts(level):
    v, f = sg.icosphere(level)
    assert len(f) == 20 * 4 ** level and len(v) == 10 * 4 ** level + 2
    np.testing.assert_allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-12)
    _closed_and_planar(v, f)


def test_workload_counts_and_determinism():
    s1, c1 = sg.make_terrain_1080p()
    assert s1.num_triangles == 211970 and s1.info["heightfield_tris"] == 2 * 255 * 255
    assert (c1.width, c1.height, c1.max_depth, s1.num_lights) == (1920, 1080, 3, 2)
    s2, _ = sg.make_terrain_1080p()
    assert np.array_equal(s1.triangles, s2.triangles) and np.array_equal(s1.tri_material, s2.tri_material)
    mirror = s1.materials[s1.tri_material][:, 6] > 0
    assert 0.28 < mirror.mean() < 0.32
    s, c = sg.make_spheres_scene()
    assert (s.num_spheres, s.num_planes, c.width, c.max_depth) == (8, 1, 256, 1)
    assert np.all((s.spheres[:, 3] >= 0.2) & (s.spheres[:, 3] <= 0.6))


def test_heightfield_faces_up():
    h = sg.FBm(np.random.default_rng(0), octaves=3, base_freq=0.5)
    t = sg.heightfield_triangles(h, 9, -1, 1, 0, 2)
    n = np.cross(t[:, 1] - t[:, 0], t[:, 2] - t[:, 0])
    assert len(t) == 2 * 8 * 8 and np.all(n[:, 1] > 0)
    assert np.all(np.abs(h(np.linspace(-5, 5, 101), np.linspace(0, 9, 101))) <= 1.0)


def test_sample_paths_seeded():
    _, cam = sg.make_spheres_scene()
    a = sg.sample_paths(cam, 100, seed=3)
    assert np.array_equal(a, sg.sample_paths(cam, 100, seed=3)) and len(np.unique(a)) == 100
    assert a.min() >= 0 and a.max() < 2 * 256 * 256
