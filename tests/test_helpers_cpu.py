"""Host-side test helpers."""
import numpy as np

import oracle
import scenegen as sg
from tests.helpers import oracle_sampled


def test_chunked_oracle_equals_one_call():
    scene, cam = sg.make_small_terrain(seed=3, grid=12, n_spheres=2, level=1, lights=2, depth=2)
    cam = cam.resized(24, 16)
    samples = sg.sample_paths(cam, 300, seed=5)
    one = oracle.render(scene, cam, samples=samples)
    parts = oracle_sampled(scene, cam, samples, chunk=77, say=lambda *a: None)
    assert set(one) == set(parts)
    for k in set(one) - {"seconds"}:  # wall times differ
        assert np.array_equal(one[k], parts[k], equal_nan=k == "hit_cos"), k  # NaN where a ray misses
