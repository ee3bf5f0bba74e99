"""The numpy Morton-code reference that the GPU build's triangle order is checked against: pinned on
triangles whose box centroids sit at the corners and the centre of the centroids' bounds."""
import numpy as np

from tests.test_gpu_render import _morton_keys


def _tri_at(c, h=0.01):
    c = np.asarray(c, np.float64)
    return [c + [-h, 0, 0], c + [h, 0, 0], c + [0, 0, h]]  # box centroid (c.x, c.y, c.z + h/2)


def test_morton_codes_at_corners_and_centre():
    h = 0.01
    corners = [(0, 0, 0), (4, 0, 0), (0, 4, 0), (0, 0, 4), (4, 4, 4), (2, 2, 2)]
    keys = _morton_keys(np.array([_tri_at(c, h) for c in corners]))
    x_bits = sum(1 << (3 * b + 2) for b in range(21))
    y_bits, z_bits = x_bits >> 1, x_bits >> 2
    # the low corner is cell 0 on every axis; the high corner the last cell, 2^21 - 1
    assert keys[0] == 0 and keys[1] == x_bits and keys[2] == y_bits and keys[3] == z_bits
    assert keys[4] == (1 << 63) - 1
    # the centre is cell 2^20 on each axis: only the top bit of each axis is set
    assert keys[5] == (1 << 62) | (1 << 61) | (1 << 60)
    # a stable sort keeps equal codes in input order
    dup = _morton_keys(np.array([_tri_at(c, h) for c in [(4, 4, 4), (0, 0, 0), (4, 4, 4), (0, 0, 0)]]))
    assert list(np.argsort(dup, kind="stable")) == [1, 3, 0, 2]
