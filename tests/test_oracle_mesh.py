"""Pins of the surface-extraction oracle (marching tetrahedra on the SDF lattice).

Fixed by geometry, not by the oracle's formulas: a linear SDF has its zero
crossings exactly on its plane, so every vertex lies on it and the triangles
tile the plane's section of the lattice box; a sphere's vertices lie within
O(h^2) of it, its area is close to 4 pi r^2, and the surface is closed (every
edge shared by two triangles); single inside corners give known counts.
"""
import collections

import numpy as np
import pytest

from oracle import mesh as MS


def _area(tris):
    return 0.5 * np.linalg.norm(np.cross(tris[:, 1] - tris[:, 0], tris[:, 2] - tris[:, 0]), axis=1).sum()


def test_plane_vertices_lie_on_the_plane_and_tile_its_section():
    h, dims, p0 = 0.1, (11, 9, 7), (0.0, 0.0, 0.0)
    x = MS.lattice_points(p0, h, dims)
    n = np.array([1.0, 0.3, -0.2])
    n /= np.linalg.norm(n)
    c = 0.52
    phi = (x @ n - c).reshape(dims[2], dims[1], dims[0])
    tris = MS.marching_tetrahedra(phi, p0, h)
    assert len(tris) > 0
    np.testing.assert_allclose(tris.reshape(-1, 3) @ n, c, atol=1e-12)


def test_axis_plane_area_equals_the_box_section():
    h, dims, p0 = 0.05, (9, 12, 10), (-0.2, 0.1, 0.3)
    x = MS.lattice_points(p0, h, dims)
    phi = (x[:, 0] - (-0.2 + 0.137)).reshape(dims[2], dims[1], dims[0])
    tris = MS.marching_tetrahedra(phi, p0, h)
    assert _area(tris) == pytest.approx((dims[1] - 1) * h * (dims[2] - 1) * h, rel=1e-12)


def test_sphere_is_closed_near_its_radius_with_its_area():
    h, r = 0.04, 0.5
    dims = (33, 33, 33)
    p0 = (-0.64, -0.64, -0.64)
    x = MS.lattice_points(p0, h, dims)
    phi = (np.linalg.norm(x, axis=1) - r).reshape(dims[2], dims[1], dims[0])
    tris = MS.marching_tetrahedra(phi, p0, h)
    rad = np.linalg.norm(tris.reshape(-1, 3), axis=1)
    assert np.max(np.abs(rad - r)) < h * h / r
    assert _area(tris) == pytest.approx(4 * np.pi * r * r, rel=0.02)
    edges = collections.Counter()
    q = np.round(tris / 1e-9).astype(np.int64)
    for t in q:
        for a, b in ((0, 1), (1, 2), (2, 0)):
            e = tuple(sorted((tuple(t[a]), tuple(t[b]))))
            edges[e] += 1
    assert set(edges.values()) == {2}


@pytest.mark.parametrize("corner,count", [(0, 6), (7, 6), (1, 2), (3, 2), (5, 2)])
def test_single_inside_corner(corner, count):
    phi = np.ones((2, 2, 2))
    bx, by, bz = corner & 1, (corner >> 1) & 1, (corner >> 2) & 1
    phi[bz, by, bx] = -1.0
    tris = MS.marching_tetrahedra(phi, (0.0, 0.0, 0.0), 1.0)
    assert len(tris) == count
    # every vertex is the midpoint of an edge at the inside corner
    corner_pos = np.array([bx, by, bz], dtype=float)
    d = np.linalg.norm(tris.reshape(-1, 3) - corner_pos, axis=1)
    assert np.all((np.abs(d - 0.5) < 1e-12) | (np.abs(d - np.sqrt(2) / 2) < 1e-12) | (np.abs(d - np.sqrt(3) / 2) < 1e-12))


def test_no_crossing_no_triangles():
    phi = np.full((4, 5, 6), 0.3)
    assert MS.marching_tetrahedra(phi, (0, 0, 0), 0.1).shape == (0, 3, 3)
