"""Seeded mesh generators: counts, closedness, orientation, determinism."""
import math

import numpy as np
import pytest

from paper_1711_01897_amd import inputs


def closed_and_consistent(xyz, tri):
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]]).astype(np.int64)
    nv = xyz.shape[0]
    key = e[:, 0] * nv + e[:, 1]
    rkey = e[:, 1] * nv + e[:, 0]
    return len(np.unique(key)) == len(key) and np.array_equal(np.sort(key), np.sort(rkey))


def outward_fraction(xyz, tri):
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    N = np.cross(b - a, c - a)
    return float(np.mean(np.einsum("ij,ij->i", N, (a + b + c) / 3 - xyz.mean(0)) > 0))


@pytest.mark.parametrize("level,nt,nv", [(0, 20, 12), (3, 1280, 642), (4, 5120, 2562)])
def test_icosphere_counts(level, nt, nv):
    xyz, tri = inputs.icosphere(level)
    assert tri.shape == (nt, 3) and xyz.shape == (nv, 3)
    assert np.allclose(np.linalg.norm(xyz, axis=1), 1.0)
    assert closed_and_consistent(xyz, tri)
    assert outward_fraction(xyz, tri) == 1.0


def test_spheroid_near_uniform():
    xyz, tri = inputs.spheroid(10.0, 1.0, 20000)
    assert abs(tri.shape[0] - 20000) <= 200
    assert closed_and_consistent(xyz, tri)
    assert outward_fraction(xyz, tri) == 1.0
    r = (xyz[:, 0] / 10.0) ** 2 + xyz[:, 1] ** 2 + xyz[:, 2] ** 2
    assert np.allclose(r, 1.0)
    e = inputs.edges(tri)
    el = np.linalg.norm(xyz[e[:, 0]] - xyz[e[:, 1]], axis=1)
    assert el.max() / el.min() < 2.5


def test_capped_cylinder_seeded_jitter():
    a = inputs.capped_cylinder(1.0, 16.0, 20000, jitter=0.01, seed=0)
    b = inputs.capped_cylinder(1.0, 16.0, 20000, jitter=0.01, seed=0)
    c = inputs.capped_cylinder(1.0, 16.0, 20000, jitter=0.0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert abs(a[1].shape[0] - 20000) <= 200
    assert closed_and_consistent(*a)
    assert outward_fraction(*a) == 1.0
    h = inputs.mean_edge_length(*c)
    assert np.abs(a[0] - c[0]).max() <= 0.011 * h * 1.2


def test_wavenumber_recipe():
    xyz, tri = inputs.icosphere(3)
    h = inputs.mean_edge_length(xyz, tri)
    assert abs(inputs.wavenumber(xyz, tri, 10.0) - 2 * math.pi / (10 * h)) < 1e-12
