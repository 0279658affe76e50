"""Closed-form pins on the unit sphere (oracle + its near-field fixture).

The oracle's product-facing entries cover regular pairs only; near pairs here
come from the fixture (analytic inner integral, subdivided outer rule).  With
both, the P0 Laplace matrices on icospheres must satisfy

  * sum_ij S_ij -> int_S int_S 1/(4 pi |x-y|) = 4 pi  (the single-layer
    potential of unit density on the unit sphere is 1 on the sphere), with
    O(h^2) convergence over refinement levels;
  * generalized eigenvalues of (S, M), M = diag(|T_i|), approach the
    eigenvalues 1/(2l+1) of the single-layer operator on the unit sphere,
    with multiplicity 2l+1;
  * sum_j K_ij = -1/2 int psi_i = -J_i/4 on the closed polyhedron: the
    double-layer potential of unit density is -1/2 at every point of a flat
    face (solid angle 2 pi), for outward normals.
The fixture itself is pinned first against brute-force integration and the
solid-angle sum of a closed polyhedron.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1711_01897_amd import inputs

TRI = [np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.0, 0.0]), np.array([0.2, 1.1, 0.0])]


def numeric_over_tri(f, level=6):
    xi, eta, w = O.subdivided_rule(level)
    a, b, c = TRI
    pts = a + xi[:, None] * (b - a) + eta[:, None] * (c - a)
    J = np.linalg.norm(np.cross(b - a, c - a))
    return J * float(np.sum(w * f(pts)))


@pytest.mark.parametrize("x", [[0.3, 0.2, 0.7], [1.5, -0.4, 0.2], [0.1, 0.1, -0.05], [1.5, -0.3, 0.0],
                               [-0.7, 2.0, 0.0]])
def test_fixture_potential_vs_brute_force(x):
    x = np.array(x)
    ref = numeric_over_tri(lambda p: 1.0 / np.linalg.norm(p - x, axis=1))
    assert abs(O.tri_potential(*TRI, x) - ref) < 1e-6 * abs(ref)


@pytest.mark.parametrize("x", [[0.3, 0.2, 0.7], [1.5, -0.4, 0.2], [0.2, 0.3, -0.5]])
def test_fixture_solid_angle_vs_brute_force(x):
    x = np.array(x)
    n = np.array([0.0, 0.0, 1.0])
    ref = numeric_over_tri(lambda p: ((x - p) @ n) / np.linalg.norm(p - x, axis=1) ** 3)
    assert abs(-O.tri_solid_angle(*TRI, x) - ref) < 1e-6 * abs(ref)


def test_fixture_solid_angles_of_closed_surface():
    xyz, tri = inputs.icosphere(1)
    inside = np.array([0.1, -0.2, 0.15])
    outside = np.array([1.4, 0.3, -0.2])
    s_in = sum(O.tri_solid_angle(*xyz[t], inside) for t in tri)
    s_out = sum(O.tri_solid_angle(*xyz[t], outside) for t in tri)
    assert abs(s_in - 4 * math.pi) < 1e-12
    assert abs(s_out) < 1e-12


def sphere_matrices(level, op):
    xyz, tri = inputs.icosphere(level)
    m = O.OracleMesh(xyz, tri, 6)
    h = inputs.mean_edge_length(xyz, tri)
    return m, m.p0_matrix_with_nearfield(op, 3.0 * h, 3)


def test_sphere_single_layer_sum():
    errs = []
    for level in (2, 3):
        _, S = sphere_matrices(level, O.LAPLACE_SLP)
        errs.append(abs(S.sum() - 4.0 * math.pi) / (4.0 * math.pi))
    assert errs[-1] < 1e-2
    assert 3.0 < errs[0] / errs[1] < 5.0  # O(h^2)


def test_sphere_single_layer_spectrum():
    m, S = sphere_matrices(3, O.LAPLACE_SLP)
    J, _, _ = m.geometry()
    Mh = 1.0 / np.sqrt(J / 2.0)
    ev = np.linalg.eigvalsh(Mh[:, None] * (0.5 * (S + S.T)) * Mh[None, :])[::-1]
    start = 0
    for l in range(4):
        group = ev[start:start + 2 * l + 1]
        assert np.abs(group * (2 * l + 1) - 1.0).max() < 0.02, (l, group)
        start += 2 * l + 1
    # the next eigenvalue belongs to l = 4
    assert abs(ev[start] * 9 - 1.0) < 0.05


@pytest.mark.parametrize("level", [2, 3])
def test_double_layer_constant_density_identity(level):
    m, K = sphere_matrices(level, O.LAPLACE_DLP)
    J, _, _ = m.geometry()
    rel = np.abs(K.sum(axis=1) + J / 4.0) / (J / 4.0)
    assert rel.max() < 1e-6


def test_fixture_and_regular_entries_agree_when_separated():
    xyz, tri = inputs.icosphere(3)
    m = O.OracleMesh(xyz, tri, 6)
    cen = xyz[tri].mean(axis=1)
    j = int(np.argmax(np.linalg.norm(cen - cen[0], axis=1)))
    for op in (O.LAPLACE_SLP, O.LAPLACE_DLP):
        reg = m.entries(op, O.P0, 0.0, [0], [j])[0, 0]
        nf = m.nearfield_entry(op, 0, j, 2)
        assert abs(reg - nf) < 1e-9 * abs(nf)
