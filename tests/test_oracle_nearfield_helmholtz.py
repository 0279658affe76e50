"""Pins of the oracle's Helmholtz near-field fixture (P0 single and double
layer of Eq. slp/dlp with g = e^{ikr}/(4 pi r)) for vertex-sharing pairs.

The fixture expands the kernel around r = 0, integrates 1/r, r (and the
solid angle) over the trial triangle in closed form and the O(r^2)
remainder with a subdivided rule.  Pinned here against what does not share
that decomposition:
  * int_T |x - y| dy (closed form) against a fine subdivided rule at points
    where the integrand is smooth;
  * separated pairs: the whole Helmholtz part against a product rule of the
    full kernel (smooth there), so a dropped or mis-signed term of the
    expansion shows;
  * vertex-sharing pairs: the imaginary part, sin(kr)/r and
    (sin kr - kr cos kr)/r^3 being smooth, against the same product rule; the
    real part of the k-dependent correction against the product rule within
    that rule's error for a kernel with a cusp at r = 0;
  * k -> 0 returns the Laplace fixture.
"""
import numpy as np
import pytest

import oracle as O
from paper_1711_01897_amd import inputs


@pytest.fixture(scope="module")
def ico2():
    xyz, tri = inputs.icosphere(2)
    return xyz, tri, O.OracleMesh(xyz, tri, 6)


@pytest.mark.parametrize("x", [[0.4, 0.3, 0.5], [0.5, 0.05, 0.2], [2.0, 1.0, 0.0], [-0.3, -0.2, 0.01],
                               [5.0, 5.0, 5.0]])
def test_moment_r_closed_form_vs_brute_force(x):
    v0, v1, v2 = np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.1, 0.0]), np.array([0.3, 0.8, 0.05])
    xi, eta, w = O.subdivided_rule(6)
    Y = v0 + xi[:, None] * (v1 - v0) + eta[:, None] * (v2 - v0)
    J = np.linalg.norm(np.cross(v1 - v0, v2 - v0))
    bf = J * np.sum(w * np.linalg.norm(Y - np.asarray(x), axis=1))
    assert abs(O.tri_moment_r(v0, v1, v2, x) - bf) <= 1e-12 * bf


def product_rule(xyz, tri, op, k, i, j, level=3):
    """Real part of the k-dependent correction and the imaginary part of the
    P0 entry by the subdivided 6-point rule on both triangles."""
    xi, eta, w = O.subdivided_rule(level)
    a, b, c = xyz[tri[i]]
    u0, u1, u2 = xyz[tri[j]]
    X = a + xi[:, None] * (b - a) + eta[:, None] * (c - a)
    Y = u0 + xi[:, None] * (u1 - u0) + eta[:, None] * (u2 - u0)
    Ji = np.linalg.norm(np.cross(b - a, c - a))
    Nj = np.cross(u1 - u0, u2 - u0)
    Jj = np.linalg.norm(Nj)
    D = X[:, None, :] - Y[None, :, :]
    r = np.linalg.norm(D, axis=2)
    r0 = r == 0.0
    r = np.where(r0, 1.0, r)
    z = k * r
    if op == O.HELMHOLTZ_SLP:
        re, im = (np.cos(z) - 1.0) / r, np.where(r0, k, np.sin(z) / r)
    else:
        hgt = D @ (Nj / Jj)
        re = (np.cos(z) + z * np.sin(z) - 1.0) * hgt / r ** 3
        im = (np.sin(z) - z * np.cos(z)) * hgt / r ** 3
    re, im = np.where(r0, 0.0, re), np.where(r0 & (op != O.HELMHOLTZ_SLP), 0.0, im)
    W = w[:, None] * w[None, :] * Ji * Jj / (4 * np.pi)
    return np.sum(W * re), np.sum(W * im)


@pytest.mark.parametrize("op", [O.HELMHOLTZ_SLP, O.HELMHOLTZ_DLP])
@pytest.mark.parametrize("k", [0.8, 6.0])
def test_separated_pairs_vs_product_rule(ico2, op, k):
    xyz, tri, om = ico2
    cen = xyz[tri].mean(1)
    h = inputs.mean_edge_length(xyz, tri)
    d = np.linalg.norm(cen[0] - cen, axis=1)
    cols = [int(np.argmin(abs(d - f * h))) for f in (3, 6)]
    nf = om.nearfield_entries(op, k, [0] * len(cols), cols, 3, 3)
    lap = om.nearfield_entries(op - 2, 0.0, [0] * len(cols), cols, 3, 3)
    for q, j in enumerate(cols):
        re, im = product_rule(xyz, tri, op, k, 0, j)
        ref = lap[q].real + re + 1j * im
        assert abs(nf[q] - ref) <= 1e-10 * abs(ref), (j, nf[q], ref)


@pytest.mark.parametrize("op", [O.HELMHOLTZ_SLP, O.HELMHOLTZ_DLP])
@pytest.mark.parametrize("k", [2.0, 8.0])
def test_adjacent_pairs_vs_product_rule(ico2, op, k):
    xyz, tri, om = ico2
    adj = [j for j in range(tri.shape[0]) if set(tri[0]) & set(tri[j])]
    assert len(adj) == 12   # triangle 0 touches one of the valence-5 vertices
    nf = om.nearfield_entries(op, k, [0] * len(adj), adj, 3, 3)
    lap = om.nearfield_entries(op - 2, 0.0, [0] * len(adj), adj, 3, 3)
    pr = np.array([product_rule(xyz, tri, op, k, 0, j) for j in adj])
    # the imaginary part is smooth: both rules are accurate
    assert np.abs(nf.imag - pr[:, 1]).max() <= 1e-12 * np.abs(nf.imag).max()
    # the real correction has a cusp at r = 0: the product rule's error (~5e-5)
    corr = nf.real - lap.real
    assert np.abs(corr - pr[:, 0]).max() <= 2e-4 * np.abs(corr).max()


def test_small_k_returns_laplace(ico2):
    """k -> 0: real parts tend to the Laplace fixture, the imaginary part of
    the single layer to k |T_i| |T_j| / (4 pi) (Im g = k/(4 pi) + O(k^3 r^2)),
    that of the double layer to zero (O(k^3))."""
    xyz, tri, om = ico2
    adj = [j for j in range(tri.shape[0]) if set(tri[0]) & set(tri[j])]
    area = 0.5 * np.linalg.norm(np.cross(xyz[tri[:, 1]] - xyz[tri[:, 0]], xyz[tri[:, 2]] - xyz[tri[:, 0]]), axis=1)
    k = 1e-6
    for op in (O.HELMHOLTZ_SLP, O.HELMHOLTZ_DLP):
        nf = om.nearfield_entries(op, k, [0] * len(adj), adj, 2, 2)
        lap = om.nearfield_entries(op - 2, 0.0, [0] * len(adj), adj, 2, 2)
        assert np.abs(nf.real - lap.real).max() <= 1e-10 * np.abs(lap).max()
        im_ref = k * area[0] * area[adj] / (4 * np.pi) if op == O.HELMHOLTZ_SLP else np.zeros(len(adj))
        assert np.abs(nf.imag - im_ref).max() <= 1e-12 * k * area[0] ** 2
        assert all(abs(lap[q].real - om.nearfield_entry(op - 2, 0, j, 2)) <= 1e-15 * abs(lap).max()
                   for q, j in enumerate(adj))
