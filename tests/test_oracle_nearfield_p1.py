"""Pins of the oracle's P1 near-field fixtures: 3 x 3 local matrices of the
Laplace single and double layer (and, at the end, of the Helmholtz single
and double layer, whose expansion adds int (y - rho) R; pinned the same way
plus the smooth imaginary part and k -> 0) for a triangle pair,
M[a][b] = int_T phi_a int_S psi_b K, from the closed-form potentials of a
linear density (the constant part's potential or solid angle, plus the
in-plane vector moments int (y - rho)/R and int (y - rho)/R^3 from edge
integrals), outer rule on 4^L sub-triangles.

Pinned against what does not share that construction:
  * the vector moments against a fine subdivided rule where the integrand
    is smooth;
  * separated pairs: M against a product rule with the hat functions as
    weights (smooth kernel there);
  * the local matrices sum to the P0 near-field value (partition of unity);
  * single layer: M(T, S) = M(S, T)^T on vertex-sharing pairs, up to the
    outer rule's error;
  * closed surface: with every pair included, the P1 double layer applied
    to the constant is -1/2 times the hat function's integral (the solid
    angle of a closed polyhedron is 2 pi at face points), and the single
    layer of the unit sphere's constant density is 1 on the sphere (row sums
    converge like h^2 on the polyhedral icospheres).
"""
import numpy as np
import pytest

import oracle as O
from paper_1711_01897_amd import inputs


@pytest.fixture(scope="module")
def ico2():
    xyz, tri = inputs.icosphere(2)
    return xyz, tri, O.OracleMesh(xyz, tri, 6)


@pytest.mark.parametrize("x", [[0.4, 0.3, 0.5], [2.0, 1.0, 0.0], [-0.3, -0.2, 0.31], [5.0, 5.0, 5.0]])
def test_vector_moments_vs_brute_force(x):
    v0, v1, v2 = np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.1, 0.0]), np.array([0.3, 0.8, 0.05])
    xi, eta, w = O.subdivided_rule(6)
    Y = v0 + xi[:, None] * (v1 - v0) + eta[:, None] * (v2 - v0)
    N = np.cross(v1 - v0, v2 - v0)
    J = np.linalg.norm(N)
    x = np.asarray(x)
    rho = x - ((x - v0) @ (N / J)) * (N / J)
    R = np.linalg.norm(Y - x, axis=1)[:, None]
    bf1 = J * np.sum(w[:, None] * (Y - rho) / R, axis=0)
    bf3 = J * np.sum(w[:, None] * (Y - rho) / R ** 3, axis=0)
    V1, V3 = O.tri_vector_moments(v0, v1, v2, x)
    assert np.abs(V1 - bf1).max() <= 1e-12 * np.abs(bf1).max()
    assert np.abs(V3 - bf3).max() <= 1e-11 * np.abs(bf3).max()


def product_rule_local(xyz, tri, op, i, j, level=3):
    xi, eta, w = O.subdivided_rule(level)
    a, b, c = xyz[tri[i]]
    u0, u1, u2 = xyz[tri[j]]
    X = a + xi[:, None] * (b - a) + eta[:, None] * (c - a)
    Y = u0 + xi[:, None] * (u1 - u0) + eta[:, None] * (u2 - u0)
    Nj = np.cross(u1 - u0, u2 - u0)
    Jj = np.linalg.norm(Nj)
    Ji = np.linalg.norm(np.cross(b - a, c - a))
    D = X[:, None, :] - Y[None, :, :]
    r = np.linalg.norm(D, axis=2)
    K = 1.0 / r if op == O.LAPLACE_SLP else (D @ (Nj / Jj)) / r ** 3
    phi = np.stack([1 - xi - eta, xi, eta])
    return Ji * Jj / (4 * np.pi) * np.einsum("ap,bq,p,q,pq->ab", phi, phi, w, w, K)


@pytest.mark.parametrize("op", [O.LAPLACE_SLP, O.LAPLACE_DLP])
def test_separated_pairs_vs_product_rule(ico2, op):
    xyz, tri, om = ico2
    cen = xyz[tri].mean(1)
    h = inputs.mean_edge_length(xyz, tri)
    d = np.linalg.norm(cen[0] - cen, axis=1)
    cols = [int(np.argmin(abs(d - f * h))) for f in (2.5, 6.0)]
    M = om.nearfield_p1_local(op, [0] * len(cols), cols, 3)
    for q, j in enumerate(cols):
        ref = product_rule_local(xyz, tri, op, 0, j)
        # the level-3 product rule itself: ~5e-10 on the double layer's small values at 2.5 h
        assert np.abs(M[q] - ref).max() <= 1e-8 * np.abs(ref).max(), j


@pytest.mark.parametrize("op", [O.LAPLACE_SLP, O.LAPLACE_DLP])
def test_local_matrices_sum_to_p0_value(ico2, op):
    xyz, tri, om = ico2
    adj = [j for j in range(tri.shape[0]) if set(tri[0]) & set(tri[j])]
    M = om.nearfield_p1_local(op, [0] * len(adj), adj, 3)
    p0 = np.array([om.nearfield_entry(op, 0, j, 3) for j in adj])
    assert np.abs(M.sum((1, 2)) - p0).max() <= 1e-14 * np.abs(p0).max()


def test_single_layer_symmetric_on_adjacent_pairs(ico2):
    xyz, tri, om = ico2
    adj = [j for j in range(tri.shape[0]) if set(tri[0]) & set(tri[j]) and j != 0]

    def rich(rows, cols):
        return (4 * om.nearfield_p1_local(O.LAPLACE_SLP, rows, cols, 5) -
                om.nearfield_p1_local(O.LAPLACE_SLP, rows, cols, 4)) / 3
    M = rich([0] * len(adj), adj)
    Mt = rich(adj, [0] * len(adj))
    # levels 4 and 5 extrapolated leave ~2e-7 on linear densities
    assert np.abs(M - Mt.transpose(0, 2, 1)).max() <= 1e-6 * np.abs(M).max()


def full_p1_matrix(xyz, tri, om, op, level):
    nv, nt = xyz.shape[0], tri.shape[0]
    idx = np.arange(nv, dtype=np.int32)
    A = om.entries(op, O.P1, 0.0, idx, idx, near=O.NEAR_SKIP)
    rows, cols = np.nonzero(np.array([[bool(set(tri[a]) & set(tri[b])) for b in range(nt)] for a in range(nt)]))
    M = om.nearfield_p1_local(op, rows, cols, level)
    for t, (i, j) in enumerate(zip(rows, cols)):
        A[np.ix_(tri[i], tri[j])] += M[t]
    return A


def hat_integrals(xyz, tri):
    area = 0.5 * np.linalg.norm(np.cross(xyz[tri[:, 1]] - xyz[tri[:, 0]], xyz[tri[:, 2]] - xyz[tri[:, 0]]), axis=1)
    return np.bincount(tri.ravel(), np.repeat(area / 3.0, 3), minlength=xyz.shape[0])


def test_double_layer_constant_density_p1(ico2):
    xyz, tri, om = ico2
    A = full_p1_matrix(xyz, tri, om, O.LAPLACE_DLP, 3)
    hat = hat_integrals(xyz, tri)
    rel = np.abs(A.sum(1) + 0.5 * hat) / (0.5 * hat)
    assert rel.max() <= 1e-4   # the regular pairs' 6-point rule error


def test_single_layer_sphere_constant_density_p1():
    errs = []
    for level in (2, 3):
        xyz, tri = inputs.icosphere(level)
        om = O.OracleMesh(xyz, tri, 6)
        A = full_p1_matrix(xyz, tri, om, O.LAPLACE_SLP, 3)
        hat = hat_integrals(xyz, tri)
        errs.append(np.abs(A.sum(1) - hat).max() / hat.max())
    assert errs[-1] < 2e-2
    assert 3.0 < errs[0] / errs[1] < 5.0   # O(h^2): the polyhedron against the sphere


def full_hyps_matrix(level, with_singular=True):
    xyz, tri = inputs.icosphere(level)
    om = O.OracleMesh(xyz, tri, 6)
    nv, nt = xyz.shape[0], tri.shape[0]
    idx = np.arange(nv, dtype=np.int32)
    A = om.entries(O.LAPLACE_HYPS, O.P1, 0.0, idx, idx, near=O.NEAR_SKIP)
    if with_singular:
        rows, cols = np.nonzero(np.array([[bool(set(tri[a]) & set(tri[b])) for b in range(nt)] for a in range(nt)]))
        M = (4 * om.nearfield_p1_local(O.LAPLACE_HYPS, rows, cols, 3) -
             om.nearfield_p1_local(O.LAPLACE_HYPS, rows, cols, 2)) / 3
        for t, (i, j) in enumerate(zip(rows, cols)):
            A[np.ix_(tri[i], tri[j])] += M[t]
    area = 0.5 * np.linalg.norm(np.cross(xyz[tri[:, 1]] - xyz[tri[:, 0]], xyz[tri[:, 2]] - xyz[tri[:, 0]]), axis=1)
    mass = np.zeros((nv, nv))
    for t in range(nt):
        mass[np.ix_(tri[t], tri[t])] += area[t] / 12.0 * (np.ones((3, 3)) + np.eye(3))
    return xyz, A, mass


def test_hypersingular_sphere_linear_functions():
    """Laplace hypersingular operator on the unit sphere: the degree-1
    spherical harmonics (the coordinates) are eigenfunctions with eigenvalue
    n(n+1)/(2n+1) = 2/3, so the complete P1 Galerkin matrix D satisfies
    D x ~ (2/3) M x (M the mass matrix) with an O(h^2) error from the
    polyhedral surface; without the singular pairs it fails outright."""
    errs = []
    for level in (2, 3):
        xyz, D, mass = full_hyps_matrix(level)
        u = xyz[:, 0]
        errs.append(np.linalg.norm(D @ u - (2.0 / 3.0) * mass @ u) / np.linalg.norm((2.0 / 3.0) * mass @ u))
    assert errs[-1] < 5e-3
    assert 3.0 < errs[0] / errs[1] < 5.0
    xyz, Ds, mass = full_hyps_matrix(2, with_singular=False)
    u = xyz[:, 0]
    assert np.linalg.norm(Ds @ u - (2.0 / 3.0) * mass @ u) / np.linalg.norm((2.0 / 3.0) * mass @ u) > 0.1


@pytest.mark.parametrize("x", [[0.4, 0.3, 0.5], [2.0, 1.0, 0.0], [-0.3, -0.2, 0.31], [5.0, 5.0, 5.0]])
def test_vector_moment_r_vs_brute_force(x):
    v0, v1, v2 = np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.1, 0.0]), np.array([0.3, 0.8, 0.05])
    xi, eta, w = O.subdivided_rule(6)
    Y = v0 + xi[:, None] * (v1 - v0) + eta[:, None] * (v2 - v0)
    N = np.cross(v1 - v0, v2 - v0)
    J = np.linalg.norm(N)
    x = np.asarray(x)
    rho = x - ((x - v0) @ (N / J)) * (N / J)
    bf = J * np.sum(w[:, None] * (Y - rho) * np.linalg.norm(Y - x, axis=1)[:, None], axis=0)
    W1 = O.tri_vector_moment_r(v0, v1, v2, x)
    assert np.abs(W1 - bf).max() <= 1e-12 * np.abs(bf).max()


def product_rule_local_c(xyz, tri, op, k, i, j, level=3):
    """Helmholtz P1 local matrix by the subdivided rule on both triangles:
    the real part of the k-dependent correction and the imaginary part."""
    xi, eta, w = O.subdivided_rule(level)
    a, b, c = xyz[tri[i]]
    u0, u1, u2 = xyz[tri[j]]
    X = a + xi[:, None] * (b - a) + eta[:, None] * (c - a)
    Y = u0 + xi[:, None] * (u1 - u0) + eta[:, None] * (u2 - u0)
    Nj = np.cross(u1 - u0, u2 - u0)
    Jj = np.linalg.norm(Nj)
    Ji = np.linalg.norm(np.cross(b - a, c - a))
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
        im = np.where(r0, 0.0, (np.sin(z) - z * np.cos(z)) * hgt / r ** 3)
    re = np.where(r0, 0.0, re)
    phi = np.stack([1 - xi - eta, xi, eta])
    f = Ji * Jj / (4 * np.pi)
    return (f * np.einsum("ap,bq,p,q,pq->ab", phi, phi, w, w, re),
            f * np.einsum("ap,bq,p,q,pq->ab", phi, phi, w, w, im))


@pytest.mark.parametrize("op", [O.HELMHOLTZ_SLP, O.HELMHOLTZ_DLP])
def test_helmholtz_p1_separated_pairs_vs_product_rule(ico2, op):
    xyz, tri, om = ico2
    cen = xyz[tri].mean(1)
    h = inputs.mean_edge_length(xyz, tri)
    d = np.linalg.norm(cen[0] - cen, axis=1)
    cols = [int(np.argmin(abs(d - f * h))) for f in (2.5, 6.0)]
    k = 6.0
    M = om.nearfield_p1_local_c(op, k, [0] * len(cols), cols, 3, 3)
    L = om.nearfield_p1_local(op - 2, [0] * len(cols), cols, 3)
    for q, j in enumerate(cols):
        re, im = product_rule_local_c(xyz, tri, op, k, 0, j)
        ref = L[q] + re + 1j * im
        assert np.abs(M[q] - ref).max() <= 1e-8 * np.abs(ref).max(), j


@pytest.mark.parametrize("op", [O.HELMHOLTZ_SLP, O.HELMHOLTZ_DLP])
def test_helmholtz_p1_adjacent_pairs(ico2, op):
    """Vertex-sharing pairs: the imaginary part (smooth kernel) against the
    product rule; the local matrices sum to the P0 value; k -> 0 gives the
    Laplace fixture."""
    xyz, tri, om = ico2
    adj = [j for j in range(tri.shape[0]) if set(tri[0]) & set(tri[j])]
    k = 4.0
    M = om.nearfield_p1_local_c(op, k, [0] * len(adj), adj, 3, 3)
    im = np.array([product_rule_local_c(xyz, tri, op, k, 0, j)[1] for j in adj])
    assert np.abs(M.imag - im).max() <= 1e-12 * np.abs(M.imag).max()
    p0 = om.nearfield_entries(op, k, [0] * len(adj), adj, 3, 3)
    assert np.abs(M.sum((1, 2)) - p0).max() <= 1e-14 * np.abs(p0).max()
    M0 = om.nearfield_p1_local_c(op, 1e-7, [0] * len(adj), adj, 2, 2)
    L = om.nearfield_p1_local(op - 2, [0] * len(adj), adj, 2)
    assert np.abs(M0.real - L).max() <= 1e-12 * np.abs(L).max()


def test_helmholtz_hypersingular_sphere_linear_functions():
    """Helmholtz hypersingular operator (Eq. hypsHelmholtz) on the unit
    sphere: the degree-1 spherical harmonics are eigenfunctions with
    eigenvalue -i k^3 j_1'(k) h_1'(k) (spherical Bessel and Hankel functions;
    2/3 as k -> 0), so the complete P1 matrix D satisfies D x ~ mu M x with an
    O(h^2) error."""
    from scipy.special import spherical_jn, spherical_yn
    k = 1.5
    jp = spherical_jn(1, k, derivative=True)
    mu = -1j * k ** 3 * jp * (jp + 1j * spherical_yn(1, k, derivative=True))
    errs = []
    for level in (2, 3):
        xyz, tri = inputs.icosphere(level)
        om = O.OracleMesh(xyz, tri, 6)
        nv, nt = xyz.shape[0], tri.shape[0]
        idx = np.arange(nv, dtype=np.int32)
        D = om.entries(O.HELMHOLTZ_HYPS, O.P1, k, idx, idx, near=O.NEAR_SKIP)
        rows, cols = np.nonzero(np.array([[bool(set(tri[a]) & set(tri[b])) for b in range(nt)] for a in range(nt)]))
        M = (4 * om.nearfield_p1_local_c(O.HELMHOLTZ_HYPS, k, rows, cols, 3, 2) -
             om.nearfield_p1_local_c(O.HELMHOLTZ_HYPS, k, rows, cols, 2, 2)) / 3
        for t, (i, j) in enumerate(zip(rows, cols)):
            D[np.ix_(tri[i], tri[j])] += M[t]
        area = 0.5 * np.linalg.norm(np.cross(xyz[tri[:, 1]] - xyz[tri[:, 0]], xyz[tri[:, 2]] - xyz[tri[:, 0]]), axis=1)
        mass = np.zeros((nv, nv))
        for t in range(nt):
            mass[np.ix_(tri[t], tri[t])] += area[t] / 12.0 * (np.ones((3, 3)) + np.eye(3))
        u = xyz[:, 0]
        errs.append(np.linalg.norm(D @ u - mu * (mass @ u)) / np.linalg.norm(mu * (mass @ u)))
    assert errs[-1] < 1e-2
    assert 3.0 < errs[0] / errs[1] < 5.0
