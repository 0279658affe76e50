"""Pins of the oracle's Galerkin entries (Eqs. slp, dlp over regular pairs).

Independent references used here:
  * brute force: a tensor Gauss-Legendre rule on the Duffy-collapsed square
    (numpy, 20 points per direction), i.e. a different discretisation of the
    same 4-D integral; the oracle's 6-point result must converge to it as the
    separation grows, at the rate of a degree-4 rule;
  * the far-field limit A_ij -> |T_i| |T_j| K(c_i, c_j);
  * invariants: symmetry of the single layer, the P1/P0 partition of unity,
    scaling, rigid motions, the near-pair policy.
"""
import math

import numpy as np
import pytest

import oracle as O

RNG = np.random.Generator(np.random.PCG64(3))


def gl01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def duffy_points(a, b, c, n=20):
    """Points, weights (including the area Jacobian) and barycentric coords."""
    u, wu = gl01(n)
    v, wv = gl01(n)
    U, V = np.meshgrid(u, v, indexing="ij")
    W = np.outer(wu, wv) * (1.0 - U)
    xi = U.ravel()
    eta = ((1.0 - U) * V).ravel()
    J = np.linalg.norm(np.cross(b - a, c - a))
    pts = a + xi[:, None] * (b - a) + eta[:, None] * (c - a)
    lam = np.stack([1.0 - xi - eta, xi, eta], axis=1)
    return pts, J * W.ravel(), lam


def brute_pair(op, k, A, B, a_loc=None, b_loc=None, n=20):
    """int_A int_B psi(x) K(x,y) phi(y) by the Duffy/Gauss-Legendre rule."""
    xp, xw, xl = duffy_points(*A, n=n)
    yp, yw, yl = duffy_points(*B, n=n)
    if a_loc is not None:
        xw = xw * xl[:, a_loc]
    if b_loc is not None:
        yw = yw * yl[:, b_loc]
    ny = np.cross(B[1] - B[0], B[2] - B[0])
    ny /= np.linalg.norm(ny)
    d = xp[:, None, :] - yp[None, :, :]
    r = np.linalg.norm(d, axis=2)
    g = np.exp(1j * k * r) / (4 * math.pi * r)
    if op in (O.LAPLACE_DLP, O.HELMHOLTZ_DLP):
        g = g * (1.0 - 1j * k * r) * (d @ ny) / (r * r)
    val = np.einsum("i,ij,j->", xw, g, yw)
    return val if op in (O.HELMHOLTZ_SLP, O.HELMHOLTZ_DLP) else val.real


def two_triangle_mesh(A, B):
    xyz = np.vstack([A, B])
    tri = np.array([[0, 1, 2], [3, 4, 5]], dtype=np.int32)
    return xyz, tri


def rotation(rng):
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


T1 = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.3, 0.8, 0.0]])
T2_LOCAL = np.array([[0.0, 0.0, 0.0], [0.7, 0.1, 0.2], [0.1, 0.9, -0.4]])
DIR = np.array([0.6, -0.48, 0.64])


def placed_pair(d):
    B = T2_LOCAL + d * DIR
    return T1, B


@pytest.mark.parametrize("op", [O.LAPLACE_SLP, O.LAPLACE_DLP])
def test_far_field_limit_laplace(op):
    errs = []
    for d in (40.0, 80.0, 160.0):
        A, B = placed_pair(d)
        errs.append(abs(entry(op, 0.0, A, B) / centroid_value(op, 0.0, A, B) - 1.0))
    assert errs[0] < 2e-3
    # second-order approach to the centroid limit
    assert errs[1] < errs[0] / 3.0 and errs[2] < errs[1] / 3.0


@pytest.mark.parametrize("op", [O.HELMHOLTZ_SLP, O.HELMHOLTZ_DLP])
def test_far_field_limit_helmholtz(op):
    """Small triangles (k h = 0.017) far apart (k d ~ 68): the entry tends to
    the centroid value, phase exp(+i k |c_i - c_j|) included."""
    k = 1.7
    for d in (40.0, 55.0):
        A = T1 * 0.01
        B = T2_LOCAL * 0.01 + d * DIR
        e = entry(op, k, A, B)
        c = centroid_value(op, k, A, B)
        assert abs(e / c - 1.0) < 1e-3
        # the opposite time convention is far off
        assert abs(np.conj(e) / c - 1.0) > 0.1


def entry(op, k, A, B):
    m = O.OracleMesh(*two_triangle_mesh(A, B), 6)
    return m.entries(op, O.P0, k, [0], [1])[0, 0]


def centroid_value(op, k, A, B):
    cA, cB = A.mean(0), B.mean(0)
    areaA = 0.5 * np.linalg.norm(np.cross(A[1] - A[0], A[2] - A[0]))
    nB = np.cross(B[1] - B[0], B[2] - B[0])
    areaB = 0.5 * np.linalg.norm(nB)
    return areaA * areaB * O.kernel(op, k, cA, cB, nB / np.linalg.norm(nB))


@pytest.mark.parametrize("op", [O.LAPLACE_SLP, O.LAPLACE_DLP])
def test_brute_force_convergence_laplace(op):
    errs = []
    for d in (2.0, 4.0, 8.0, 16.0, 32.0):
        A, B = placed_pair(d)
        ref = brute_pair(op, 0.0, A, B)
        errs.append(abs(entry(op, 0.0, A, B) - ref) / abs(ref))
    # degree-4 tensor rule: the relative error falls ~2^5 per doubling of d
    assert errs[-1] < 1e-10
    for e0, e1 in zip(errs[1:], errs[2:]):
        assert e1 < e0 / 16.0


@pytest.mark.parametrize("op", [O.HELMHOLTZ_SLP, O.HELMHOLTZ_DLP])
def test_brute_force_helmholtz(op):
    """At k h ~ 2 the 6-point rule errs by ~3e-5 at any distance; a wrong
    phase sign or a dropped (1 - i k r) factor errs by O(1)."""
    k = 2.0
    for d in (4.0, 8.0):
        A, B = placed_pair(d)
        ref = brute_pair(op, k, A, B)
        got = entry(op, k, A, B)
        assert abs(got - ref) < 1e-4 * abs(ref)
        assert abs(np.conj(got) - ref) > 0.05 * abs(ref)
        if op == O.HELMHOLTZ_DLP:
            ny = np.cross(B[1] - B[0], B[2] - B[0])
            # the same integrand without the (1 - i k r) factor
            xp, xw, _ = duffy_points(*A)
            yp, yw, _ = duffy_points(*B)
            d_ = xp[:, None, :] - yp[None, :, :]
            r = np.linalg.norm(d_, axis=2)
            alt = np.einsum("i,ij,j->", xw, np.exp(1j * k * r) * (d_ @ (ny / np.linalg.norm(ny))) / (4 * math.pi * r ** 3), yw)
            assert abs(got - alt) > 0.05 * abs(ref)


def p1_brute(op, k, xyz, tri, m, I, J, rotate_test_basis=False):
    ref = 0.0
    for tA in np.flatnonzero((tri == I).any(1)):
        for tB in np.flatnonzero((tri == J).any(1)):
            if m.adjacent(int(tA), int(tB)):
                continue
            a_loc = int(np.flatnonzero(tri[tA] == I)[0])
            if rotate_test_basis:
                a_loc = (a_loc + 1) % 3
            b_loc = int(np.flatnonzero(tri[tB] == J)[0])
            ref = ref + brute_pair(op, k, xyz[tri[tA]], xyz[tri[tB]], a_loc, b_loc)
    return ref


@pytest.mark.parametrize("op,k", [(O.LAPLACE_SLP, 0.0), (O.LAPLACE_DLP, 0.0), (O.HELMHOLTZ_SLP, 1.3),
                                  (O.HELMHOLTZ_DLP, 1.3)])
def test_p1_entries_brute_force(op, k, ico):
    """P1 entries between a vertex and vertices 3-5 edges away on a level-2
    icosphere: within the 6-point rule's error of the brute-force integral,
    and far from the value with the test hat function moved to another
    corner of each triangle."""
    xyz, tri = ico(2)
    m = O.OracleMesh(xyz, tri, 6)
    I = 0
    dist = np.linalg.norm(xyz - xyz[I], axis=1)
    Js = [int(j) for j in np.argsort(dist) if 0.8 < dist[j] < 1.6][:4]
    assert Js
    got = m.entries(op, O.P1, k, [I], Js)[0]
    for J, g in zip(Js, got):
        ref = p1_brute(op, k, xyz, tri, m, I, J)
        assert abs(g - ref) <= 2e-4 * abs(ref), (J, g, ref)
        wrong = p1_brute(op, k, xyz, tri, m, I, J, rotate_test_basis=True)
        assert abs(wrong - ref) > 5e-3 * abs(ref)


@pytest.mark.parametrize("op,k", [(O.LAPLACE_SLP, 0.0), (O.HELMHOLTZ_SLP, 3.0)])
def test_single_layer_symmetric(op, k, ico):
    xyz, tri = ico(2)
    m = O.OracleMesh(xyz, tri, 6)
    idx = np.arange(m.nt)
    A = m.entries(op, O.P0, k, idx, idx)
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    idx = np.arange(m.nv)
    A = m.entries(op, O.P1, k, idx, idx)
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()


@pytest.mark.parametrize("op", [O.LAPLACE_SLP, O.LAPLACE_DLP, O.HELMHOLTZ_DLP])
def test_p1_partition_of_unity(op, ico):
    """Hat functions sum to one on every triangle, so the sum of all P1
    entries equals the sum of all P0 entries over the same regular pairs."""
    xyz, tri = ico(1)
    m = O.OracleMesh(xyz, tri, 6)
    k = 2.5 if op == O.HELMHOLTZ_DLP else 0.0
    p0 = m.entries(op, O.P0, k, np.arange(m.nt), np.arange(m.nt))
    p1 = m.entries(op, O.P1, k, np.arange(m.nv), np.arange(m.nv))
    assert abs(p1.sum() - p0.sum()) <= 1e-13 * np.abs(p0).sum()


@pytest.mark.parametrize("space", [O.P0, O.P1])
def test_scaling_laws(space, ico):
    xyz, tri = ico(1)
    s = 2.5
    m1 = O.OracleMesh(xyz, tri, 6)
    m2 = O.OracleMesh(s * xyz, tri, 6)
    n = m1.nt if space == O.P0 else m1.nv
    idx = np.arange(n)
    for op, power in [(O.LAPLACE_SLP, 3), (O.LAPLACE_DLP, 2)]:
        a = m1.entries(op, space, 0.0, idx, idx)
        b = m2.entries(op, space, 0.0, idx, idx)
        assert np.abs(b - s ** power * a).max() <= 1e-13 * np.abs(b).max()
    # Helmholtz: (s mesh, k/s) = s^3 (mesh, k)
    a = m1.entries(O.HELMHOLTZ_SLP, space, 4.0, idx, idx)
    b = m2.entries(O.HELMHOLTZ_SLP, space, 4.0 / s, idx, idx)
    assert np.abs(b - s ** 3 * a).max() <= 1e-13 * np.abs(b).max()


def test_rigid_motion_invariance(ico):
    xyz, tri = ico(1)
    R = rotation(RNG)
    moved = xyz @ R.T + np.array([1e3, -2e3, 5e2])
    m1 = O.OracleMesh(xyz, tri, 6)
    m2 = O.OracleMesh(moved, tri, 6)
    idx = np.arange(m1.nt)
    for op, k in [(O.LAPLACE_SLP, 0.0), (O.LAPLACE_DLP, 0.0), (O.HELMHOLTZ_DLP, 3.0)]:
        a = m1.entries(op, O.P0, k, idx, idx)
        b = m2.entries(op, O.P0, k, idx, idx)
        assert np.abs(b - a).max() <= 1e-9 * np.abs(a).max()


def test_near_policy(ico):
    xyz, tri = ico(1)
    m = O.OracleMesh(xyz, tri, 6)
    nbr = [t for t in range(m.nt) if t != 0 and m.adjacent(0, t)]
    far = [t for t in range(m.nt) if not m.adjacent(0, t)]
    with pytest.raises(O.NearFieldError):
        m.entries(O.LAPLACE_SLP, O.P0, 0.0, [0], [nbr[0]], near=O.NEAR_ERROR)
    with pytest.raises(O.NearFieldError):
        m.entries(O.LAPLACE_SLP, O.P0, 0.0, [0], [0], near=O.NEAR_ERROR)
    a = m.entries(O.LAPLACE_SLP, O.P0, 0.0, [0], nbr + far[:3], near=O.NEAR_SKIP)
    assert (a[0, :len(nbr)] == 0).all() and (a[0, len(nbr):] > 0).all()
    b = m.entries(O.LAPLACE_SLP, O.P0, 0.0, [0], far[:3], near=O.NEAR_ERROR)
    assert np.array_equal(a[0, len(nbr):], b[0])


def test_icosphere_level3_regular_pair_count(ico):
    """1280 triangles: 16,580 ordered pairs share a vertex (self included),
    so a full dense request has 1,621,820 regular entries."""
    xyz, tri = ico(3)
    m = O.OracleMesh(xyz, tri, 6)
    idx = np.arange(m.nt)
    A = m.entries(O.LAPLACE_SLP, O.P0, 0.0, idx, idx)
    assert int((A != 0).sum()) == 1621820
    # the count of vertex-sharing pairs from the mesh alone
    share = np.zeros((m.nt, m.nt), dtype=bool)
    for k in range(3):
        for l in range(3):
            share |= tri[:, k][:, None] == tri[:, l][None, :]
    assert int(share.sum()) == 16580
    assert np.array_equal(share, A == 0)


@pytest.mark.parametrize("space", [O.P0, O.P1])
@pytest.mark.parametrize("pair,k", [((O.LAPLACE_ADLP, O.LAPLACE_DLP), 0.0), ((O.HELMHOLTZ_ADLP, O.HELMHOLTZ_DLP), 2.3)])
def test_adjoint_double_layer_is_transposed_double_layer(space, pair, k, ico):
    """Eqs. dlp and adlp with the same space and rule on both sides:
    [K'_h]_ij = [K_h]_ji (the summation order differs, so not bitwise).  A
    jittered mesh keeps K_h far from symmetric, so a double layer returned
    for the adjoint, a dropped sign or the trial normal in place of the test
    normal all fail."""
    xyz, tri = ico(2)
    rng = np.random.Generator(np.random.PCG64(3))
    xyz = xyz * (1.0 + 0.08 * rng.uniform(-1, 1, size=(xyz.shape[0], 1)))
    m = O.OracleMesh(xyz, tri, 6)
    n = m.nt if space == O.P0 else m.nv
    rows = rng.choice(n, 40, replace=False)
    cols = rng.choice(n, 55, replace=False)
    adj, dl = pair
    A = m.entries(adj, space, k, rows, cols, near=O.NEAR_SKIP)
    K = m.entries(dl, space, k, cols, rows, near=O.NEAR_SKIP)
    scale = np.abs(K).max()
    assert np.abs(A - K.T).max() <= 1e-13 * scale
    assert np.abs(A - m.entries(dl, space, k, rows, cols, near=O.NEAR_SKIP)).max() > 1e-3 * scale


# ---------------------------------------------------------------------------
# Hypersingular operator, Eq. hypsHelmholtz (P1 only).


def surface_curl(T, a):
    """curl of the hat function of local vertex a on triangle T: n x grad,
    the gradient from the linear system g.(v1-v0), g.(v2-v0) = hat
    differences, g.n = 0."""
    n = np.cross(T[1] - T[0], T[2] - T[0])
    n /= np.linalg.norm(n)
    hat = [1.0 if j == a else 0.0 for j in range(3)]
    g = np.linalg.solve(np.array([T[1] - T[0], T[2] - T[0], n]), [hat[1] - hat[0], hat[2] - hat[0], 0.0])
    return np.cross(n, g), n


def hyps_brute(k, A, B, a_loc, b_loc):
    ca, na = surface_curl(A, a_loc)
    cb, nb = surface_curl(B, b_loc)
    slp = O.LAPLACE_SLP if k == 0.0 else O.HELMHOLTZ_SLP
    val = np.dot(ca, cb) * brute_pair(slp, k, A, B)
    if k != 0.0:
        val = val - k * k * np.dot(na, nb) * brute_pair(slp, k, A, B, a_loc, b_loc)
    return val


@pytest.mark.parametrize("k", [0.0, 1.1])
@pytest.mark.parametrize("a_loc,b_loc", [(0, 1), (2, 0), (1, 2)])
def test_hypersingular_pair_brute_force(k, a_loc, b_loc):
    """One regular pair (two disjoint triangles, so the P1 entry is that
    pair alone): the oracle matches the high-order integral of
    curl.curl g - k^2 n.n lam lam g, with the curls from a linear solve."""
    A, B = placed_pair(16.0)
    m = O.OracleMesh(*two_triangle_mesh(A, B), 6)
    op = O.LAPLACE_HYPS if k == 0.0 else O.HELMHOLTZ_HYPS
    got = m.entries(op, O.P1, k, [a_loc], [3 + b_loc])[0, 0]
    ref = hyps_brute(k, A, B, a_loc, b_loc)
    # the 6-point rule's own error: ~1e-9 for Laplace at this distance, ~1e-6
    # on exp(ikr) at k h ~ 1.1 (the Helmholtz single-layer pin allows 1e-4 at k = 2)
    assert abs(got - ref) <= (1e-7 if k == 0.0 else 1e-5) * abs(ref)
    if k != 0.0:
        # the k^2 term with the opposite sign is far off
        alt = ref + 2 * k * k * np.dot(surface_curl(A, 0)[1], surface_curl(B, 0)[1]) * \
            brute_pair(O.HELMHOLTZ_SLP, k, A, B, a_loc, b_loc)
        assert abs(got - alt) > 1e-2 * abs(ref)


def jittered(ico, level=2, seed=3):
    xyz, tri = ico(level)
    rng = np.random.Generator(np.random.PCG64(seed))
    return xyz * (1.0 + 0.08 * rng.uniform(-1, 1, size=(xyz.shape[0], 1))), tri


def test_laplace_hypersingular_annihilates_constants(ico):
    """curl of the constant function vanishes, triangle by triangle, so every
    row of the Laplace hypersingular matrix sums to zero (regular pairs only
    or not)."""
    xyz, tri = jittered(ico)
    m = O.OracleMesh(xyz, tri, 6)
    rows = np.random.Generator(np.random.PCG64(5)).choice(m.nv, 15, replace=False)
    D = m.entries(O.LAPLACE_HYPS, O.P1, 0.0, rows, np.arange(m.nv))
    assert np.all(np.abs(D.sum(1)) <= 1e-13 * np.abs(D).sum(1))


@pytest.mark.parametrize("op,k", [(O.LAPLACE_HYPS, 0.0), (O.HELMHOLTZ_HYPS, 2.1)])
def test_hypersingular_symmetric(op, k, ico):
    xyz, tri = jittered(ico)
    m = O.OracleMesh(xyz, tri, 6)
    idx = np.random.Generator(np.random.PCG64(6)).choice(m.nv, 40, replace=False)
    D = m.entries(op, O.P1, k, idx, idx)
    assert np.abs(D - D.T).max() <= 1e-13 * np.abs(D).max()


def test_laplace_hypersingular_scales_linearly(ico):
    """Under x -> s x: curls scale 1/s each, g 1/s, areas s^2 each: D -> s D."""
    xyz, tri = jittered(ico)
    idx = np.arange(0, 162, 7)
    D1 = O.OracleMesh(xyz, tri, 6).entries(O.LAPLACE_HYPS, O.P1, 0.0, idx, idx)
    D2 = O.OracleMesh(2.5 * xyz, tri, 6).entries(O.LAPLACE_HYPS, O.P1, 0.0, idx, idx)
    assert np.abs(D2 - 2.5 * D1).max() <= 1e-13 * np.abs(D2).max()


def test_hypersingular_needs_p1(ico):
    xyz, tri = ico(1)
    m = O.OracleMesh(xyz, tri, 6)
    with pytest.raises(Exception):
        m.entries(O.LAPLACE_HYPS, O.P0, 0.0, [0], [1])


# ---------------------------------------------------------------------------
# Discontinuous P1 (dof 3 t + a) and the hypersingular operator through the
# single layer on it (Eq. hyp_via_slp).


@pytest.mark.parametrize("op,k", [(O.LAPLACE_SLP, 0.0), (O.LAPLACE_DLP, 0.0), (O.HELMHOLTZ_SLP, 1.7),
                                  (O.HELMHOLTZ_DLP, 1.7)])
def test_dp1_entry_brute_force(op, k):
    """A DP1 entry of two disjoint triangles is the basis-weighted pair
    integral: against the Duffy/Gauss-Legendre product rule, within the
    6-point rule's error, which falls as the pair moves apart; the entry
    with the basis functions' corners exchanged is far off."""
    # Helmholtz at k = 1.7 keeps the phase error of the rule across a
    # triangle (k h ~ 1.7) at any distance; Laplace's falls like (h/d)^5
    far = 3e-6 if k == 0.0 else 5e-4
    for d, bound in ((2.5, 5e-4), (8.0, far)):
        A, B = placed_pair(d)
        xyz, tri = two_triangle_mesh(A, B)
        m = O.OracleMesh(xyz, tri, 6)
        for a in range(3):
            for b in range(3):
                got = m.entries(op, O.DP1, k, [a], [3 + b], near=O.NEAR_ERROR)[0, 0]
                ref = brute_pair(op, k, A, B, a, b, n=24)
                assert abs(got - ref) <= bound * abs(ref), (d, a, b, got, ref)
                if d < 3:
                    wrong = brute_pair(op, k, A, B, (a + 1) % 3, b, n=24)
                    assert abs(wrong - ref) > 1e-2 * abs(ref)


@pytest.mark.parametrize("op,k", [(O.LAPLACE_SLP, 0.0), (O.LAPLACE_DLP, 0.0), (O.HELMHOLTZ_SLP, 2.1)])
def test_dp1_sums_to_p0_and_assembles_p1(op, k, ico):
    """Partition of unity: the three local functions of a triangle sum to
    its indicator, so DP1 blocks summed over local indices give the P0
    entries; gathering DP1 entries over the stars of two vertices (the
    continuity map, an incidence matrix) gives the P1 entries."""
    xyz, tri = ico(2)
    m = O.OracleMesh(xyz, tri, 6)
    nt, nv = tri.shape[0], xyz.shape[0]
    rt = np.arange(0, nt, 7)
    ct = np.arange(3, nt, 5)
    dr = (3 * rt[:, None] + np.arange(3)).ravel()
    dc = (3 * ct[:, None] + np.arange(3)).ravel()
    D = m.entries(op, O.DP1, k, dr, dc)
    P0 = m.entries(op, O.P0, k, rt, ct)
    S = D.reshape(rt.size, 3, ct.size, 3).sum(axis=(1, 3))
    assert np.abs(S - P0).max() <= 1e-13 * np.abs(P0).max()
    C = np.zeros((nv, 3 * nt))
    for t in range(nt):
        for a in range(3):
            C[tri[t, a], 3 * t + a] = 1.0
    Dfull = m.entries(op, O.DP1, k, np.arange(3 * nt), np.arange(3 * nt))
    rows, cols = np.arange(0, nv, 9), np.arange(2, nv, 4)
    P1 = m.entries(op, O.P1, k, rows, cols)
    G = C[rows] @ Dfull @ C[cols].T
    assert np.abs(G - P1).max() <= 1e-12 * np.abs(P1).max()


@pytest.mark.parametrize("op,k", [(O.LAPLACE_HYPS, 0.0), (O.HELMHOLTZ_HYPS, 2.3)])
def test_hypersingular_via_single_layer_on_dp1(op, k, ico):
    """Eq. hyp_via_slp: D = sum_j Q_j^T S Q_j - k^2 sum_j P_j^T S P_j with S
    the single layer on DP1, Q_j the curl components and P_j the normal
    components (oracle.hyp_via_slp_factors), equals the direct P1
    hypersingular entries on the same regular pairs; a transposed or
    sign-flipped factor, or a missing k^2 term, fails."""
    xyz, tri = jittered(ico, level=1)
    m = O.OracleMesh(xyz, tri, 6)
    nt, nv = tri.shape[0], xyz.shape[0]
    slp = O.LAPLACE_SLP if k == 0.0 else O.HELMHOLTZ_SLP
    S = m.entries(slp, O.DP1, k, np.arange(3 * nt), np.arange(3 * nt))
    Q, P = O.hyp_via_slp_factors(xyz, tri)
    D = sum(Q[j].T @ S @ Q[j] for j in range(3)) - k * k * sum(P[j].T @ S @ P[j] for j in range(3))
    ref = m.entries(op, O.P1, k, np.arange(nv), np.arange(nv))
    assert np.abs(D - ref).max() <= 1e-11 * np.abs(ref).max()
    if k != 0.0:
        D0 = sum(Q[j].T @ S @ Q[j] for j in range(3))
        assert np.abs(D0 - ref).max() > 1e-3 * np.abs(ref).max()
    Dbad = sum(Q[j].T @ S @ Q[(j + 1) % 3] for j in range(3))
    assert np.abs(Dbad - ref).max() > 1e-3 * np.abs(ref).max()
