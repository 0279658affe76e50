"""GPU parity: weak-form entries from the HIP path vs the FP64 oracle.

Tolerances (stated for the hot path): FP64 path 1e-12 entrywise for the
Laplace single layer (all 1,621,820 regular entries of the level-3
icosphere), 1e-11 normwise otherwise; FP32 compensated path 1e-5 for
Laplace, 1e-4 for Helmholtz.  Error measures: entrywise relative error where
every entry is a sum of positive terms (Laplace single layer, positive
weights), per-request normwise max|a-b| / max|b| elsewhere (double-layer
entries vanish for coplanar pairs, Helmholtz sums cancel).
"""
import numpy as np
import pytest

import oracle as O
from paper_1711_01897_amd import bem, inputs

pytestmark = pytest.mark.gpu

OPS = [bem.LAPLACE_SLP, bem.LAPLACE_DLP, bem.HELMHOLTZ_SLP, bem.HELMHOLTZ_DLP, bem.LAPLACE_ADLP, bem.HELMHOLTZ_ADLP]
K = {bem.LAPLACE_SLP: 0.0, bem.LAPLACE_DLP: 0.0, bem.HELMHOLTZ_SLP: 7.5, bem.HELMHOLTZ_DLP: 7.5,
     bem.LAPLACE_ADLP: 0.0, bem.HELMHOLTZ_ADLP: 7.5}


def tol(op, prec):
    if prec == bem.FP64:
        return 1e-11
    return 1e-5 if op in (bem.LAPLACE_SLP, bem.LAPLACE_DLP, bem.LAPLACE_ADLP) else 1e-4


def normwise(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def entrywise(a, b):
    nz = b != 0
    assert np.all(a[~nz] == 0)
    return np.max(np.abs(a[nz] - b[nz]) / np.abs(b[nz]))


@pytest.fixture(scope="module")
def sphere2():
    xyz, tri = inputs.icosphere(2)
    return xyz, tri, bem.mesh_create(xyz, tri, 6), O.OracleMesh(xyz, tri, 6)


@pytest.mark.parametrize("prec,bound", [(bem.FP64, 1e-12), (bem.FP32, 1e-5)])
def test_icosphere3_dense_laplace_slp_p0(prec, bound):
    """All 1280 x 1280 entries; vertex-sharing pairs are zero on both sides."""
    xyz, tri = inputs.icosphere(3)
    mesh = bem.mesh_create(xyz, tri, 6)
    idx = np.arange(tri.shape[0], dtype=np.int32)
    got = bem.eval_entries(mesh, bem.LAPLACE_SLP, bem.P0, 0.0, idx, idx, prec=prec, near=bem.NEAR_SKIP)
    ref = O.OracleMesh(xyz, tri, 6).entries(O.LAPLACE_SLP, O.P0, 0.0, idx, idx)
    assert int((ref != 0).sum()) == 1621820
    err = entrywise(got.astype(np.float64), ref)
    print(f"prec={prec} max entrywise rel err {err:.3e}")
    assert err <= bound
    mesh.destroy()


SHAPES = [(37, 150), (150, 1), (1, 150), (70, 70), (1, 1), (129, 3)]


@pytest.mark.parametrize("op", OPS)
@pytest.mark.parametrize("space", [bem.P0, bem.P1])
@pytest.mark.parametrize("prec", [bem.FP64, bem.FP32])
def test_requests_vs_oracle(sphere2, op, space, prec):
    xyz, tri, mesh, om = sphere2
    n = tri.shape[0] if space == bem.P0 else xyz.shape[0]
    rng = np.random.Generator(np.random.PCG64(3))
    for nr, nc in SHAPES:
        rows = rng.choice(n, size=min(nr, n), replace=False).astype(np.int32)
        cols = rng.choice(n, size=min(nc, n), replace=False).astype(np.int32)
        got = bem.eval_entries(mesh, op, space, K[op], rows, cols, prec=prec)
        ref = om.entries(op, space, K[op], rows, cols)
        assert got.shape == ref.shape
        if np.max(np.abs(ref)) == 0:
            assert np.all(got == 0)
            continue
        e = normwise(got.astype(ref.dtype), ref)
        assert e <= tol(op, prec), (nr, nc, e)
        if op == bem.LAPLACE_SLP:
            assert entrywise(got.astype(np.float64), ref) <= (1e-12 if prec == bem.FP64 else 1e-5)


@pytest.mark.parametrize("pair", [(bem.LAPLACE_ADLP, bem.LAPLACE_DLP), (bem.HELMHOLTZ_ADLP, bem.HELMHOLTZ_DLP)])
@pytest.mark.parametrize("space", [bem.P0, bem.P1])
@pytest.mark.parametrize("prec", [bem.FP64, bem.FP32])
def test_adjoint_double_layer_is_exact_transpose(sphere2, pair, space, prec):
    """The adjoint double layer runs as the double layer with test and trial
    exchanged: A'[rows, cols] equals K[cols, rows]^T bit for bit, for both
    fixed sides (short and long row lists)."""
    xyz, tri, mesh, om = sphere2
    adj, dl = pair
    n = tri.shape[0] if space == bem.P0 else xyz.shape[0]
    rng = np.random.Generator(np.random.PCG64(4))
    for nr, nc in [(1, 120), (120, 1), (33, 77), (77, 33)]:
        rows = rng.choice(n, nr, replace=False).astype(np.int32)
        cols = rng.choice(n, nc, replace=False).astype(np.int32)
        a = bem.eval_entries(mesh, adj, space, K[adj], rows, cols, prec=prec)
        d = bem.eval_entries(mesh, dl, space, K[dl], cols, rows, prec=prec)
        assert a.shape == (nr, nc)
        assert np.array_equal(a, d.T)


@pytest.mark.parametrize("op", [bem.LAPLACE_SLP, bem.LAPLACE_DLP, bem.HELMHOLTZ_SLP, bem.LAPLACE_ADLP])
@pytest.mark.parametrize("prec", [bem.FP64, bem.FP32])
def test_p1_scrambled_long_lane_lists(op, prec):
    """P1 lane lists longer than one chunk are reordered along a space-filling
    curve inside the library; the entries still land at the caller's
    positions, duplicates included, for both fixed sides."""
    xyz, tri = inputs.icosphere(3)
    mesh = bem.mesh_create(xyz, tri, 6)
    om = O.OracleMesh(xyz, tri, 6)
    rng = np.random.Generator(np.random.PCG64(9))
    nv = xyz.shape[0]
    long_ = rng.permutation(nv)[:600].astype(np.int32)
    long_ = np.concatenate([long_, long_[:37]])          # duplicated positions
    short = rng.choice(nv, 5, replace=False).astype(np.int32)
    for rows, cols in ((short, long_), (long_, short)):
        got = bem.eval_entries(mesh, op, bem.P1, K[op], rows, cols, prec=prec)
        ref = om.entries(op, O.P1, K[op], rows, cols)
        e = normwise(got.astype(ref.dtype), ref)
        assert e <= tol(op, prec), (rows.size, cols.size, e)
        # duplicated indices give identical entries
        if cols.size > rows.size:
            assert np.array_equal(got[:, 600:], got[:, :37])
        else:
            assert np.array_equal(got[600:], got[:37])
    mesh.destroy()


@pytest.mark.parametrize("prec", [bem.FP64, bem.FP32])
def test_four_point_rule_helmholtz_spheroid(prec):
    """4-point rule, elongated spheroid, Helmholtz single layer at 10
    elements per wavelength (the complex64/complex128 workload, small)."""
    xyz, tri = inputs.spheroid(10.0, 1.0, 6000)
    k = inputs.wavenumber(xyz, tri, 10.0)
    mesh = bem.mesh_create(xyz, tri, 4)
    om = O.OracleMesh(xyz, tri, 4)
    rng = np.random.Generator(np.random.PCG64(3))
    for nr, nc in [(1, 2000), (2000, 1), (40, 300)]:
        rows = rng.choice(tri.shape[0], nr, replace=False).astype(np.int32)
        cols = rng.choice(tri.shape[0], nc, replace=False).astype(np.int32)
        got = bem.eval_entries(mesh, bem.HELMHOLTZ_SLP, bem.P0, k, rows, cols, prec=prec)
        ref = om.entries(O.HELMHOLTZ_SLP, O.P0, k, rows, cols)
        e = normwise(got.astype(np.complex128), ref)
        print(f"k={k:.2f} shape={nr}x{nc} err={e:.2e}")
        assert e <= tol(bem.HELMHOLTZ_SLP, prec)


def test_translated_mesh_fp32():
    """Centroid-relative FP32 geometry: a mesh moved by 10^3 keeps FP32
    accuracy (absolute FP32 coordinates would lose ~1e-4 here)."""
    xyz, tri = inputs.icosphere(3)
    xyz = xyz * 0.5 + np.array([1000.0, -700.0, 300.0])
    mesh = bem.mesh_create(xyz, tri, 6)
    om = O.OracleMesh(xyz, tri, 6)
    rows = np.arange(0, 1280, 11, dtype=np.int32)
    cols = np.arange(1280, dtype=np.int32)
    for op in (bem.LAPLACE_SLP, bem.LAPLACE_DLP):
        got = bem.eval_entries(mesh, op, bem.P0, 0.0, rows, cols, prec=bem.FP32)
        ref = om.entries(op, O.P0, 0.0, rows, cols)
        assert normwise(got.astype(np.float64), ref) <= 1e-5
    got = bem.eval_entries(mesh, bem.LAPLACE_SLP, bem.P1, 0.0, np.arange(50), np.arange(642), prec=bem.FP32)
    ref = om.entries(O.LAPLACE_SLP, O.P1, 0.0, np.arange(50), np.arange(642))
    assert entrywise(got.astype(np.float64), ref) <= 1e-5


def test_near_field_policies(sphere2):
    xyz, tri, mesh, om = sphere2
    nbr = [t for t in range(tri.shape[0]) if om.adjacent(0, t)]
    far = [t for t in range(tri.shape[0]) if not om.adjacent(0, t)][:40]
    with pytest.raises(bem.NearFieldError):
        bem.eval_entries(mesh, bem.LAPLACE_SLP, bem.P0, 0.0, [0], nbr[:3] + far, near=bem.NEAR_ERROR)
    got = bem.eval_entries(mesh, bem.LAPLACE_SLP, bem.P0, 0.0, [0], nbr + far, near=bem.NEAR_SKIP)
    assert np.all(got[0, :len(nbr)] == 0) and np.all(got[0, len(nbr):] > 0)
    ok = bem.eval_entries(mesh, bem.LAPLACE_SLP, bem.P0, 0.0, [0], far, near=bem.NEAR_ERROR)
    assert np.array_equal(ok[0], got[0, len(nbr):])
    # P1: vertex 0 against its neighbours
    vn = np.unique(tri[(tri == 0).any(1)])
    with pytest.raises(bem.NearFieldError):
        bem.eval_entries(mesh, bem.LAPLACE_SLP, bem.P1, 0.0, [0], vn, near=bem.NEAR_ERROR)
    got = bem.eval_entries(mesh, bem.LAPLACE_SLP, bem.P1, 0.0, [0], np.arange(162), near=bem.NEAR_SKIP,
                           prec=bem.FP64)
    ref = om.entries(O.LAPLACE_SLP, O.P1, 0.0, [0], np.arange(162), near=O.NEAR_SKIP)
    assert normwise(got, ref) <= 1e-12


def test_argument_errors_and_edge_cases(sphere2):
    xyz, tri, mesh, om = sphere2
    with pytest.raises(bem.BemError) as ei:
        bem.eval_entries(mesh, bem.LAPLACE_SLP, bem.P0, 0.0, [0], [tri.shape[0]])
    assert ei.value.code == bem.E_ARG
    with pytest.raises(bem.BemError):
        bem.eval_entries(mesh, bem.LAPLACE_SLP, bem.P1, 0.0, [-1], [0])
    with pytest.raises(bem.BemError):
        bem.eval_entries(mesh, bem.LAPLACE_SLP, bem.P0, 1.0, [0], [5])
    with pytest.raises(bem.BemError):
        bem.eval_entries(mesh, bem.HELMHOLTZ_SLP, bem.P0, 0.0, [0], [5])
    assert bem.eval_entries(mesh, bem.LAPLACE_SLP, bem.P0, 0.0, [], [1, 2]).shape == (0, 2)
    assert bem.eval_entries(mesh, bem.HELMHOLTZ_DLP, bem.P1, 2.0, [3], []).shape == (1, 0)
    # duplicated indices give duplicated rows and columns
    rows = np.array([40, 40, 41], dtype=np.int32)
    cols = np.array([100, 150, 100, 160], dtype=np.int32)
    for space in (bem.P0, bem.P1):
        got = bem.eval_entries(mesh, bem.LAPLACE_DLP, space, 0.0, rows, cols)
        assert np.array_equal(got[0], got[1]) and np.array_equal(got[:, 0], got[:, 2])


def test_degenerate_mesh_rejected():
    xyz = np.array([[0, 0, 0], [1, 0, 0], [2, 0, 0], [0, 1, 0]], dtype=np.float64)
    tri = np.array([[0, 1, 2], [0, 1, 3]], dtype=np.int32)
    with pytest.raises(bem.BemError):
        bem.mesh_create(xyz, tri, 6)
    with pytest.raises(bem.BemError):
        bem.mesh_create(xyz, np.array([[0, 1, 3]], dtype=np.int32), 5)


def test_async_device_output_matches_sync(sphere2):
    import torch
    xyz, tri, mesh, om = sphere2
    rows = np.arange(0, 162, 3, dtype=np.int32)
    cols = np.arange(162, dtype=np.int32)
    for op, space, prec, dt in [(bem.LAPLACE_SLP, bem.P1, bem.FP32, torch.float32),
                                (bem.HELMHOLTZ_DLP, bem.P1, bem.FP64, torch.complex128),
                                (bem.HELMHOLTZ_SLP, bem.P0, bem.FP32, torch.complex64)]:
        n = 162 if space == bem.P1 else 320
        c = np.arange(n, dtype=np.int32)
        out = torch.empty((rows.size, n), dtype=dt, device="cuda")
        bem.eval_entries_async(mesh, op, space, K[op], rows, c, out, prec=prec)
        torch.cuda.synchronize()
        ref = bem.eval_entries(mesh, op, space, K[op], rows, c, prec=prec)
        assert np.array_equal(out.cpu().numpy(), ref)


def test_result_independent_of_batch_mix(sphere2):
    """Each request's result is bitwise the same alone and when it shares
    fused launches with other requests of other sizes and operators."""
    xyz, tri, mesh, om = sphere2
    rng = np.random.Generator(np.random.PCG64(2))
    reqs = []
    for i in range(60):
        op = OPS[i % 4]
        space = bem.P0 if i % 3 else bem.P1
        n = tri.shape[0] if space == bem.P0 else xyz.shape[0]
        nr, nc = (1, int(rng.integers(16, n))) if i % 2 else (int(rng.integers(16, n)), 1)
        rows = rng.choice(n, nr, replace=False).astype(np.int32)
        cols = rng.choice(n, nc, replace=False).astype(np.int32)
        reqs.append((op, space, rows, cols))
    alone = [bem.eval_entries(mesh, op, sp, K[op], r, c) for op, sp, r, c in reqs]
    tickets = [bem.submit(mesh, op, sp, K[op], r, c) for op, sp, r, c in reqs]
    mixed = [t.wait() for t in tickets]
    for a, b in zip(alone, mixed):
        assert np.array_equal(a, b)
    st = bem.server_stats()
    assert st["batches"] >= 1 and st["requests"] >= 120


def test_full_size_icosphere6_sampled_rows():
    """The 81,920-triangle / 40,962-vertex icosphere at full size: P1
    single- and double-layer rows and columns of admissible-block shape,
    FP32, against the oracle on a seeded sample."""
    xyz, tri = inputs.icosphere(6)
    mesh = bem.mesh_create(xyz, tri, 6)
    om = O.OracleMesh(xyz, tri, 6)
    perm, ranges, blocks = bem.partition(xyz, tri, bem.P1, 100, 1.0)
    adm = blocks[blocks[:, 2] == 1]
    rng = np.random.Generator(np.random.PCG64(3))
    pick = rng.choice(adm.shape[0], 8, replace=False)
    for b in pick:
        t, s = adm[b, 0], adm[b, 1]
        rows = perm[ranges[t, 0]:ranges[t, 1]]
        cols = perm[ranges[s, 0]:ranges[s, 1]]
        i = rows[int(rng.integers(rows.size))]
        for op in (bem.LAPLACE_SLP, bem.LAPLACE_DLP):
            got = bem.eval_entries(mesh, op, bem.P1, 0.0, [i], cols, prec=bem.FP32, near=bem.NEAR_ERROR)
            ref = om.entries(op, O.P1, 0.0, [i], cols)
            assert normwise(got.astype(np.float64), ref) <= 1e-5
            gotc = bem.eval_entries(mesh, op, bem.P1, 0.0, rows, cols[:1], prec=bem.FP32, near=bem.NEAR_ERROR)
            refc = om.entries(op, O.P1, 0.0, rows, cols[:1])
            assert normwise(gotc.astype(np.float64), refc) <= 1e-5
    mesh.destroy()


def test_p1_chunk_edge_cases():
    """P1 lane sides cut into chunks: a dof repeated far more often than a
    workgroup has threads, a vertex that belongs to no triangle (its entries
    are zero), and lane lists spanning many chunks, against the oracle."""
    xyz, tri = inputs.icosphere(2)
    xyz = np.vstack([xyz, [[5.0, 5.0, 5.0]]])          # vertex 162: in no triangle
    mesh = bem.mesh_create(xyz, tri, 6)
    om = O.OracleMesh(xyz, tri, 6)
    lone = xyz.shape[0] - 1
    rows = np.array([0, 77, lone], dtype=np.int32)
    cols = np.arange(xyz.shape[0], dtype=np.int32)
    for prec in (bem.FP64, bem.FP32):
        for op in (bem.LAPLACE_SLP, bem.HELMHOLTZ_DLP):
            got = bem.eval_entries(mesh, op, bem.P1, K[op], rows, cols, prec=prec, near=bem.NEAR_SKIP)
            ref = om.entries(op, O.P1, K[op], rows, cols, near=O.NEAR_SKIP)
            assert np.all(got[2] == 0) and np.all(got[:, lone] == 0)
            assert normwise(got.astype(ref.dtype), ref) <= tol(op, prec)
            # the transposed request runs with the row side on the lanes
            gotT = bem.eval_entries(mesh, op, bem.P1, K[op], cols, rows, prec=prec, near=bem.NEAR_SKIP)
            refT = om.entries(op, O.P1, K[op], cols, rows, near=O.NEAR_SKIP)
            assert normwise(gotT.astype(refT.dtype), refT) <= tol(op, prec)
    # 700 copies of one far dof: one chunk, 700 entries from the same partials
    rep = np.full(700, 120, dtype=np.int32)
    got = bem.eval_entries(mesh, bem.LAPLACE_SLP, bem.P1, 0.0, [3], rep, prec=bem.FP32)
    single = bem.eval_entries(mesh, bem.LAPLACE_SLP, bem.P1, 0.0, [3], [120], prec=bem.FP32)
    assert np.all(got == single[0, 0])
    mesh.destroy()


def _bipyramid(n, height=3.0):
    """Closed double cone: n rim vertices on the unit circle and two apexes at
    z = +-height, so both apex stars hold n triangles (outward winding)."""
    phi = 2.0 * np.pi * np.arange(n) / n
    xyz = np.vstack([np.stack([np.cos(phi), np.sin(phi), np.zeros(n)], axis=1), [[0.0, 0.0, height]],
                     [[0.0, 0.0, -height]]])
    top, bot = n, n + 1
    tri = []
    for i in range(n):
        j = (i + 1) % n
        tri.append([i, j, top])
        tri.append([j, i, bot])
    return xyz, np.array(tri, dtype=np.int32)


@pytest.mark.parametrize("n", [9, 20])
def test_p1_high_valence_stars_span_stages(n):
    """A P1 dof whose star has more triangles than one staging round holds
    (8): the apexes of a double cone with 9 and 20 rim vertices.  The row
    request stages the apex star on the test side, the transposed request on
    the trial side; both precisions, four operators, against the oracle with
    vertex-sharing pairs skipped on both sides."""
    xyz, tri = _bipyramid(n)
    mesh = bem.mesh_create(xyz, tri, 6)
    om = O.OracleMesh(xyz, tri, 6)
    apex = np.array([n, n + 1], dtype=np.int32)
    cols = np.arange(n + 2, dtype=np.int32)
    try:
        for op in (bem.LAPLACE_SLP, bem.LAPLACE_DLP, bem.HELMHOLTZ_SLP, bem.HELMHOLTZ_DLP):
            k = 2.0 if op in (bem.HELMHOLTZ_SLP, bem.HELMHOLTZ_DLP) else 0.0
            ref = om.entries(op, O.P1, k, apex, cols, near=O.NEAR_SKIP)
            refT = om.entries(op, O.P1, k, cols, apex, near=O.NEAR_SKIP)
            assert np.max(np.abs(ref)) > 0 and np.max(np.abs(refT)) > 0
            for prec in (bem.FP64, bem.FP32):
                got = bem.eval_entries(mesh, op, bem.P1, k, apex, cols, prec=prec, near=bem.NEAR_SKIP)
                gotT = bem.eval_entries(mesh, op, bem.P1, k, cols, apex, prec=prec, near=bem.NEAR_SKIP)
                assert normwise(got.astype(ref.dtype), ref) <= tol(op, prec), (n, op, prec)
                assert normwise(gotT.astype(refT.dtype), refT) <= tol(op, prec), (n, op, prec)
    finally:
        mesh.destroy()
