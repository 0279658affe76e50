"""GPU parity at the full sizes of the stated workloads, on sampled requests.

Each case builds the full mesh, partitions it like the assembly does, picks
seeded admissible blocks plus the two largest ones, and compares one ACA row
request and one column request per block (the request shapes the served
path evaluates) with the FP64 oracle:
  * 10:1:1 prolate spheroid, 262,186 triangles, Helmholtz single layer, P0,
    4-point rule, k at 10 elements per wavelength: complex64 (FP32 path,
    1e-4) and complex128 (FP64 path, 1e-11);
  * the same spheroid refined to 400,140 triangles at 2 elements per
    wavelength (the largest mesh and coarsest sampling of the mixed
    Helmholtz workload; phases up to ~2,600 rad): complex64, 1e-4;
  * capped cylinder (R = 1, L = 16, +-1% jitter), 1,049,540 triangles,
    Laplace single layer, P1, 6-point rule, leaf 16: FP32, 1e-5.
Error measure: per-request normwise max|a - b| / max|b|.
"""
import numpy as np
import pytest

import oracle as O
from paper_1711_01897_amd import bem, inputs

pytestmark = pytest.mark.gpu


def normwise(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def sampled_blocks(xyz, tri, space, leaf, nblocks, seed):
    perm, ranges, blocks = bem.partition(xyz, tri, space, leaf, 1.0)
    adm = blocks[blocks[:, 2] == 1]
    rng = np.random.Generator(np.random.PCG64(seed))
    # seeded random blocks (mostly small and close) plus the two largest
    # (far apart: the longest distances and phases)
    size = (ranges[adm[:, 0], 1] - ranges[adm[:, 0], 0]) + (ranges[adm[:, 1], 1] - ranges[adm[:, 1], 0])
    pick = list(rng.choice(adm.shape[0], nblocks, replace=False)) + list(np.argsort(size)[-2:])
    out = []
    for b in pick:
        t, s = adm[b, 0], adm[b, 1]
        rows = perm[ranges[t, 0]:ranges[t, 1]].astype(np.int32)
        cols = perm[ranges[s, 0]:ranges[s, 1]].astype(np.int32)
        out.append((rows, cols, int(rng.integers(rows.size)), int(rng.integers(cols.size))))
    return out


def check_blocks(mesh, om, op, space, k, blocks, prec, bound):
    worst = 0.0
    for rows, cols, i, j in blocks:
        for r, c in (([rows[i]], cols), (rows, [cols[j]])):
            got = bem.eval_entries(mesh, op, space, k, np.asarray(r, np.int32), np.asarray(c, np.int32), prec=prec,
                                   near=bem.NEAR_ERROR)
            ref = om.entries(op, space, k, r, c)
            e = normwise(got.astype(ref.dtype), ref)
            worst = max(worst, e)
            assert e <= bound, (len(r), len(c), e)
    return worst


def test_spheroid_262k_helmholtz_p0_ten_per_wavelength():
    xyz, tri = inputs.spheroid(10.0, 1.0, 262144)
    assert tri.shape[0] == 262186
    k = inputs.wavenumber(xyz, tri, 10.0)
    mesh = bem.mesh_create(xyz, tri, 4)
    om = O.OracleMesh(xyz, tri, 4)
    blocks = sampled_blocks(xyz, tri, bem.P0, 100, 6, seed=3)
    w32 = check_blocks(mesh, om, bem.HELMHOLTZ_SLP, bem.P0, k, blocks, bem.FP32, 1e-4)
    w64 = check_blocks(mesh, om, bem.HELMHOLTZ_SLP, bem.P0, k, blocks, bem.FP64, 1e-11)
    print(f"k={k:.2f} complex64 {w32:.2e} complex128 {w64:.2e}")
    mesh.destroy()


def test_spheroid_400k_helmholtz_p0_two_per_wavelength():
    xyz, tri = inputs.spheroid(10.0, 1.0, 400000)
    k = inputs.wavenumber(xyz, tri, 2.0)
    mesh = bem.mesh_create(xyz, tri, 4)
    om = O.OracleMesh(xyz, tri, 4)
    blocks = sampled_blocks(xyz, tri, bem.P0, 100, 6, seed=3)
    w32 = check_blocks(mesh, om, bem.HELMHOLTZ_SLP, bem.P0, k, blocks, bem.FP32, 1e-4)
    print(f"k={k:.2f} complex64 {w32:.2e}")
    mesh.destroy()


def test_cylinder_1m_laplace_p1_leaf16():
    xyz, tri = inputs.capped_cylinder()
    assert tri.shape[0] == 1049540
    mesh = bem.mesh_create(xyz, tri, 6)
    om = O.OracleMesh(xyz, tri, 6)
    blocks = sampled_blocks(xyz, tri, bem.P1, 16, 6, seed=3)
    w = check_blocks(mesh, om, bem.LAPLACE_SLP, bem.P1, 0.0, blocks, bem.FP32, 1e-5)
    print(f"FP32 {w:.2e}")
    mesh.destroy()


def test_spheroid_262k_helmholtz_singular_pairs_sampled():
    """The singular scheme at the full spheroid size (262,186 triangles,
    10 elements per wavelength): requests of seeded triangles against their
    neighbourhoods with BEM_NEAR_SINGULAR; regular entries bitwise those of
    BEM_NEAR_SKIP, vertex-sharing entries against the oracle's Helmholtz
    near-field (levels 3 and 4 extrapolated, ~1e-7 here) within 1e-6 of the
    largest (FP64) and 2e-6 (complex64)."""
    xyz, tri = inputs.spheroid(10.0, 1.0, 262144)
    k = inputs.wavenumber(xyz, tri, 10.0)
    mesh = bem.mesh_create(xyz, tri, 4)
    om = O.OracleMesh(xyz, tri, 4)
    rng = np.random.Generator(np.random.PCG64(5))
    rows = np.sort(rng.choice(tri.shape[0], 4, replace=False)).astype(np.int32)
    # columns: every triangle around the rows' vertices plus a few distant ones
    near_cols = np.flatnonzero(np.isin(tri, tri[rows].ravel()).any(1))
    cols = np.unique(np.concatenate([near_cols, rng.choice(tri.shape[0], 16, replace=False)])).astype(np.int32)
    near = np.array([[len(set(tri[a]) & set(tri[b])) > 0 for b in cols] for a in rows])
    ri, ci = np.nonzero(near)
    ref = (4 * om.nearfield_entries(bem.HELMHOLTZ_SLP, k, rows[ri], cols[ci], 4, 2) -
           om.nearfield_entries(bem.HELMHOLTZ_SLP, k, rows[ri], cols[ci], 3, 2)) / 3
    for prec, bound in ((bem.FP64, 1e-6), (bem.FP32, 2e-6)):
        got = bem.eval_entries(mesh, bem.HELMHOLTZ_SLP, bem.P0, k, rows, cols, prec=prec, near=bem.NEAR_SINGULAR)
        skip = bem.eval_entries(mesh, bem.HELMHOLTZ_SLP, bem.P0, k, rows, cols, prec=prec, near=bem.NEAR_SKIP)
        assert np.array_equal(got[~near], skip[~near])
        err = np.abs(got[near].astype(np.complex128) - ref).max() / np.abs(ref).max()
        print(f"prec {prec}: {near.sum()} singular entries, k={k:.2f}, max rel err {err:.2e}")
        assert err <= bound
    mesh.destroy()
