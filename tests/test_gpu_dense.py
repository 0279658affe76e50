"""GPU: pair-based P1 blocks (bem_eval_dense), the dense assembly.

  * the full dense P1 matrix of the level-3 icosphere (642 x 642, vertex-
    sharing pairs skipped) against the oracle: FP64 1e-12 (single layer
    entrywise, double layer normwise), FP32 1e-5, Helmholtz 1e-11 / 1e-4;
  * against the star kernels (bem_eval_entries) on the same block (FP64,
    the same sums in another order);
  * row panels: a small device budget cuts the block into many panels and
    leaves every entry bitwise unchanged (each entry's sum does not depend on
    the panel that holds it);
  * sampled rows of the level-4 icosphere's full matrix, ragged shapes and
    duplicated indices; BEM_NEAR_ERROR fails before anything runs.
"""
import os

import numpy as np
import pytest

import oracle as O
from paper_1711_01897_amd import bem, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ico3():
    xyz, tri = inputs.icosphere(3)
    mesh = bem.mesh_create(xyz, tri, 6)
    yield xyz, tri, mesh, O.OracleMesh(xyz, tri, 6)
    mesh.destroy()


def rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("op,k", [(bem.LAPLACE_SLP, 0.0), (bem.LAPLACE_DLP, 0.0), (bem.HELMHOLTZ_SLP, 3.0),
                                  (bem.HELMHOLTZ_DLP, 3.0)])
def test_full_dense_p1_matrix_vs_oracle(ico3, op, k):
    xyz, tri, mesh, om = ico3
    idx = np.arange(xyz.shape[0], dtype=np.int32)
    ref = om.entries(op, O.P1, k, idx, idx, near=O.NEAR_SKIP)
    g64, st = bem.eval_dense(mesh, op, bem.P1, k, idx, idx, prec=bem.FP64, stats=True)
    g32 = bem.eval_dense(mesh, op, bem.P1, k, idx, idx, prec=bem.FP32)
    assert st["pairs"] == tri.shape[0] ** 2   # every pair once (one panel covers all rows)
    if op == bem.LAPLACE_SLP:
        nz = ref != 0
        assert np.all(g64[~nz] == 0) and np.all(g32[~nz] == 0)
        assert np.max(np.abs(g64[nz] - ref[nz]) / np.abs(ref[nz])) <= 1e-12
        assert np.max(np.abs(g32[nz] - ref[nz]) / np.abs(ref[nz])) <= 1e-5
    else:
        assert rel(g64, ref) <= 1e-11
        assert rel(g32.astype(ref.dtype), ref) <= (1e-4 if bem.is_complex(op) else 1e-5)
    # the star kernels give the same block in another summation order
    s64 = bem.eval_entries(mesh, op, bem.P1, k, idx, idx, prec=bem.FP64, near=bem.NEAR_SKIP)
    assert rel(g64, s64) <= 1e-13


def test_panels_leave_entries_unchanged(ico3, monkeypatch):
    xyz, tri, mesh, om = ico3
    idx = np.arange(xyz.shape[0], dtype=np.int32)
    one = bem.eval_dense(mesh, bem.LAPLACE_DLP, bem.P1, 0.0, idx, idx, prec=bem.FP32)
    monkeypatch.setenv("BEM_DENSE_BUDGET_MB", "16")
    many, st = bem.eval_dense(mesh, bem.LAPLACE_DLP, bem.P1, 0.0, idx, idx, prec=bem.FP32, stats=True)
    assert st["panels"] > 2
    assert np.array_equal(one, many)


def test_level4_sampled_rows_ragged_and_duplicates():
    xyz, tri = inputs.icosphere(4)
    mesh = bem.mesh_create(xyz, tri, 6)
    om = O.OracleMesh(xyz, tri, 6)
    nv = xyz.shape[0]
    rng = np.random.Generator(np.random.PCG64(41))
    cols = np.arange(nv, dtype=np.int32)
    rows = rng.choice(nv, 37, replace=False).astype(np.int32)
    rows = np.concatenate([rows, rows[:5]])   # duplicated rows
    got = bem.eval_dense(mesh, bem.LAPLACE_SLP, bem.P1, 0.0, rows, cols, prec=bem.FP32)
    ref = om.entries(O.LAPLACE_SLP, O.P1, 0.0, rows, cols)
    nz = ref != 0
    assert np.max(np.abs(got[nz] - ref[nz]) / np.abs(ref[nz])) <= 1e-5
    assert np.array_equal(got[:5], got[37:])
    for shape in ((1, 1), (1, 500), (500, 1), (129, 3)):
        r = rng.choice(nv, shape[0], replace=False).astype(np.int32)
        c = rng.choice(nv, shape[1], replace=False).astype(np.int32)
        g = bem.eval_dense(mesh, bem.HELMHOLTZ_DLP, bem.P1, 5.0, r, c, prec=bem.FP64)
        f = om.entries(O.HELMHOLTZ_DLP, O.P1, 5.0, r, c)
        if np.abs(f).max() > 0:
            assert rel(g, f) <= 1e-11
    far_rows = np.array([0], dtype=np.int32)
    with pytest.raises(bem.NearFieldError):
        bem.eval_dense(mesh, bem.LAPLACE_SLP, bem.P1, 0.0, far_rows, cols, prec=bem.FP32, near=bem.NEAR_ERROR)
    with pytest.raises(bem.BemError):
        bem.eval_dense(mesh, bem.LAPLACE_SLP, bem.P0, 0.0, far_rows, cols, prec=bem.FP32)
    assert bem.eval_dense(mesh, bem.LAPLACE_SLP, bem.P1, 0.0, far_rows[:0], cols, prec=bem.FP32).shape == (0, nv)
    mesh.destroy()
