"""GPU parity of the hypersingular operator (Eq. hypsHelmholtz, P1) against
the FP64 oracle.

Tolerances: FP64 path, per-request normwise max|a-b| / max|b| <= 1e-11.
FP32 path: entries far from the diagonal cancel like (h/r)^2 (the curls of a
triangle's three hat functions sum to zero), so the FP32 rounding of each
pair integral (a few units of u = 2^-24) is amplified by that factor:
entrywise |a-b| <= 8 u (1 + (r/h)^2) |b| + 1e-6 max|b|, with r the distance
of the two vertices and h the mean edge length (measured: about 0.6 u
(r/h)^2 in the median on the level-4 icosphere).  Requests that hold near
entries also meet the normwise 1e-5 (Laplace) / 1e-4 (Helmholtz) of the
other operators.
"""
import numpy as np
import pytest

import oracle as O
from paper_1711_01897_amd import bem, inputs

pytestmark = pytest.mark.gpu

OPS = [(bem.LAPLACE_HYPS, 0.0), (bem.HELMHOLTZ_HYPS, 2.5)]


def normwise(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module", params=[2, 4])
def sphere(request):
    xyz, tri = inputs.icosphere(request.param)
    mesh = bem.mesh_create(xyz, tri, 6)
    yield xyz, tri, mesh, O.OracleMesh(xyz, tri, 6)
    mesh.destroy()


@pytest.mark.parametrize("op,k", OPS)
@pytest.mark.parametrize("prec", [bem.FP64, bem.FP32])
def test_hypersingular_requests_vs_oracle(sphere, op, k, prec):
    xyz, tri, mesh, om = sphere
    nv = xyz.shape[0]
    rng = np.random.Generator(np.random.PCG64(3))
    h = mesh.info().mean_edge
    u = 2.0 ** -24
    for nr, nc in [(1, 150), (150, 1), (37, 90), (1, 1), (129, 3)]:
        rows = rng.choice(nv, nr, replace=False).astype(np.int32)
        cols = rng.choice(nv, nc, replace=False).astype(np.int32)
        got = bem.eval_entries(mesh, op, bem.P1, k, rows, cols, prec=prec)
        ref = om.entries(op, O.P1, k, rows, cols)
        if np.max(np.abs(ref)) == 0:
            assert np.all(got == 0)
            continue
        err = np.abs(got.astype(ref.dtype) - ref)
        if prec == bem.FP64:
            assert err.max() / np.abs(ref).max() <= 1e-11, (nr, nc)
            continue
        r = np.linalg.norm(xyz[rows][:, None, :] - xyz[cols][None, :, :], axis=2)
        allowed = 8 * u * (1.0 + (r / h) ** 2) * np.abs(ref) + 1e-6 * np.abs(ref).max()
        assert np.all(err <= allowed), (nr, nc, float(np.max(err / allowed)))
        if nr * nc >= 150:
            assert normwise(got.astype(ref.dtype), ref) <= (1e-5 if op == bem.LAPLACE_HYPS else 1e-4)


@pytest.mark.parametrize("prec,bound", [(bem.FP64, 1e-14), (bem.FP32, 1e-6)])
def test_laplace_hypersingular_rows_sum_to_zero(sphere, prec, bound):
    """The Laplace hypersingular operator annihilates constants pair by pair."""
    xyz, tri, mesh, om = sphere
    nv = xyz.shape[0]
    rows = np.arange(0, nv, max(1, nv // 25), dtype=np.int32)
    D = bem.eval_entries(mesh, bem.LAPLACE_HYPS, bem.P1, 0.0, rows, np.arange(nv, dtype=np.int32), prec=prec)
    D = D.astype(np.float64)
    assert np.max(np.abs(D.sum(1)) / np.abs(D).sum(1)) <= bound


@pytest.mark.parametrize("op,k", OPS)
def test_hypersingular_symmetric_fp64(sphere, op, k):
    xyz, tri, mesh, om = sphere
    idx = np.random.Generator(np.random.PCG64(6)).choice(xyz.shape[0], 60, replace=False).astype(np.int32)
    D = bem.eval_entries(mesh, op, bem.P1, k, idx, idx, prec=bem.FP64)
    assert np.abs(D - D.T).max() <= 1e-13 * np.abs(D).max()


def test_hypersingular_hmat_matvec():
    xyz, tri = inputs.icosphere(3)
    mesh = bem.mesh_create(xyz, tri, 6)
    om = O.OracleMesh(xyz, tri, 6)
    H = bem.hmat_assemble(mesh, bem.LAPLACE_HYPS, bem.P1, 0.0, leaf_size=32, eta=1.0, aca_tol=1e-6, max_rank=100,
                          n_workers=4, blocks_per_worker=8, prec=bem.FP64, dense_mode=1)
    st = H.stats()
    n = st["ndof"]
    A = om.entries(O.LAPLACE_HYPS, O.P1, 0.0, np.arange(n), np.arange(n), near=O.NEAR_SKIP)
    x = np.random.Generator(np.random.PCG64(3)).normal(size=n)
    err = np.linalg.norm(H.matvec(x) - A @ x) / np.linalg.norm(A @ x)
    print(st, err)
    assert err <= 1e-5
    assert st["admissible_blocks"] > 0
    H.destroy()
    mesh.destroy()


def test_hypersingular_rejects_p0():
    xyz, tri = inputs.icosphere(1)
    mesh = bem.mesh_create(xyz, tri, 6)
    with pytest.raises(bem.BemError):
        bem.eval_entries(mesh, bem.LAPLACE_HYPS, bem.P0, 0.0, np.array([0], np.int32), np.array([5], np.int32))
    mesh.destroy()
