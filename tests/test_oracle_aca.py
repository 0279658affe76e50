"""Pins of the ACA oracle (Algorithm "ACA", Section 2.1).

  * exact-rank special case: a rank-r matrix is reproduced after r steps;
  * the running Frobenius norm of S_k equals ||U V^T||_F;
  * on admissible blocks of a real mesh the approximation error against the
    dense oracle block is bounded by a small multiple of the tolerance;
  * a vanishing residual row is skipped, not used as a pivot row, before
    the first pivot; after it, a vanishing residual at the pivot-row
    candidate ends the approximation instead of walking the other rows.
"""
import numpy as np
import pytest

import oracle as O
import oracle.aca as A
import oracle.tree as T
from paper_1711_01897_amd import inputs

RNG = np.random.Generator(np.random.PCG64(3))


@pytest.mark.parametrize("cplx", [False, True])
def test_exact_rank_reproduced(cplx):
    m, n, r = 60, 50, 5
    X = RNG.normal(size=(m, r))
    Y = RNG.normal(size=(n, r))
    if cplx:
        X = X + 1j * RNG.normal(size=(m, r))
        Y = Y + 1j * RNG.normal(size=(n, r))
    M = X @ Y.T
    U, V, piv, _ = A.aca_dense(M, tol=1e-14, max_rank=40, zero_abs=1e-9 * np.abs(M).max())
    assert U.shape[1] == r
    assert np.linalg.norm(M - U @ V.T) <= 1e-12 * np.linalg.norm(M)
    # the first pivot column is the largest entry of row 0
    assert piv[0] == (0, int(np.argmax(np.abs(M[0]))))


def test_norm_update_matches_direct_norm():
    m, n = 80, 70
    M = np.exp(-np.subtract.outer(np.linspace(0, 1, m), np.linspace(3, 4, n)) ** 2)
    U, V, _, est = A.aca_dense(M, tol=1e-10, max_rank=30)
    assert abs(est - np.linalg.norm(U @ V.T)) <= 1e-12 * est


def test_vanishing_rows_are_skipped():
    M = np.zeros((6, 5))
    M[3:] = RNG.normal(size=(3, 1)) @ RNG.normal(size=(1, 5))
    U, V, piv, _ = A.aca_dense(M, tol=1e-12, max_rank=5, zero_abs=1e-12)
    assert piv[0][0] == 3
    assert U.shape[1] == 1
    assert np.linalg.norm(M - U @ V.T) <= 1e-14 * np.linalg.norm(M)


def test_vanishing_row_after_a_pivot_stops():
    # rank 2 plus noise far below the vanishing threshold: after two pivots the
    # next candidate row's residual is noise, so ACA stops with one extra row
    # request instead of requesting every remaining row
    m, n = 40, 30
    M = RNG.normal(size=(m, 2)) @ RNG.normal(size=(2, n)) + 1e-10 * RNG.normal(size=(m, n))
    calls = {"row": 0, "col": 0}

    def row(i):
        calls["row"] += 1
        return M[i]

    def col(j):
        calls["col"] += 1
        return M[:, j]

    U, V, piv, _ = A.aca(row, col, m, n, tol=1e-14, max_rank=20, zero_abs=1e-7)
    assert U.shape[1] == 2
    assert calls == {"row": 3, "col": 2}
    assert np.linalg.norm(M - U @ V.T) <= 1e-8 * np.linalg.norm(M)
    # before the first pivot a vanishing row is skipped: zero leading rows are walked
    Z = M.copy()
    Z[:5] = 0.0
    U, V, piv, _ = A.aca_dense(Z, tol=1e-14, max_rank=20, zero_abs=1e-7)
    assert piv[0][0] == 5 and U.shape[1] == 2


def admissible_blocks(space, leaf=40, count=6):
    xyz, tri = inputs.icosphere(4)
    nodes, leaves = T.partition(xyz, tri, space, leaf, 1.0)
    adm = [(nodes[a].idx, nodes[b].idx) for a, b, ok in leaves if ok]
    adm.sort(key=lambda p: -(p[0].size * p[1].size))
    return xyz, tri, adm[:count]


@pytest.mark.parametrize("op,space,k", [(O.LAPLACE_SLP, O.P1, 0.0), (O.LAPLACE_DLP, O.P1, 0.0),
                                        (O.HELMHOLTZ_SLP, O.P0, 6.0)])
@pytest.mark.parametrize("tol", [1e-4, 1e-6])
def test_block_error_against_dense(op, space, k, tol):
    xyz, tri, blocks = admissible_blocks(space)
    m = O.OracleMesh(xyz, tri, 6)
    for rows, cols in blocks:
        D = m.entries(op, space, k, rows, cols, near=O.NEAR_ERROR)
        U, V, _, _ = A.aca(lambda i: m.entries(op, space, k, rows[i:i + 1], cols, near=O.NEAR_ERROR)[0],
                           lambda j: m.entries(op, space, k, rows, cols[j:j + 1], near=O.NEAR_ERROR)[:, 0],
                           rows.size, cols.size, tol, 200, zero_abs=1e-14 * np.abs(D).max(),
                           dtype=D.dtype)
        err = np.linalg.norm(D - U @ V.T) / np.linalg.norm(D)
        assert err <= 10 * tol, (rows.size, cols.size, U.shape[1], err)
        assert U.shape[1] < min(rows.size, cols.size) // 2
