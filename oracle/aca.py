"""Adaptive cross approximation, FP64 (TEST INFRASTRUCTURE ONLY).

Follows Algorithm "ACA" of Section 2.1 (the recursion of Eq.
acaRecursionFormula, the column pivot as the largest entry of the residual
row), with the choices the paper leaves to the literature:

  * row pivot (Section 2.1 defers to Bebendorf, Section 3.4.3): start at the
    first local row; afterwards take the unused row where the newest column
    u_k has its largest modulus (partial pivoting); ties go to the lowest
    index;
  * "does not vanish": the residual row vanishes when max|v~| <= zero_abs,
    an absolute threshold supplied by the caller.  Before the first pivot a
    vanishing row is marked used and the next unused row (lowest index) is
    tried (a block may start with zero rows); after it, the row was chosen
    where the newest column is largest, so a vanishing residual there ends
    the approximation;
  * stopping criterion: ||u_k|| ||v_k|| <= tol ||S_k||_F, or every row used,
    or k = min(m, n), or k = max_rank; ||S_k||_F is updated from
    ||S_k||^2 = ||S_{k-1}||^2 + 2 Re sum_{l<k} (u_l^H u_k)(v_l^H v_k)
               + ||u_k||^2 ||v_k||^2.

The block is approximated by U V^T with U = [u_1..u_k], V = [v_1..v_k].
"""
from __future__ import annotations

import numpy as np


def aca(get_row, get_col, m: int, n: int, tol: float, max_rank: int, zero_abs: float = 0.0,
        dtype=np.float64):
    """Run ACA on an m x n block given row/column callbacks.

    get_row(i) returns block row i (length n), get_col(j) block column j
    (length m), both in local indices.  Returns (U, V, pivots) with U of
    shape (m, k), V of shape (n, k) and pivots the list of (i_k, j_k).
    """
    U: list[np.ndarray] = []
    V: list[np.ndarray] = []
    pivots: list[tuple[int, int]] = []
    used = np.zeros(m, dtype=bool)
    norm2 = 0.0
    k = 0
    i = 0
    limit = min(m, n, max_rank)
    while True:
        # residual row v~ = a_{i,:} - sum_l (u_l)_i v_l
        v = np.array(get_row(i), dtype=dtype, copy=True)
        for l in range(k):
            v = v - U[l][i] * V[l]
        used[i] = True
        if np.max(np.abs(v)) <= zero_abs:
            if used.all() or k > 0:
                break
            i = int(np.flatnonzero(~used)[0])
            continue
        j = int(np.argmax(np.abs(v)))  # first maximum = lowest index on ties
        v = v / v[j]
        u = np.array(get_col(j), dtype=dtype, copy=True)
        for l in range(k):
            u = u - V[l][j] * U[l]
        cross = 0.0
        for l in range(k):
            cross += (np.vdot(U[l], u) * np.vdot(V[l], v)).real
        nu = np.linalg.norm(u)
        nv = np.linalg.norm(v)
        norm2 = norm2 + 2.0 * cross + (nu * nv) ** 2
        U.append(u)
        V.append(v)
        pivots.append((i, j))
        k += 1
        if nu * nv <= tol * np.sqrt(max(norm2, 0.0)):
            break
        if used.all() or k >= limit:
            break
        cand = np.where(used, -1.0, np.abs(u))
        i = int(np.argmax(cand))
    if k == 0:
        return np.zeros((m, 0), dtype=dtype), np.zeros((n, 0), dtype=dtype), pivots, 0.0
    return np.stack(U, axis=1), np.stack(V, axis=1), pivots, float(np.sqrt(max(norm2, 0.0)))


def aca_dense(A: np.ndarray, tol: float, max_rank: int, zero_abs: float = 0.0):
    """ACA on an explicit matrix (rows/columns read from A)."""
    m, n = A.shape
    return aca(lambda i: A[i, :], lambda j: A[:, j], m, n, tol, max_rank, zero_abs, dtype=A.dtype)
