"""Host-side checks of the C-ABI library (no GPU needed).

  * libbem.so loads and exports every function include/bem.h declares;
  * the library's geometric partition equals the oracle's, block for block;
  * the library's ACA (bem_aca_callback, same state machine the device path
    uses) reproduces the oracle's ACA pivots and factors on the same entries;
  * the device quadrature table agrees with the oracle's rule.
"""
import os
import re

import numpy as np
import pytest

import oracle as O
import oracle.aca as OA
import oracle.tree as OT
from paper_1711_01897_amd import bem, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bem.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bem_\w+)\s*\(", text)) - {"bem_row_fn", "bem_col_fn"})


def test_library_exports_every_declared_symbol():
    L = bem.lib()
    names = declared_functions()
    assert names, "no declarations found"
    for n in names:
        assert hasattr(L, n), n
    assert sorted(bem.EXPORTS) == names


def test_library_error_path_without_device():
    # argument validation happens before any device work
    with pytest.raises(bem.BemError):
        bem.mesh_create(np.zeros((3, 3)), np.array([[0, 1, 5]], dtype=np.int32))


@pytest.mark.parametrize("space,level,leaf,max_block", [(0, 3, 32, 0), (1, 3, 32, 0), (1, 6, 100, 0), (0, 5, 100, 0),
                                                        (1, 5, 16, 256), (0, 4, 16, 64), (2, 3, 48, 0),
                                                        (2, 4, 100, 512)])
def test_partition_matches_oracle(space, level, leaf, max_block):
    xyz, tri = inputs.icosphere(level)
    perm, ranges, blocks = bem.partition(xyz, tri, space, leaf, 1.0, max_block)
    nodes, leaves = OT.partition(xyz, tri, space, leaf, 1.0, max_block)
    assert len(nodes) == ranges.shape[0]
    for c, node in enumerate(nodes):
        b, e = ranges[c]
        if node.children:
            assert np.array_equal(np.sort(perm[b:e]), np.sort(node.idx)), c
        else:
            assert np.array_equal(perm[b:e], node.idx), c
    assert [tuple(x) for x in blocks] == [(a, b, int(ok)) for a, b, ok in leaves]


def test_partition_matches_oracle_on_spheroid():
    xyz, tri = inputs.spheroid(10.0, 1.0, 20000)
    perm, ranges, blocks = bem.partition(xyz, tri, 0, 64, 1.0)
    nodes, leaves = OT.partition(xyz, tri, 0, 64, 1.0)
    assert [tuple(x) for x in blocks] == [(a, b, int(ok)) for a, b, ok in leaves]
    for c, node in enumerate(nodes):
        got = perm[ranges[c, 0]:ranges[c, 1]]
        assert np.array_equal(got if not node.children else np.sort(got),
                              node.idx if not node.children else np.sort(node.idx))


@pytest.mark.parametrize("cplx", [False, True])
def test_aca_callback_exact_rank(cplx):
    rng = np.random.Generator(np.random.PCG64(3))
    m, n, r = 70, 55, 6
    X, Y = rng.normal(size=(m, r)), rng.normal(size=(n, r))
    if cplx:
        X = X + 1j * rng.normal(size=(m, r))
        Y = Y + 1j * rng.normal(size=(n, r))
    M = X @ Y.T
    za = 1e-9 * np.abs(M).max()
    U, V = bem.aca_callback(lambda i: M[i], lambda j: M[:, j], m, n, 1e-14, 40, za, cplx)
    Uo, Vo, _, _ = OA.aca_dense(M, 1e-14, 40, za)
    assert U.shape == Uo.shape == (m, r)
    assert np.abs(U - Uo).max() <= 1e-12 * np.abs(Uo).max()
    assert np.abs(V - Vo).max() <= 1e-12 * np.abs(Vo).max()


def test_aca_callback_stops_at_a_vanishing_row_like_the_oracle():
    # after the first pivot a vanishing residual row ends the approximation in
    # both state machines: same rank, same number of row and column requests
    rng = np.random.Generator(np.random.PCG64(3))
    m, n = 40, 30
    M = rng.normal(size=(m, 2)) @ rng.normal(size=(2, n)) + 1e-10 * rng.normal(size=(m, n))
    counts = []
    for run in ("lib", "oracle"):
        c = {"row": 0, "col": 0}

        def row(i, c=c):
            c["row"] += 1
            return M[i]

        def col(j, c=c):
            c["col"] += 1
            return M[:, j]

        if run == "lib":
            U, V = bem.aca_callback(row, col, m, n, 1e-14, 20, 1e-7, False)
        else:
            U, V, _, _ = OA.aca(row, col, m, n, 1e-14, 20, 1e-7)
        counts.append((U.shape[1], c["row"], c["col"]))
    assert counts[0] == counts[1] == (2, 3, 2)


@pytest.mark.parametrize("op,space,k", [(O.LAPLACE_SLP, O.P1, 0.0), (O.LAPLACE_DLP, O.P1, 0.0),
                                        (O.HELMHOLTZ_SLP, O.P0, 5.0), (O.HELMHOLTZ_DLP, O.P0, 5.0)])
def test_aca_callback_matches_oracle_on_admissible_blocks(op, space, k):
    xyz, tri = inputs.icosphere(4)
    nodes, leaves = OT.partition(xyz, tri, space, 40, 1.0)
    adm = sorted([(nodes[a].idx, nodes[b].idx) for a, b, ok in leaves if ok], key=lambda p: -p[0].size * p[1].size)
    m = O.OracleMesh(xyz, tri, 6)
    for rows, cols in adm[:4]:
        D = m.entries(op, space, k, rows, cols, near=O.NEAR_ERROR)
        za = 1e-12 * np.abs(D).max()
        Uo, Vo, piv, _ = OA.aca_dense(D, 1e-6, 100, za)
        U, V = bem.aca_callback(lambda i: D[i], lambda j: D[:, j], rows.size, cols.size, 1e-6, 100, za,
                                np.iscomplexobj(D))
        assert U.shape == Uo.shape
        assert np.abs(U @ V.T - Uo @ Vo.T).max() <= 1e-12 * np.abs(D).max()


def test_device_rule_table_matches_oracle():
    text = open(os.path.join(ROOT, "paper_1711_01897_amd", "csrc", "quad_rules.hpp")).read()
    vals = dict(re.findall(r"constexpr double (kA1|kA2|kW1|kW2) = ([0-9.eE+-]+)", text))
    a1, a2 = float(vals["kA1"]), float(vals["kA2"])
    w1, w2 = float(vals["kW1"]) * 0.5, float(vals["kW2"]) * 0.5
    xi, eta, w = O.rule(6)
    pts = sorted(zip(np.round(xi, 14), np.round(eta, 14), np.round(w, 14)))
    mine = sorted([(round(a, 14), round(b, 14), round(c, 14)) for a, b, c in
                   [(a1, a1, w1), (1 - 2 * a1, a1, w1), (a1, 1 - 2 * a1, w1),
                    (a2, a2, w2), (1 - 2 * a2, a2, w2), (a2, 1 - 2 * a2, w2)]])
    assert np.allclose(np.array(pts), np.array(mine), rtol=0, atol=2e-15)


def test_server_config_rejects_small_arena():
    """Argument checks run before the device is touched."""
    with pytest.raises(bem.BemError) as ei:
        bem.server_config(1 << 20)
    assert ei.value.code == bem.E_ARG
    with pytest.raises(bem.BemError) as ei:
        bem.server_config(64 << 20, 0)
    assert ei.value.code == bem.E_ARG


def test_hypersingular_p0_rejected_on_host():
    """Argument checks run before anything reaches a device."""
    from paper_1711_01897_amd import bem
    assert bem.LAPLACE_HYPS == 6 and bem.HELMHOLTZ_HYPS == 7
    assert bem.is_complex(bem.HELMHOLTZ_HYPS) and not bem.is_complex(bem.LAPLACE_HYPS)
