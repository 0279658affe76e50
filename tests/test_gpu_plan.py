"""GPU: served ACA block streams (bem_aca_plan_*).

A plan keeps the partition and resident lane sets of one operator; runs
approximate lists of its admissible blocks as Poisson-arriving streams.
Checks: every block's U V^T against the dense oracle block (within a small
multiple of the tolerance), the same factors whether the blocks arrive at
once or spread out in time (the pivots depend only on the block's entries,
and a request's entries do not depend on the batch it lands in), a second
run replacing the first, the largest block dimension of the partition, FP32
request counts against FP64 ones, and argument errors.
"""
import numpy as np
import pytest

import oracle as O
from paper_1711_01897_amd import bem, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sphere4():
    xyz, tri = inputs.icosphere(4)
    return xyz, tri, bem.mesh_create(xyz, tri, 6), O.OracleMesh(xyz, tri, 6)


@pytest.mark.parametrize("op", [bem.LAPLACE_SLP, bem.LAPLACE_DLP])
def test_plan_blocks_against_dense_oracle(sphere4, op):
    xyz, tri, mesh, om = sphere4
    plan = bem.aca_plan_create(mesh, op, bem.P1, 0.0, leaf_size=16, eta=1.0, aca_tol=1e-5, max_rank=100,
                               n_workers=4, blocks_per_worker=16, prec=bem.FP32, max_block=128)
    nb = plan.info()["blocks"]
    rng = inputs.rng(inputs.SEED_SAMPLING)
    sel = rng.choice(nb, size=min(nb, 300), replace=False)
    arr = np.cumsum(rng.exponential(2e-5, size=sel.size))
    st = plan.run(sel, arr, bem.FP32)
    assert st["blocks"] == sel.size and st["entries"] > 0
    for b in sel[:40]:
        rows, cols = plan.block(b)
        assert max(rows.size, cols.size) <= 128
        D = om.entries(op, bem.P1, 0.0, rows, cols, near=O.NEAR_ERROR)
        U, V = plan.factors(b)
        err = np.linalg.norm(D - U @ V.T) / np.linalg.norm(D)
        assert err <= 10 * 1e-5, (b, rows.size, cols.size, U.shape[1], err)
    # all at once: the same blocks give the same factors, bit for bit
    keep = {int(b): plan.factors(b) for b in sel[:20]}
    st2 = plan.run(sel, None, bem.FP32)
    assert st2["entries"] == st["entries"] and st2["rank_sum"] == st["rank_sum"]
    for b, (U, V) in keep.items():
        U2, V2 = plan.factors(b)
        assert np.array_equal(U, U2) and np.array_equal(V, V2)
    plan.destroy()


def test_plan_runs_replace_factors_and_check_arguments(sphere4):
    xyz, tri, mesh, om = sphere4
    plan = bem.aca_plan_create(mesh, bem.LAPLACE_SLP, bem.P1, 0.0, leaf_size=16, eta=1.0, aca_tol=1e-5,
                               max_rank=100, n_workers=2, blocks_per_worker=8, prec=bem.FP32, max_block=128)
    nb = plan.info()["blocks"]
    plan.run(np.arange(0, 50), None, bem.FP32)
    plan.run(np.arange(50, 60), None, bem.FP64)
    U, V = plan.factors(55)
    assert U.dtype == np.float64 and U.shape[1] >= 1
    with pytest.raises(bem.BemError):
        plan.factors(10)   # not in the last run
    with pytest.raises(bem.BemError):
        plan.run(np.array([nb]), None, bem.FP32)
    with pytest.raises(bem.BemError):
        plan.run(np.array([1, 2]), np.array([0.2, 0.1]), bem.FP32)
    st = plan.run(np.array([], dtype=np.int64), None, bem.FP32)
    assert st["blocks"] == 0 and st["entries"] == 0
    plan.destroy()


def test_plan_fp32_requests_close_to_fp64(sphere4):
    # with the vanishing-row rule ending converged blocks, FP32 entries need
    # about as many requests as FP64 ones on the same blocks
    xyz, tri, mesh, om = sphere4
    for op in (bem.LAPLACE_SLP, bem.LAPLACE_DLP):
        plan = bem.aca_plan_create(mesh, op, bem.P1, 0.0, leaf_size=16, eta=1.0, aca_tol=1e-5, max_rank=100,
                                   n_workers=4, blocks_per_worker=32, prec=bem.FP32, max_block=256)
        allb = np.arange(plan.info()["blocks"])
        s32 = plan.run(allb, None, bem.FP32)
        s64 = plan.run(allb, None, bem.FP64)
        assert s32["requests"] <= 1.05 * s64["requests"], (op, s32["requests"], s64["requests"])
        assert s32["rank_sum"] <= 1.2 * s64["rank_sum"]
        plan.destroy()


def test_plans_run_serves_several_plans_in_one_stream():
    """One pool of workers over the blocks of four plans (two meshes x two
    wavenumbers, Helmholtz single layer P0): every block's factors equal those
    of its plan run alone (bit for bit: the pivots depend only on the block's
    entries, and a request's entries do not depend on the batch it lands in),
    sampled blocks match the dense oracle block, and mixed value types or bad
    indices are refused."""
    meshes = []
    for xyz, tri in (inputs.icosphere(3), inputs.spheroid(10.0, 1.0, 4000)):
        meshes.append((xyz, tri, bem.mesh_create(xyz, tri, 4), O.OracleMesh(xyz, tri, 4)))
    plans, ks, oms = [], [], []
    for xyz, tri, mesh, om in meshes:
        for epw in (5.0, 10.0):
            k = inputs.wavenumber(xyz, tri, epw)
            plans.append(bem.aca_plan_create(mesh, bem.HELMHOLTZ_SLP, bem.P0, k, leaf_size=16, eta=1.0,
                                             aca_tol=1e-4, max_rank=100, n_workers=1, blocks_per_worker=8,
                                             prec=bem.FP32))
            ks.append(k)
            oms.append(om)
    rng = inputs.rng(inputs.SEED_REQUESTS)
    pidx, blocks = [], []
    for p, pl in enumerate(plans):
        sel = rng.choice(pl.info()["blocks"], size=60, replace=False)
        pidx += [p] * sel.size
        blocks += list(sel)
    order = rng.permutation(len(blocks))
    pidx, blocks = np.array(pidx)[order], np.array(blocks)[order]
    arr = np.cumsum(rng.exponential(1e-5, size=blocks.size))
    st = bem.aca_plans_run(plans, pidx, blocks, arr, bem.FP32, n_workers=6, blocks_per_worker=16)
    assert st["blocks"] == blocks.size and st["entries"] > 0
    together = {(int(p), int(b)): plans[p].factors(b) for p, b in zip(pidx, blocks)}
    for p, pl in enumerate(plans):
        mine = blocks[pidx == p]
        pl.run(mine, None, bem.FP32)
        for b in mine:
            U, V = pl.factors(b)
            U2, V2 = together[(p, int(b))]
            assert np.array_equal(U, U2) and np.array_equal(V, V2)
        for b in mine[:5]:
            rows, cols = pl.block(b)
            D = oms[p].entries(O.HELMHOLTZ_SLP, O.P0, ks[p], rows, cols, near=O.NEAR_ERROR)
            U, V = pl.factors(b)
            assert np.linalg.norm(D - U @ V.T) / np.linalg.norm(D) <= 10 * 1e-4
    lap = bem.aca_plan_create(meshes[0][2], bem.LAPLACE_SLP, bem.P0, 0.0, leaf_size=16, eta=1.0, aca_tol=1e-4,
                              max_rank=100, n_workers=1, blocks_per_worker=8, prec=bem.FP32)
    with pytest.raises(bem.BemError):
        bem.aca_plans_run([plans[0], lap], [0, 1], [0, 0])
    with pytest.raises(bem.BemError):
        bem.aca_plans_run(plans, [0, 9], [0, 0])
    lap.destroy()
    for pl in plans:
        pl.destroy()
    for xyz, tri, mesh, om in meshes:
        mesh.destroy()
