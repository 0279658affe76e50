"""GPU: persistent launches serving the request server's fast batches.

With BEM_SERVER_PERSIST=1 (the default) each closed batch of ACA rows and
columns is published to one resident launch of its kernel variant, which
claims the batch's blocks and stores a completion word per batch; with 0
every batch is a launch of its own.  Checks: the same factors bit for bit
both ways (a request's entries do not depend on how its blocks are served),
launches that end after a short idle time and start again (many launches,
the same factors), batches of two kernel variants interleaved in one stream
(a launch of one variant ends once a batch of the other finds it idle; that
batch is launched on its own), FP64 and P0 variants, and the statistics
record of the resident launches.
"""
import os

import numpy as np
import pytest

from paper_1711_01897_amd import bem, inputs

pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="persistent launches are switched off: two variants stalled the served "
                                      "ACA run of the first test (a batch never completed) and the cause was not "
                                      "found; not to be run on the GPU until it is")]

_KNOBS = ("BEM_SERVER_PERSIST", "BEM_SERVER_PERSIST_IDLE_US", "BEM_SERVER_PERSIST_WGS")


def _restart(**env):
    """Sets the server's persistent-launch knobs (None: default) and restarts
    the idle server so that it reads them."""
    for k in _KNOBS:
        v = env.get(k)
        if v is None:
            os.environ.pop(k, None)
        else:
            os.environ[k] = str(v)
    bem.server_config(1 << 30)


@pytest.fixture(scope="module")
def sphere4():
    xyz, tri = inputs.icosphere(4)
    mesh = bem.mesh_create(xyz, tri, 6)
    yield mesh
    _restart()


def _plan(mesh, op, space=bem.P1, prec=bem.FP32):
    return bem.aca_plan_create(mesh, op, space, 0.0, leaf_size=16, eta=1.0, aca_tol=1e-5, max_rank=100,
                               n_workers=4, blocks_per_worker=16, prec=prec, max_block=128)


def _factors(plan, blocks):
    return {int(b): plan.factors(b) for b in blocks}


def _same(fa, fb):
    assert fa.keys() == fb.keys()
    for b in fa:
        (U, V), (U2, V2) = fa[b], fb[b]
        assert np.array_equal(U, U2) and np.array_equal(V, V2), b


def _persistent_records(ks):
    return [k for k in ks if k["persistent"]]


@pytest.mark.parametrize("space,prec", [(bem.P1, bem.FP32), (bem.P1, bem.FP64), (bem.P0, bem.FP32)])
def test_persistent_and_launched_batches_give_the_same_factors(sphere4, space, prec):
    plan = _plan(sphere4, bem.LAPLACE_SLP, space, prec)
    rng = inputs.rng(inputs.SEED_SAMPLING)
    sel = rng.choice(plan.info()["blocks"], size=min(plan.info()["blocks"], 400), replace=False)
    _restart(BEM_SERVER_PERSIST=0)
    bem.server_kernel_stats(reset=True)
    st0 = plan.run(sel, None, prec)
    f0 = _factors(plan, sel)
    assert not _persistent_records(bem.server_kernel_stats(reset=True))
    _restart(BEM_SERVER_PERSIST=1)
    bem.server_kernel_stats(reset=True)
    st1 = plan.run(sel, None, prec)
    ks = _persistent_records(bem.server_kernel_stats(reset=True))
    assert st1["entries"] == st0["entries"] and st1["rank_sum"] == st0["rank_sum"]
    _same(f0, _factors(plan, sel))
    # the resident launches served the run: one record of this variant with its work
    assert len(ks) == 1 and ks[0]["op"] == bem.LAPLACE_SLP and ks[0]["space"] == space
    assert ks[0]["prec"] == prec and ks[0]["launches"] >= 1 and ks[0]["pair_evals"] > 0
    assert ks[0]["seconds_events"] > 0 and ks[0]["workgroups"] > ks[0]["launches"]
    plan.destroy()


def test_launches_that_end_when_idle_start_again(sphere4):
    plan = _plan(sphere4, bem.LAPLACE_DLP)
    rng = inputs.rng(inputs.SEED_REQUESTS)
    sel = rng.choice(plan.info()["blocks"], size=300, replace=False)
    _restart(BEM_SERVER_PERSIST=0)
    plan.run(sel, None, bem.FP32)
    f0 = _factors(plan, sel)
    # arrivals ~200 us apart against a 20 us idle limit: launches end and
    # start again all through the run
    _restart(BEM_SERVER_PERSIST=1, BEM_SERVER_PERSIST_IDLE_US=20)
    bem.server_kernel_stats(reset=True)
    arr = np.cumsum(rng.exponential(2e-4, size=sel.size))
    st = plan.run(sel, arr, bem.FP32)
    ks = _persistent_records(bem.server_kernel_stats(reset=True))
    assert st["blocks"] == sel.size
    _same(f0, _factors(plan, sel))
    assert len(ks) == 1 and ks[0]["launches"] > 5, ks
    _restart()
    plan.destroy()


def test_two_variants_interleaved_in_one_stream(sphere4):
    """Single and double layer blocks in one worker pool: batches of both
    variants alternate; each block's factors equal those of launched batches."""
    plans = [_plan(sphere4, bem.LAPLACE_SLP), _plan(sphere4, bem.LAPLACE_DLP)]
    rng = inputs.rng(inputs.SEED_ARRIVALS)
    pidx, blocks = [], []
    for p, pl in enumerate(plans):
        sel = rng.choice(pl.info()["blocks"], size=200, replace=False)
        pidx += [p] * sel.size
        blocks += list(sel)
    order = rng.permutation(len(blocks))
    pidx, blocks = np.array(pidx)[order], np.array(blocks)[order]
    arr = np.cumsum(rng.exponential(2e-5, size=blocks.size))
    _restart(BEM_SERVER_PERSIST=0)
    bem.aca_plans_run(plans, pidx, blocks, arr, bem.FP32, n_workers=4, blocks_per_worker=8)
    ref = {(int(p), int(b)): plans[p].factors(b) for p, b in zip(pidx, blocks)}
    _restart(BEM_SERVER_PERSIST=1, BEM_SERVER_PERSIST_IDLE_US=200)
    bem.server_kernel_stats(reset=True)
    st = bem.aca_plans_run(plans, pidx, blocks, arr, bem.FP32, n_workers=4, blocks_per_worker=8)
    ks = bem.server_kernel_stats(reset=True)
    assert st["blocks"] == blocks.size
    for p, b in zip(pidx, blocks):
        U, V = plans[p].factors(b)
        U2, V2 = ref[(int(p), int(b))]
        assert np.array_equal(U, U2) and np.array_equal(V, V2), (p, b)
    assert _persistent_records(ks)
    _restart()
    for pl in plans:
        pl.destroy()
