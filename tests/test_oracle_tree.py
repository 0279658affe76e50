"""Pins of the cluster/block tree oracle (Section 2.1 partition).

Exact, index-level checks: the leaves partition the dofs, the blocks tile the
index square exactly once, admissible blocks satisfy the admissibility
condition and contain no vertex-sharing triangle pair.
"""
import numpy as np
import pytest

import oracle.tree as T
from paper_1711_01897_amd import inputs


@pytest.mark.parametrize("space", [0, 1])
def test_cluster_tree_partitions_dofs(space):
    xyz, tri = inputs.icosphere(3)
    pts, slo, shi = T.dof_geometry(xyz, tri, space)
    nodes = T.build_cluster_tree(pts, slo, shi, 32)
    n = pts.shape[0]
    leaves = [c for c in nodes if not c.children]
    allidx = np.concatenate([c.idx for c in leaves])
    assert np.array_equal(np.sort(allidx), np.arange(n))
    for c in nodes:
        if c.children:
            l, r = c.children
            assert np.array_equal(np.sort(np.concatenate([l.idx, r.idx])), np.sort(c.idx))
            assert l.idx.size > 0 and r.idx.size > 0
        else:
            assert c.idx.size <= 32
        assert np.all(pts[c.idx] >= c.lo) and np.all(pts[c.idx] <= c.hi)


@pytest.mark.parametrize("space,leaf,max_block", [(0, 32, 0), (1, 32, 0), (1, 8, 48), (0, 8, 40), (2, 24, 0)])
def test_block_tree_tiles_square_and_admissible_blocks_are_regular(space, leaf, max_block):
    xyz, tri = inputs.icosphere(3 if space != 2 else 2)
    nodes, leaves = T.partition(xyz, tri, space, leaf, 1.0, max_block)
    n = {0: tri.shape[0], 1: xyz.shape[0], 2: 3 * tri.shape[0]}[space]
    cover = np.zeros((n, n), dtype=np.int32)
    # triangles supporting each dof
    if space == 0:
        support = [np.array([t]) for t in range(n)]
    elif space == 2:
        support = [np.array([d // 3]) for d in range(n)]
    else:
        support = [np.flatnonzero((tri == v).any(1)) for v in range(n)]
    for a, b, ok in leaves:
        ra, cb = nodes[a].idx, nodes[b].idx
        cover[np.ix_(ra, cb)] += 1
        if ok:
            d = T.box_dist(nodes[a].slo, nodes[a].shi, nodes[b].slo, nodes[b].shi)
            assert d > 0
            assert min(T.box_diam(nodes[a].slo, nodes[a].shi), T.box_diam(nodes[b].slo, nodes[b].shi)) <= d
            va = np.unique(tri[np.concatenate([support[i] for i in ra])])
            vb = np.unique(tri[np.concatenate([support[j] for j in cb])])
            assert np.intersect1d(va, vb).size == 0
            if max_block:
                assert max(ra.size, cb.size) <= max_block
        else:
            assert not nodes[a].children or not nodes[b].children
    assert (cover == 1).all()


def test_icosphere_level6_p1_partition_counts():
    """Leaf 100, eta 1 on the 40,962-vertex icosphere (the H-matrix workload
    of the benchmark): block counts and sizes as measured independently."""
    xyz, tri = inputs.icosphere(6)
    nodes, leaves = T.partition(xyz, tri, 1, 100, 1.0)
    adm = [(a, b) for a, b, ok in leaves if ok]
    den = [(a, b) for a, b, ok in leaves if not ok]
    assert len(adm) == 24256 and len(den) == 17178
    assert sum(nodes[a].idx.size + nodes[b].idx.size for a, b in adm) == 8839546
    assert sum(nodes[a].idx.size * nodes[b].idx.size for a, b in den) == 112017666


def test_max_block_only_splits_oversized_admissible_blocks():
    """With a largest block dimension, every admissible block of the
    unbounded partition that fits is kept, every one that does not is
    replaced by blocks tiling the same index rectangle."""
    xyz, tri = inputs.icosphere(4)
    nodes, free = T.partition(xyz, tri, 1, 16, 1.0)
    _, capped = T.partition(xyz, tri, 1, 16, 1.0, 96)
    big = [(a, b) for a, b, ok in free if ok and max(nodes[a].idx.size, nodes[b].idx.size) > 96]
    assert big, "the level-4 icosphere has admissible blocks above 96 dofs"
    small = {(a, b) for a, b, ok in free if ok and (a, b) not in set(big)}
    kept = {(a, b) for a, b, ok in capped if ok}
    assert small <= kept
    n = xyz.shape[0]
    for a, b in big:
        cover = np.zeros((n, n), dtype=np.int32)
        cover[np.ix_(nodes[a].idx, nodes[b].idx)] = -1
        for c, d, ok in capped:
            sub = np.ix_(nodes[c].idx, nodes[d].idx)
            if (cover[sub] != 0).any():
                cover[sub] += 1
        assert (cover[np.ix_(nodes[a].idx, nodes[b].idx)] == 0).all()
