"""Cluster tree and block tree, FP64 (TEST INFRASTRUCTURE ONLY).

Section 2.1 partitions the matrix by a geometric tree whose leaves are either
admissible (compressed by ACA) or dense.  The paper does not fix the rules;
this oracle takes them as follows, step by step:

  cluster tree
    * dof points: triangle centroids (P0, and all three dofs of a triangle
      for the discontinuous P1 space, dof 3 t + a) or vertices (P1);
    * each dof carries a support box: the bounding box of the vertices of the
      triangles on which its basis function lives;
    * a cluster with more than leaf_size dofs is split at the midpoint of the
      longest side of its points' bounding box (lowest axis on ties): points
      with coordinate < midpoint go left, the rest right, both keeping their
      order; if one side is empty the split is at the median instead (sort
      by coordinate, then dof index; the first floor(n/2) go left);
  block tree, from (root, root)
    * admissible iff dist > 0 and min(diam(tau), diam(sigma)) <= eta dist,
      diameters and distance taken on the clusters' support boxes, and, when
      a largest block dimension max_block > 0 is given, both clusters hold at
      most max_block dofs (larger pairs split further, so no ACA row or
      column is longer than max_block);
    * otherwise a dense leaf if either cluster is a leaf, else the four child
      pairs (t1,s1), (t1,s2), (t2,s1), (t2,s2) in that order.
Support boxes make every admissible block free of vertex-sharing pairs.
"""
from __future__ import annotations

import math

import numpy as np


class Cluster:
    __slots__ = ("idx", "lo", "hi", "slo", "shi", "children", "id")

    def __init__(self, idx, lo, hi, slo, shi):
        self.idx = idx
        self.lo = lo
        self.hi = hi
        self.slo = slo
        self.shi = shi
        self.children = []
        self.id = -1


def dof_geometry(xyz, tri, space: int):
    """(points, support_lo, support_hi) per dof; space 0 = P0, 1 = P1,
    2 = discontinuous P1."""
    xyz = np.asarray(xyz, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    tlo = np.minimum(np.minimum(a, b), c)
    thi = np.maximum(np.maximum(a, b), c)
    if space == 0:
        pts = (a + b + c) / 3.0
        return pts, tlo, thi
    if space == 2:
        pts = (a + b + c) / 3.0
        return np.repeat(pts, 3, axis=0), np.repeat(tlo, 3, axis=0), np.repeat(thi, 3, axis=0)
    nv = xyz.shape[0]
    slo = np.full((nv, 3), np.inf)
    shi = np.full((nv, 3), -np.inf)
    for k in range(3):
        np.minimum.at(slo, tri[:, k], tlo)
        np.maximum.at(shi, tri[:, k], thi)
    return xyz.copy(), slo, shi


def build_cluster_tree(points, slo, shi, leaf_size: int):
    """Returns the list of clusters in depth-first pre-order (root first)."""
    points = np.asarray(points, dtype=np.float64)
    nodes: list[Cluster] = []

    def make(idx):
        p = points[idx]
        cl = Cluster(idx, p.min(axis=0), p.max(axis=0), slo[idx].min(axis=0), shi[idx].max(axis=0))
        cl.id = len(nodes)
        nodes.append(cl)
        if idx.size <= leaf_size:
            return cl
        ext = cl.hi - cl.lo
        axis = int(np.argmax(ext))
        mid = (cl.lo[axis] + cl.hi[axis]) / 2.0
        coord = p[:, axis]
        mask = coord < mid
        left, right = idx[mask], idx[~mask]
        if left.size == 0 or right.size == 0:
            order = np.lexsort((idx, coord))
            half = idx.size // 2
            left = idx[order[:half]]
            right = idx[order[half:]]
        cl.children = [make(left), make(right)]
        return cl

    make(np.arange(points.shape[0], dtype=np.int64))
    return nodes


def box_diam(lo, hi) -> float:
    dx, dy, dz = float(hi[0] - lo[0]), float(hi[1] - lo[1]), float(hi[2] - lo[2])
    return math.sqrt(dx * dx + dy * dy + dz * dz)


def box_dist(lo1, hi1, lo2, hi2) -> float:
    g = []
    for k in range(3):
        gk = max(0.0, float(lo1[k] - hi2[k]), float(lo2[k] - hi1[k]))
        g.append(gk)
    return math.sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2])


def admissible(t: Cluster, s: Cluster, eta: float, max_block: int = 0) -> bool:
    if max_block > 0 and max(t.idx.size, s.idx.size) > max_block:
        return False
    d = box_dist(t.slo, t.shi, s.slo, s.shi)
    if not d > 0.0:
        return False
    return min(box_diam(t.slo, t.shi), box_diam(s.slo, s.shi)) <= eta * d


def build_block_tree(nodes, eta: float, max_block: int = 0):
    """Leaves as (tau_id, sigma_id, is_admissible) in depth-first order."""
    leaves = []
    stack = [(nodes[0], nodes[0])]
    while stack:
        t, s = stack.pop()
        if admissible(t, s, eta, max_block):
            leaves.append((t.id, s.id, True))
        elif not t.children or not s.children:
            leaves.append((t.id, s.id, False))
        else:
            t1, t2 = t.children
            s1, s2 = s.children
            # push in reverse so that (t1,s1) is handled first
            stack.extend([(t2, s2), (t2, s1), (t1, s2), (t1, s1)])
    return leaves


def partition(xyz, tri, space: int, leaf_size: int = 100, eta: float = 1.0, max_block: int = 0):
    pts, slo, shi = dof_geometry(xyz, tri, space)
    nodes = build_cluster_tree(pts, slo, shi, leaf_size)
    return nodes, build_block_tree(nodes, eta, max_block)
