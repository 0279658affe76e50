"""Seeded synthetic inputs: surface meshes and request streams.

This module holds no boundary-element arithmetic (no quadrature, no kernels,
no integrals).  It only builds closed, outward-oriented, welded triangle
meshes of the shapes the method is benchmarked on and draws index sets, so
that the FP64 oracle and the HIP path can be fed identical data.

Shapes:
  * icosphere(level): recursive 4-split of the icosahedron with midpoints
    projected to the unit sphere (the paper benchmarks on unit spheres,
    Section 5 "Benchmarks", continuous P1 spaces).
  * spheroid(a, b, target_nt): near-uniform ring mesh of the prolate
    spheroid x^2/a^2 + (y^2+z^2)/b^2 = 1 (stand-in for the elongated
    submarine hull of Section 6 at 6-10 elements per wavelength).
  * capped_cylinder(R, L, target_nt, jitter, seed): ring mesh of a cylinder
    with flat disk caps welded to the side, vertices jittered by a seeded
    uniform offset of +-jitter*h per coordinate.

Seeds (numpy PCG64): 0 mesh jitter, 1 arrival times, 2 block order and
request sizes, 3 oracle sampling.
"""
from __future__ import annotations

import math

import numpy as np

SEED_JITTER = 0
SEED_ARRIVALS = 1
SEED_REQUESTS = 2
SEED_SAMPLING = 3


# ----------------------------------------------------------------------------
# icosphere
# ----------------------------------------------------------------------------
def _icosahedron():
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    v /= np.linalg.norm(v, axis=1)[:, None]
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    return v, f


def icosphere(level: int):
    """Unit icosphere after `level` 4-splits: 20*4^level triangles,
    10*4^level + 2 vertices, counter-clockwise seen from outside."""
    v, f = _icosahedron()
    verts = [row for row in v]
    for _ in range(level):
        cache = {}
        nf = np.empty((f.shape[0] * 4, 3), dtype=np.int64)

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            idx = cache.get(key)
            if idx is None:
                m = verts[a] + verts[b]
                m = m / np.linalg.norm(m)
                idx = len(verts)
                verts.append(m)
                cache[key] = idx
            return idx

        for k, (a, b, c) in enumerate(f):
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf[4 * k + 0] = (a, ab, ca)
            nf[4 * k + 1] = (b, bc, ab)
            nf[4 * k + 2] = (c, ca, bc)
            nf[4 * k + 3] = (ab, bc, ca)
        f = nf
    xyz = np.ascontiguousarray(np.array(verts, dtype=np.float64))
    return xyz, np.ascontiguousarray(f.astype(np.int32))


# ----------------------------------------------------------------------------
# ring meshes of surfaces of revolution about the x axis
# ----------------------------------------------------------------------------
def _ring_strip(a_idx, a_phi, b_idx, b_phi):
    """Triangulate the band between two closed rings by a merge walk on the
    unwrapped angle.  Rings are ordered by increasing angle; every triangle
    is counter-clockwise in the (phi, s) chart with ring a at the lower s."""
    na, nb = len(a_idx), len(b_idx)
    tris = []
    i = j = 0
    two_pi = 2.0 * math.pi
    # unwrapped angles with one extra wrap-around entry
    pa = np.concatenate([a_phi, [a_phi[0] + two_pi]])
    pb = np.concatenate([b_phi, [b_phi[0] + two_pi]])
    while i < na or j < nb:
        if j >= nb or (i < na and pa[i + 1] <= pb[j + 1]):
            tris.append((a_idx[i % na], a_idx[(i + 1) % na], b_idx[j % nb]))
            i += 1
        else:
            tris.append((a_idx[i % na], b_idx[(j + 1) % nb], b_idx[j % nb]))
            j += 1
    return tris


def _revolve(profile_x, profile_r, h, pole_start, pole_end, stagger=True):
    """Build a ring mesh from profile samples (x_k, r_k), k = 0..K.

    profile_r[k] == 0 only at poles.  Ring k gets max(3, round(2 pi r_k / h))
    points; consecutive rings are staggered by half a step."""
    verts = []
    rings = []  # list of (indices, angles) or ('pole', index)
    for k, (x, r) in enumerate(zip(profile_x, profile_r)):
        if r <= 0.0:
            idx = len(verts)
            verts.append((x, 0.0, 0.0))
            rings.append(("pole", idx))
            continue
        n = max(3, int(round(2.0 * math.pi * r / h)))
        off = (0.5 * (k % 2) if stagger else 0.0) * 2.0 * math.pi / n
        phi = off + 2.0 * math.pi * np.arange(n) / n
        start = len(verts)
        for p in phi:
            verts.append((x, r * math.cos(p), r * math.sin(p)))
        rings.append((np.arange(start, start + n), phi))
    tris = []
    for k in range(len(rings) - 1):
        A, B = rings[k], rings[k + 1]
        if isinstance(A[0], str):
            P = A[1]
            idx, _ = B
            n = len(idx)
            for j in range(n):
                tris.append((P, idx[(j + 1) % n], idx[j]))
        elif isinstance(B[0], str):
            P = B[1]
            idx, _ = A
            n = len(idx)
            for i in range(n):
                tris.append((idx[i], idx[(i + 1) % n], P))
        else:
            tris.extend(_ring_strip(A[0], A[1], B[0], B[1]))
    xyz = np.array(verts, dtype=np.float64)
    tri = np.array(tris, dtype=np.int64)
    return _orient_outward(xyz, tri)


def _orient_outward(xyz, tri):
    a, b, c = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    vol = np.einsum("ij,ij->", a, np.cross(b, c)) / 6.0
    if vol < 0:
        tri = tri[:, [0, 2, 1]]
    return np.ascontiguousarray(xyz), np.ascontiguousarray(tri.astype(np.int32))


def _spheroid_profile(a, b, h):
    """Profile (x, r) of x^2/a^2 + r^2/b^2 = 1 sampled at uniform arc length
    with spacing h*sqrt(3)/2 (height of an equilateral triangle of edge h)."""
    th = np.linspace(0.0, math.pi, 200001)
    x = a * np.cos(th)
    r = b * np.sin(th)
    ds = np.hypot(np.diff(x), np.diff(r))
    s = np.concatenate([[0.0], np.cumsum(ds)])
    total = s[-1]
    nr = max(2, int(round(total / (h * math.sqrt(3.0) / 2.0))))
    sk = np.linspace(0.0, total, nr + 1)
    thk = np.interp(sk, s, th)
    xk = a * np.cos(thk)
    rk = b * np.sin(thk)
    rk[0] = 0.0
    rk[-1] = 0.0
    return xk, rk


def _fit_h(build, target_nt, h0):
    """Scale h so that the triangle count lands within 1% of target_nt."""
    h = h0
    best = None
    for _ in range(40):
        xyz, tri = build(h)
        nt = tri.shape[0]
        if best is None or abs(nt - target_nt) < abs(best[1].shape[0] - target_nt):
            best = (xyz, tri, h)
        if abs(nt - target_nt) <= 0.01 * target_nt:
            break
        h *= math.sqrt(nt / target_nt)
    return best


def spheroid(a: float = 10.0, b: float = 1.0, target_nt: int = 262144):
    """Near-uniform ring mesh of the prolate spheroid with semi-axes (a,b,b)
    along (x,y,z); the triangle count is within 1% of target_nt."""
    # area of a prolate spheroid
    e = math.sqrt(1.0 - (b * b) / (a * a))
    area = 2.0 * math.pi * b * b * (1.0 + a / (b * e) * math.asin(e))
    h0 = math.sqrt(4.0 * area / (math.sqrt(3.0) * target_nt))

    def build(h):
        xk, rk = _spheroid_profile(a, b, h)
        return _revolve(xk, rk, h, True, True)

    xyz, tri, _ = _fit_h(build, target_nt, h0)
    return xyz, tri


def capped_cylinder(R: float = 1.0, L: float = 16.0, target_nt: int = 1048576,
                    jitter: float = 0.01, seed: int = SEED_JITTER):
    """Cylinder of radius R along x in [0, L] with flat disk caps.

    Vertices are moved by U(-jitter*h, jitter*h) per coordinate (numpy
    PCG64, `seed`), h being the nominal edge length.  Returns (xyz, tri)."""
    area = 2.0 * math.pi * R * L + 2.0 * math.pi * R * R
    h0 = math.sqrt(4.0 * area / (math.sqrt(3.0) * target_nt))

    def build(h):
        dr = h * math.sqrt(3.0) / 2.0
        kc = max(1, int(round(R / dr)))
        ks = max(1, int(round(L / dr)))
        # bottom cap: r from 0 to R at x = 0; side: x from 0 to L; top cap
        xs, rs = [], []
        for k in range(kc + 1):
            xs.append(0.0)
            rs.append(R * k / kc)
        for k in range(1, ks + 1):
            xs.append(L * k / ks)
            rs.append(R)
        for k in range(kc - 1, -1, -1):
            xs.append(L)
            rs.append(R * k / kc)
        return _revolve(np.array(xs), np.array(rs), h, True, True)

    xyz, tri, h = _fit_h(build, target_nt, h0)
    if jitter > 0.0:
        rng = np.random.Generator(np.random.PCG64(seed))
        xyz = xyz + rng.uniform(-jitter * h, jitter * h, size=xyz.shape)
    return np.ascontiguousarray(xyz), tri


# ----------------------------------------------------------------------------
# mesh statistics used to pick wavenumbers and check the recipe
# ----------------------------------------------------------------------------
def edges(tri):
    e = np.concatenate([tri[:, [0, 1]], tri[:, [1, 2]], tri[:, [2, 0]]])
    e.sort(axis=1)
    return np.unique(e, axis=0)


def mean_edge_length(xyz, tri):
    e = edges(tri)
    return float(np.linalg.norm(xyz[e[:, 0]] - xyz[e[:, 1]], axis=1).mean())


def wavenumber(xyz, tri, elements_per_wavelength: float) -> float:
    """k such that one wavelength spans `elements_per_wavelength` mean edges."""
    h = mean_edge_length(xyz, tri)
    return 2.0 * math.pi / (elements_per_wavelength * h)


# ----------------------------------------------------------------------------
# request streams
# ----------------------------------------------------------------------------
def random_index_set(n: int, size: int, rng: np.random.Generator) -> np.ndarray:
    """`size` distinct indices out of range(n), in random order (int32)."""
    return rng.choice(n, size=size, replace=False).astype(np.int32)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))
