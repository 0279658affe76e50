"""FP64 CPU oracle of the weak-form entry path (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the product
library ``paper_1711_01897_amd`` and imports nothing from it.

Contents
  * ``OracleMesh`` (C, ``bem_oracle.c``): geometry, Gauss rules, kernels and
    P0/P1 Galerkin entries of the Laplace/Helmholtz single, double and
    adjoint double layer, and P1 entries of the hypersingular operator, over
    regular triangle pairs (Section 2, Eqs. slp, dlp, adlp, hypsHelmholtz;
    Section 3.2); also entries on the discontinuous P1 space (DP1, dof
    3 t + a: the barycentric function of local vertex a on triangle t), the
    space whose single layer gives the hypersingular operator by sparse
    transformations (Eq. hyp_via_slp), and those transformations
    (``hyp_via_slp_factors``).
  * near-field fixtures (C, ``nearfield.c``) for vertex-sharing pairs, the
    reference of the device's singular scheme and of the closed-form sphere
    checks: P0 Laplace (closed-form inner potential and solid angle), P0
    Helmholtz (the kernel expanded around r = 0, singular terms in closed
    form, the remainder on a subdivided rule), P1 Laplace and Helmholtz local
    matrices (closed-form potentials of a linear density, the Helmholtz
    remainder on a subdivided rule) and the Laplace hypersingular operator's.
  * ``oracle.aca``: adaptive cross approximation, Algorithm "ACA" of
    Section 2.1 with the row pivot of Bebendorf's partial pivoting.
  * ``oracle.tree``: geometric cluster tree and block tree (Section 2.1).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

LAPLACE_SLP, LAPLACE_DLP, HELMHOLTZ_SLP, HELMHOLTZ_DLP = 0, 1, 2, 3
LAPLACE_ADLP, HELMHOLTZ_ADLP = 4, 5
LAPLACE_HYPS, HELMHOLTZ_HYPS = 6, 7
P0, P1, DP1 = 0, 1, 2
NEAR_ERROR, NEAR_SKIP = 0, 1
OPS = {"laplace_slp": 0, "laplace_dlp": 1, "helmholtz_slp": 2, "helmholtz_dlp": 3, "laplace_adlp": 4,
       "helmholtz_adlp": 5, "laplace_hyps": 6, "helmholtz_hyps": 7}

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def _lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(HERE, "liborc.so")
    if not os.path.exists(path):
        from . import build as _b
        _b.build()
    lib = ctypes.CDLL(path)
    lib.orc_rule.argtypes = [ctypes.c_int, _dp, _dp, _dp]
    lib.orc_rule.restype = ctypes.c_int
    lib.orc_kernel.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp]
    lib.orc_kernel.restype = None
    lib.orc_mesh_new.argtypes = [_dp, ctypes.c_int64, _ip, ctypes.c_int64, ctypes.c_int]
    lib.orc_mesh_new.restype = ctypes.c_void_p
    lib.orc_mesh_free.argtypes = [ctypes.c_void_p]
    lib.orc_mesh_free.restype = None
    lib.orc_mesh_geometry.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
    lib.orc_mesh_geometry.restype = None
    lib.orc_adjacent.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64]
    lib.orc_adjacent.restype = ctypes.c_int
    lib.orc_entries.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                _ip, ctypes.c_int64, _ip, ctypes.c_int64, ctypes.c_int, _dp, ctypes.c_int]
    lib.orc_entries.restype = ctypes.c_int
    lib.orc_max_threads.argtypes = []
    lib.orc_max_threads.restype = ctypes.c_int
    lib.orc_tri_potential.argtypes = [_dp, _dp, _dp, _dp]
    lib.orc_tri_potential.restype = ctypes.c_double
    lib.orc_tri_solid_angle.argtypes = [_dp, _dp, _dp, _dp]
    lib.orc_tri_solid_angle.restype = ctypes.c_double
    lib.orc_subdivided_rule.argtypes = [ctypes.c_int, _dp, _dp, _dp]
    lib.orc_subdivided_rule.restype = ctypes.c_int
    lib.orc_nearfield_entry.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
    lib.orc_nearfield_entry.restype = ctypes.c_double
    lib.orc_tri_moment_r.argtypes = [_dp, _dp, _dp, _dp]
    lib.orc_tri_moment_r.restype = ctypes.c_double
    lib.orc_nearfield_entries_c.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64,
                                            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                            ctypes.c_int, ctypes.c_int, _dp]
    lib.orc_nearfield_entries_c.restype = ctypes.c_int
    lib.orc_tri_vector_moments.argtypes = [_dp, _dp, _dp, _dp, _dp, _dp]
    lib.orc_tri_vector_moments.restype = None
    lib.orc_nearfield_p1_local.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64,
                                           ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                           ctypes.c_int, _dp]
    lib.orc_nearfield_p1_local.restype = ctypes.c_int
    lib.orc_tri_vector_moment_r.argtypes = [_dp, _dp, _dp, _dp, _dp]
    lib.orc_tri_vector_moment_r.restype = None
    lib.orc_nearfield_p1_local_c.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int64,
                                             ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                             ctypes.c_int, ctypes.c_int, _dp]
    lib.orc_nearfield_p1_local_c.restype = ctypes.c_int
    lib.orc_p0_matrix_with_nearfield.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_int, _dp]
    lib.orc_p0_matrix_with_nearfield.restype = ctypes.c_int
    _LIB = lib
    return lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _i(a):
    return a.ctypes.data_as(_ip)


def _vec(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64))


def rule(npts: int):
    """(xi, eta, w) of the symmetric Gauss rule on the reference triangle."""
    xi, eta, w = np.zeros(6), np.zeros(6), np.zeros(6)
    n = _lib().orc_rule(npts, _d(xi), _d(eta), _d(w))
    if n < 0:
        raise ValueError("npts must be 4 or 6")
    return xi[:n].copy(), eta[:n].copy(), w[:n].copy()


def subdivided_rule(level: int):
    n = 6 * 4 ** level
    xi, eta, w = np.zeros(n), np.zeros(n), np.zeros(n)
    _lib().orc_subdivided_rule(level, _d(xi), _d(eta), _d(w))
    return xi, eta, w


def tri_moment_r(v0, v1, v2, x) -> float:
    """int_T |x - y| dy over the flat triangle (v0, v1, v2), closed form."""
    return _lib().orc_tri_moment_r(_d(_vec(v0)), _d(_vec(v1)), _d(_vec(v2)), _d(_vec(x)))


def tri_vector_moments(v0, v1, v2, x):
    """(int_T (y - rho)/R dy, int_T (y - rho)/R^3 dy), rho the projection of x
    on the triangle's plane, closed form."""
    V1, V3 = np.zeros(3), np.zeros(3)
    _lib().orc_tri_vector_moments(_d(_vec(v0)), _d(_vec(v1)), _d(_vec(v2)), _d(_vec(x)), _d(V1), _d(V3))
    return V1, V3


def tri_vector_moment_r(v0, v1, v2, x):
    """int_T (y - rho) |x - y| dy, rho the projection of x on the triangle's
    plane, closed form."""
    W1 = np.zeros(3)
    _lib().orc_tri_vector_moment_r(_d(_vec(v0)), _d(_vec(v1)), _d(_vec(v2)), _d(_vec(x)), _d(W1))
    return W1


def kernel(op: int, k: float, x, y, ny) -> complex:
    """g(x,y) (single layer) or dg/dn_y (double layer)."""
    out = np.zeros(2)
    _lib().orc_kernel(op, float(k), _d(_vec(x)), _d(_vec(y)), _d(_vec(ny)), _d(out))
    return complex(out[0], out[1])


def tri_potential(v0, v1, v2, x) -> float:
    return _lib().orc_tri_potential(_d(_vec(v0)), _d(_vec(v1)), _d(_vec(v2)), _d(_vec(x)))


def tri_solid_angle(v0, v1, v2, x) -> float:
    return _lib().orc_tri_solid_angle(_d(_vec(v0)), _d(_vec(v1)), _d(_vec(v2)), _d(_vec(x)))


def is_complex(op: int) -> bool:
    return op in (HELMHOLTZ_SLP, HELMHOLTZ_DLP, HELMHOLTZ_ADLP, HELMHOLTZ_HYPS)


class NearFieldError(RuntimeError):
    pass


class OracleMesh:
    """Geometry and vertex stars of one triangle mesh, FP64."""

    def __init__(self, xyz, tri, quad_points: int = 6):
        self.xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64))
        self.tri = np.ascontiguousarray(np.asarray(tri, dtype=np.int32))
        self.nv = self.xyz.shape[0]
        self.nt = self.tri.shape[0]
        self.q = quad_points
        lib = _lib()
        self._h = lib.orc_mesh_new(_d(self.xyz), self.nv, _i(self.tri), self.nt, quad_points)
        if not self._h:
            raise ValueError("invalid mesh or quadrature size")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _LIB is not None:
            _LIB.orc_mesh_free(h)
            self._h = None

    def geometry(self):
        J = np.zeros(self.nt)
        n = np.zeros((self.nt, 3))
        qp = np.zeros((self.nt, self.q, 3))
        _lib().orc_mesh_geometry(self._h, _d(J), _d(n), _d(qp))
        return J, n, qp

    def adjacent(self, a: int, b: int) -> bool:
        return bool(_lib().orc_adjacent(self._h, a, b))

    def entries(self, op: int, space: int, k: float, rows, cols, near: int = NEAR_SKIP,
                nthreads: int = 0) -> np.ndarray:
        """Sub-block A[rows, cols] (float64, or complex128 for Helmholtz)."""
        rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int32).ravel())
        cols = np.ascontiguousarray(np.asarray(cols, dtype=np.int32).ravel())
        nr, nc = rows.size, cols.size
        cplx = is_complex(op)
        out = np.zeros(nr * nc * (2 if cplx else 1))
        if nr and nc:
            st = _lib().orc_entries(self._h, op, space, float(k), _i(rows), nr, _i(cols), nc, near,
                                    _d(out), int(nthreads))
            if st == -4:
                raise NearFieldError("request touches an adjacent or identical triangle pair")
            if st != 0:
                raise ValueError(f"oracle entries failed ({st})")
        if cplx:
            return out.view(np.complex128).reshape(nr, nc)
        return out.reshape(nr, nc)

    def nearfield_entry(self, op: int, i: int, j: int, level: int = 3) -> float:
        return _lib().orc_nearfield_entry(self._h, op, i, j, level)

    def nearfield_entries(self, op: int, k: float, rows, cols, level: int = 3, inner_level: int = 3) -> np.ndarray:
        """Semi-analytic P0 entries (rows[t], cols[t]) of any of the four
        operators, complex128 (imaginary part 0 for Laplace)."""
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        c = np.ascontiguousarray(np.asarray(cols, dtype=np.int64))
        if r.shape != c.shape or r.ndim != 1:
            raise ValueError("rows and cols: equal 1D sequences")
        out = np.zeros(2 * r.size)
        p64 = ctypes.POINTER(ctypes.c_int64)
        st = _lib().orc_nearfield_entries_c(self._h, op, float(k), r.size, r.ctypes.data_as(p64),
                                            c.ctypes.data_as(p64), level, inner_level, _d(out))
        if st != 0:
            raise ValueError("operator 0..3 and levels >= 0")
        return out.view(np.complex128)

    def nearfield_p1_local(self, op: int, rows, cols, level: int = 3) -> np.ndarray:
        """3 x 3 local P1 matrices (test vertex order x trial vertex order of
        the mesh's triangles) of the pairs (rows[t], cols[t]), Laplace single
        or double layer or hypersingular operator, semi-analytic; shape
        (n, 3, 3)."""
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        c = np.ascontiguousarray(np.asarray(cols, dtype=np.int64))
        if r.shape != c.shape or r.ndim != 1:
            raise ValueError("rows and cols: equal 1D sequences")
        out = np.zeros(9 * r.size)
        p64 = ctypes.POINTER(ctypes.c_int64)
        st = _lib().orc_nearfield_p1_local(self._h, op, r.size, r.ctypes.data_as(p64), c.ctypes.data_as(p64),
                                           level, _d(out))
        if st != 0:
            raise ValueError("Laplace single, double layer or hypersingular operator and level >= 0")
        return out.reshape(r.size, 3, 3)

    def nearfield_p1_local_c(self, op: int, k: float, rows, cols, level: int = 3, inner_level: int = 3) -> np.ndarray:
        """Complex 3 x 3 local P1 matrices of the Helmholtz single or double
        layer for the pairs (rows[t], cols[t]); shape (n, 3, 3)."""
        r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
        c = np.ascontiguousarray(np.asarray(cols, dtype=np.int64))
        if r.shape != c.shape or r.ndim != 1:
            raise ValueError("rows and cols: equal 1D sequences")
        out = np.zeros(18 * r.size)
        p64 = ctypes.POINTER(ctypes.c_int64)
        st = _lib().orc_nearfield_p1_local_c(self._h, op, float(k), r.size, r.ctypes.data_as(p64),
                                             c.ctypes.data_as(p64), level, inner_level, _d(out))
        if st != 0:
            raise ValueError("Helmholtz single, double layer or hypersingular operator and levels >= 0")
        return out.view(np.complex128).reshape(r.size, 3, 3)

    def p0_matrix_with_nearfield(self, op: int, near_dist: float, level: int = 3) -> np.ndarray:
        out = np.zeros((self.nt, self.nt))
        st = _lib().orc_p0_matrix_with_nearfield(self._h, op, float(near_dist), level, _d(out))
        if st != 0:
            raise ValueError("only Laplace single/double layer")
        return out


def hyp_via_slp_factors(xyz, tri):
    """The sparse matrices of Eq. hyp_via_slp as dense numpy arrays (small
    meshes only): Q[j] (3 nt x nv), the j-th component of the surface curl
    of each continuous hat function, constant on a triangle and written on
    the discontinuous P1 space as that constant on all three local
    functions; P[j] (3 nt x nv), the hat function of a vertex on each of its
    triangles times the j-th component of the triangle's unit normal.  Then
    D = sum_j Q_j^T S Q_j - k^2 sum_j P_j^T S P_j with S the single layer on
    the discontinuous space.  The curl of the hat function of local vertex a
    is n x grad lambda_a with grad lambda_a = n x E_a / J, E_a = v_{a+2} -
    v_{a+1} the edge opposite a and J = |(v1 - v0) x (v2 - v0)|."""
    xyz = np.asarray(xyz, dtype=np.float64)
    tri = np.asarray(tri, dtype=np.int64)
    nt, nv = tri.shape[0], xyz.shape[0]
    Q = np.zeros((3, 3 * nt, nv))
    P = np.zeros((3, 3 * nt, nv))
    for t in range(nt):
        v = xyz[tri[t]]
        N = np.cross(v[1] - v[0], v[2] - v[0])
        J = np.linalg.norm(N)
        n = N / J
        for a in range(3):
            E = v[(a + 2) % 3] - v[(a + 1) % 3]
            curl = np.cross(n, np.cross(n, E)) / J
            for j in range(3):
                Q[j, 3 * t:3 * t + 3, tri[t, a]] += curl[j]
                P[j, 3 * t + a, tri[t, a]] = n[j]
    return Q, P


def max_threads() -> int:
    return int(_lib().orc_max_threads())
