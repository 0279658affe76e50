"""Thin ctypes binding of libbem's C ABI (include/bem.h).

Every function marshals arguments and calls the C entry point of the same
name; all computation happens in the library (HIP kernels on the device,
ACA, trees and the request server on the host).  There is no fallback: if
libbem.so is missing the import of any entry point raises.  PyTorch is used
only to hand device buffers and HIP streams to ``eval_entries_async``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbem.so")

LAPLACE_SLP, LAPLACE_DLP, HELMHOLTZ_SLP, HELMHOLTZ_DLP = 0, 1, 2, 3
LAPLACE_ADLP, HELMHOLTZ_ADLP = 4, 5
LAPLACE_HYPS, HELMHOLTZ_HYPS = 6, 7
P0, P1, DP1 = 0, 1, 2
FP64, FP32 = 0, 1
NEAR_ERROR, NEAR_SKIP, NEAR_SINGULAR = 0, 1, 2

OK, E_ARG, E_OOM, E_DEVICE, E_NEARFIELD, E_BUSY, E_CANCELLED, E_TIMEOUT, E_INTERNAL = 0, -1, -2, -3, -4, -5, -6, -7, -8
_NAMES = {E_ARG: "BEM_E_ARG", E_OOM: "BEM_E_OOM", E_DEVICE: "BEM_E_DEVICE", E_NEARFIELD: "BEM_E_NEARFIELD",
          E_BUSY: "BEM_E_BUSY", E_CANCELLED: "BEM_E_CANCELLED", E_TIMEOUT: "BEM_E_TIMEOUT", E_INTERNAL: "BEM_E_INTERNAL"}

# every symbol declared in include/bem.h
EXPORTS = [
    "bem_last_error", "bem_mesh_create", "bem_mesh_destroy", "bem_mesh_info", "bem_eval_entries", "bem_submit",
    "bem_ticket_wait", "bem_ticket_times", "bem_ticket_free", "bem_eval_entries_async", "bem_server_config",
    "bem_server_stats", "bem_server_kernel_stats", "bem_aca_block", "bem_aca_callback", "bem_partition", "bem_hmat_assemble",
    "bem_hmat_matvec", "bem_hmat_stats_get", "bem_hmat_block_info", "bem_hmat_block_dense", "bem_hmat_destroy",
    "bem_aca_plan_create", "bem_aca_plan_info", "bem_aca_plan_block", "bem_aca_plan_run", "bem_aca_plan_factors",
    "bem_aca_plan_destroy", "bem_eval_dense", "bem_eval_entries_async_noalloc", "bem_aca_plans_run",
]


class BemError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


class NearFieldError(BemError):
    pass


_p = ctypes.c_void_p
_i32p = ctypes.POINTER(ctypes.c_int32)
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)


class MeshInfo(ctypes.Structure):
    _fields_ = [("nv", ctypes.c_int64), ("nt", ctypes.c_int64), ("quad_points", ctypes.c_int32),
                ("max_star", ctypes.c_int32), ("mean_jacobian", ctypes.c_double), ("mean_edge", ctypes.c_double),
                ("device_bytes", ctypes.c_size_t)]


class ServerStats(ctypes.Structure):
    _fields_ = [("requests", ctypes.c_int64), ("entries", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("kernel_evals", ctypes.c_int64), ("latency_p50", ctypes.c_double),
                ("latency_p99", ctypes.c_double), ("latency_max", ctypes.c_double),
                ("busy_seconds", ctypes.c_double), ("kernel_seconds", ctypes.c_double),
                ("kernel_launches", ctypes.c_int64),
                ("dispatch_seconds", ctypes.c_double), ("complete_seconds", ctypes.c_double),
                ("wait_seconds", ctypes.c_double), ("dispatch_hip_seconds", ctypes.c_double),
                ("mean_queue_seconds", ctypes.c_double), ("mean_stage_seconds", ctypes.c_double),
                ("mean_device_seconds", ctypes.c_double), ("mean_complete_seconds", ctypes.c_double)]


class KernelStats(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("space", ctypes.c_int32), ("prec", ctypes.c_int32),
                ("quad_points", ctypes.c_int32), ("persistent", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("launches", ctypes.c_int64), ("workgroups", ctypes.c_int64), ("entries", ctypes.c_int64), ("pair_evals", ctypes.c_int64),
                ("triangle_loads", ctypes.c_int64), ("seconds", ctypes.c_double),
                ("seconds_events", ctypes.c_double), ("blocks", ctypes.c_int64)]


class AcaParams(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_rank", ctypes.c_int32), ("zero_abs", ctypes.c_double)]


class HmatParams(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_int32), ("eta", ctypes.c_double), ("aca_tol", ctypes.c_double),
                ("max_rank", ctypes.c_int32), ("n_workers", ctypes.c_int32), ("blocks_per_worker", ctypes.c_int32),
                ("prec", ctypes.c_int), ("dense_mode", ctypes.c_int32), ("max_block", ctypes.c_int32),
                ("hyps_via_slp", ctypes.c_int32)]


class DenseStats(ctypes.Structure):
    _fields_ = [("pairs", ctypes.c_int64), ("panels", ctypes.c_int64), ("seconds", ctypes.c_double),
                ("first_pairs", ctypes.c_int64), ("first_local_seconds", ctypes.c_double),
                ("first_gather_seconds", ctypes.c_double)]


class AcaRunStats(ctypes.Structure):
    _fields_ = [("blocks", ctypes.c_int64), ("entries", ctypes.c_int64), ("requests", ctypes.c_int64),
                ("rank_sum", ctypes.c_int64), ("rank_max", ctypes.c_int32), ("seconds", ctypes.c_double),
                ("mean_start_delay", ctypes.c_double), ("mean_block_seconds", ctypes.c_double)]


class HmatStats(ctypes.Structure):
    _fields_ = [("ndof", ctypes.c_int64), ("admissible_blocks", ctypes.c_int64), ("dense_blocks", ctypes.c_int64),
                ("aca_entries", ctypes.c_int64), ("dense_entries", ctypes.c_int64), ("aca_requests", ctypes.c_int64),
                ("rank_sum", ctypes.c_int64), ("rank_max", ctypes.c_int32), ("bytes", ctypes.c_size_t),
                ("seconds", ctypes.c_double), ("partition_seconds", ctypes.c_double),
                ("setup_seconds", ctypes.c_double), ("aca_seconds", ctypes.c_double),
                ("worker_busy_seconds", ctypes.c_double)]


ROW_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int64, _dp)
COL_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int64, _dp)

_LIB = None


def lib():
    """Load libbem.so once.  On a machine with a GPU torch is imported first
    so that the library binds to the HIP runtime torch already loaded."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing; build it with paper_1711_01897_amd/build_lib.py")
    try:
        import torch  # noqa: F401  (shares its HIP runtime with the library)
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    L.bem_last_error.restype = ctypes.c_char_p
    L.bem_mesh_create.argtypes = [_dp, ctypes.c_int64, _i32p, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(_p)]
    L.bem_mesh_destroy.argtypes = [_p]
    L.bem_mesh_info.argtypes = [_p, ctypes.POINTER(MeshInfo)]
    entry_args = [_p, ctypes.c_int, ctypes.c_int, ctypes.c_double, _i32p, ctypes.c_int64, _i32p, ctypes.c_int64,
                  ctypes.c_int, ctypes.c_int]
    L.bem_eval_entries.argtypes = entry_args + [_p]
    L.bem_submit.argtypes = entry_args + [_p, ctypes.POINTER(_p)]
    L.bem_ticket_wait.argtypes = [_p, ctypes.c_double]
    L.bem_ticket_times.argtypes = [_p, _dp, _dp]
    L.bem_ticket_free.argtypes = [_p]
    L.bem_eval_entries_async.argtypes = entry_args + [_p, _p]
    L.bem_eval_entries_async_noalloc.argtypes = entry_args + [_p, _p]
    L.bem_server_config.argtypes = [ctypes.c_size_t, ctypes.c_int]
    L.bem_server_stats.argtypes = [ctypes.POINTER(ServerStats), ctypes.c_int]
    L.bem_server_kernel_stats.argtypes = [ctypes.POINTER(KernelStats), ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                          ctypes.c_int]
    L.bem_aca_block.argtypes = [_p, ctypes.c_int, ctypes.c_int, ctypes.c_double, _i32p, ctypes.c_int64, _i32p,
                                ctypes.c_int64, ctypes.POINTER(AcaParams), ctypes.c_int, _p, _p, _i32p, _i64p]
    L.bem_aca_callback.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ROW_FN, COL_FN, _p,
                                   ctypes.POINTER(AcaParams), _p, _p, _i32p]
    L.bem_partition.argtypes = [_dp, ctypes.c_int64, _i32p, ctypes.c_int64, ctypes.c_int, ctypes.c_int32,
                                ctypes.c_double, ctypes.c_int32, _i32p, _i32p, _i32p, ctypes.c_int64, _i32p, ctypes.c_int64, _i64p,
                                _i64p]
    L.bem_hmat_assemble.argtypes = [_p, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(HmatParams),
                                    ctypes.POINTER(_p)]
    L.bem_hmat_matvec.argtypes = [_p, _p, _p]
    L.bem_hmat_stats_get.argtypes = [_p, ctypes.POINTER(HmatStats)]
    L.bem_hmat_block_info.argtypes = [_p, ctypes.c_int64, _i32p, _i64p, _i64p, _i32p, ctypes.POINTER(_i32p),
                                      ctypes.POINTER(_i32p)]
    L.bem_hmat_block_dense.argtypes = [_p, ctypes.c_int64, _p]
    L.bem_hmat_destroy.argtypes = [_p]
    L.bem_aca_plan_create.argtypes = [_p, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.POINTER(HmatParams),
                                      ctypes.POINTER(_p)]
    L.bem_aca_plan_info.argtypes = [_p, _i64p, _i64p, _dp]
    L.bem_aca_plan_block.argtypes = [_p, ctypes.c_int64, _i64p, _i64p, ctypes.POINTER(_i32p), ctypes.POINTER(_i32p)]
    L.bem_aca_plan_run.argtypes = [_p, _i64p, _dp, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(AcaRunStats)]
    L.bem_aca_plans_run.argtypes = [ctypes.POINTER(_p), ctypes.c_int64, _i64p, _i64p, _dp, ctypes.c_int64,
                                    ctypes.c_int, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(AcaRunStats)]
    L.bem_aca_plan_factors.argtypes = [_p, ctypes.c_int64, _i32p, _p, _p]
    L.bem_aca_plan_destroy.argtypes = [_p]
    L.bem_eval_dense.argtypes = entry_args + [_p, ctypes.POINTER(DenseStats)]
    _LIB = L
    return L


def _check(rc):
    if rc != OK:
        msg = lib().bem_last_error().decode(errors="replace")
        if rc == E_NEARFIELD:
            raise NearFieldError(rc, msg)
        raise BemError(rc, msg)


def _idx(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32).ravel())


def is_complex(op):
    return op in (HELMHOLTZ_SLP, HELMHOLTZ_DLP, HELMHOLTZ_ADLP, HELMHOLTZ_HYPS)


def out_dtype(op, prec):
    if is_complex(op):
        return np.complex64 if prec == FP32 else np.complex128
    return np.float32 if prec == FP32 else np.float64


def _ip(a):
    return a.ctypes.data_as(_i32p)


# ---------------------------------------------------------------------------
class Mesh:
    """Handle of a device-resident mesh (bem_mesh_create)."""

    def __init__(self, handle, nv, nt):
        self.handle = handle
        self.nv = nv
        self.nt = nt

    def info(self) -> MeshInfo:
        inf = MeshInfo()
        _check(lib().bem_mesh_info(self.handle, ctypes.byref(inf)))
        return inf

    def destroy(self):
        if self.handle:
            _check(lib().bem_mesh_destroy(self.handle))
            self.handle = None


def mesh_create(xyz, tri, quad_points: int = 6) -> Mesh:
    xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64))
    tri = np.ascontiguousarray(np.asarray(tri, dtype=np.int32))
    h = _p()
    _check(lib().bem_mesh_create(xyz.ctypes.data_as(_dp), xyz.shape[0], _ip(tri), tri.shape[0], quad_points,
                                 ctypes.byref(h)))
    return Mesh(h, xyz.shape[0], tri.shape[0])


def mesh_destroy(mesh: Mesh):
    mesh.destroy()


def eval_entries(mesh: Mesh, op, space, k, rows, cols, prec=FP32, near=NEAR_SKIP) -> np.ndarray:
    rows, cols = _idx(rows), _idx(cols)
    out = np.empty((rows.size, cols.size), dtype=out_dtype(op, prec))
    _check(lib().bem_eval_entries(mesh.handle, op, space, float(k), _ip(rows), rows.size, _ip(cols), cols.size,
                                  prec, near, out.ctypes.data_as(_p)))
    return out


def eval_dense(mesh: Mesh, op, space, k, rows, cols, prec=FP32, near=NEAR_SKIP, stats=False):
    """A[rows, cols] of a P1 block by triangle pairs (bem_eval_dense); with
    stats=True also returns the call's bem_dense_stats as a dict."""
    rows, cols = _idx(rows), _idx(cols)
    out = np.empty((rows.size, cols.size), dtype=out_dtype(op, prec))
    st = DenseStats()
    _check(lib().bem_eval_dense(mesh.handle, op, space, float(k), _ip(rows), rows.size, _ip(cols), cols.size, prec,
                                near, out.ctypes.data_as(_p), ctypes.byref(st)))
    if stats:
        return out, {f: getattr(st, f) for f, _ in DenseStats._fields_}
    return out


class Ticket:
    def __init__(self, handle, out, keep):
        self.handle = handle
        self.out = out
        self._keep = keep

    def wait(self, timeout: float = -1.0) -> np.ndarray:
        _check(lib().bem_ticket_wait(self.handle, float(timeout)))
        return self.out

    def times(self):
        a, b = ctypes.c_double(), ctypes.c_double()
        _check(lib().bem_ticket_times(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def free(self):
        if self.handle:
            lib().bem_ticket_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def submit(mesh: Mesh, op, space, k, rows, cols, prec=FP32, near=NEAR_SKIP) -> Ticket:
    rows, cols = _idx(rows), _idx(cols)
    out = np.empty((rows.size, cols.size), dtype=out_dtype(op, prec))
    t = _p()
    _check(lib().bem_submit(mesh.handle, op, space, float(k), _ip(rows), rows.size, _ip(cols), cols.size, prec,
                            near, out.ctypes.data_as(_p), ctypes.byref(t)))
    return Ticket(t, out, (rows, cols))


def _device_request(fn, mesh: Mesh, op, space, k, rows, cols, out, prec, near, stream):
    import torch
    rows, cols = _idx(rows), _idx(cols)
    want = {np.float32: torch.float32, np.float64: torch.float64, np.complex64: torch.complex64,
            np.complex128: torch.complex128}[out_dtype(op, prec)]
    if out.dtype != want or not out.is_cuda or not out.is_contiguous() or out.numel() != rows.size * cols.size:
        raise ValueError("out must be a contiguous device tensor of the right dtype and size")
    s = stream if stream is not None else torch.cuda.current_stream(out.device)
    _check(fn(mesh.handle, op, space, float(k), _ip(rows), rows.size, _ip(cols), cols.size, prec, near,
              ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(s.cuda_stream)))
    return out


def eval_entries_async(mesh: Mesh, op, space, k, rows, cols, out, prec=FP32, near=NEAR_SKIP, stream=None):
    """Write A[rows, cols] into the device tensor `out` (torch, row-major,
    dtype matching op/prec) on `stream` (torch.cuda.Stream; default: the
    current stream)."""
    return _device_request(lib().bem_eval_entries_async, mesh, op, space, k, rows, cols, out, prec, near, stream)


def eval_entries_async_noalloc(mesh: Mesh, op, space, k, rows, cols, out, prec=FP32, near=NEAR_SKIP, stream=None):
    """bem_eval_entries_async_noalloc: as eval_entries_async, with the
    library's fixed per-device workspace instead of any allocation."""
    return _device_request(lib().bem_eval_entries_async_noalloc, mesh, op, space, k, rows, cols, out, prec, near,
                           stream)


def server_config(arena_bytes: int, max_batch_requests: int = 16384):
    _check(lib().bem_server_config(int(arena_bytes), int(max_batch_requests)))


def server_stats(reset: bool = False) -> dict:
    s = ServerStats()
    _check(lib().bem_server_stats(ctypes.byref(s), 1 if reset else 0))
    return {f: getattr(s, f) for f, _ in ServerStats._fields_}


def server_kernel_stats(reset: bool = False) -> list:
    arr = (KernelStats * 256)()
    n = ctypes.c_int()
    _check(lib().bem_server_kernel_stats(arr, 256, ctypes.byref(n), 1 if reset else 0))
    return [{f: getattr(arr[i], f) for f, _ in KernelStats._fields_} for i in range(min(n.value, 256))]


# ---------------------------------------------------------------------------
def _aca_outputs(m, n, max_rank, cplx):
    dt = np.complex128 if cplx else np.float64
    U = np.zeros((max_rank, m), dtype=dt)   # column-major m x max_rank == row-major (max_rank, m)
    V = np.zeros((max_rank, n), dtype=dt)
    return U, V


def aca_block(mesh: Mesh, op, space, k, rows, cols, tol=1e-5, max_rank=200, prec=FP32, zero_abs=-1.0):
    """Returns (U, V, entries) with the block ~= U @ V.T."""
    rows, cols = _idx(rows), _idx(cols)
    U, V = _aca_outputs(rows.size, cols.size, max_rank, is_complex(op))
    rank = ctypes.c_int32()
    ent = ctypes.c_int64()
    prm = AcaParams(tol, max_rank, zero_abs)
    _check(lib().bem_aca_block(mesh.handle, op, space, float(k), _ip(rows), rows.size, _ip(cols), cols.size,
                               ctypes.byref(prm), prec, U.ctypes.data_as(_p), V.ctypes.data_as(_p),
                               ctypes.byref(rank), ctypes.byref(ent)))
    r = rank.value
    return U[:r].T.copy(), V[:r].T.copy(), ent.value


def aca_callback(get_row, get_col, m, n, tol=1e-5, max_rank=200, zero_abs=0.0, is_complex_=False):
    """ACA of the library on caller-supplied rows/columns (host only)."""
    cdt = np.complex128 if is_complex_ else np.float64
    f = 2 if is_complex_ else 1
    errors = []

    def fill(fn, idx, out, length):
        dst = np.ctypeslib.as_array(out, shape=(length * f,))
        try:
            v = np.ascontiguousarray(np.asarray(fn(int(idx)), dtype=cdt).ravel())
            dst[:] = v.view(np.float64)
        except Exception as e:  # surfaced after the call returns
            errors.append(e)
            dst[:] = 0.0

    rf = ROW_FN(lambda ctx, i, out: fill(get_row, i, out, n))
    cf_ = COL_FN(lambda ctx, j, out: fill(get_col, j, out, m))
    U, V = _aca_outputs(m, n, max_rank, is_complex_)
    rank = ctypes.c_int32()
    prm = AcaParams(tol, max_rank, zero_abs)
    _check(lib().bem_aca_callback(m, n, 1 if is_complex_ else 0, rf, cf_, None, ctypes.byref(prm),
                                  U.ctypes.data_as(_p), V.ctypes.data_as(_p), ctypes.byref(rank)))
    if errors:
        raise errors[0]
    r = rank.value
    return U[:r].T.copy(), V[:r].T.copy()


def partition(xyz, tri, space, leaf_size=100, eta=1.0, max_block=0):
    """(perm, cluster ranges [(begin, end)], blocks [(tau, sigma, admissible)])."""
    xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64))
    tri = np.ascontiguousarray(np.asarray(tri, dtype=np.int32))
    nd = {P0: tri.shape[0], P1: xyz.shape[0], DP1: 3 * tri.shape[0]}[space]
    nc, nb = ctypes.c_int64(), ctypes.c_int64()
    rc = lib().bem_partition(xyz.ctypes.data_as(_dp), xyz.shape[0], _ip(tri), tri.shape[0], space, leaf_size,
                             float(eta), int(max_block), None, None, None, 0, None, 0, ctypes.byref(nc), ctypes.byref(nb))
    if rc not in (OK, E_ARG) or nc.value <= 0:
        _check(rc)
    perm = np.zeros(nd, dtype=np.int32)
    cb = np.zeros(nc.value, dtype=np.int32)
    ce = np.zeros(nc.value, dtype=np.int32)
    blocks = np.zeros((nb.value, 3), dtype=np.int32)
    _check(lib().bem_partition(xyz.ctypes.data_as(_dp), xyz.shape[0], _ip(tri), tri.shape[0], space, leaf_size,
                               float(eta), int(max_block), _ip(perm), _ip(cb), _ip(ce), nc.value, _ip(blocks), nb.value,
                               ctypes.byref(nc), ctypes.byref(nb)))
    return perm, np.stack([cb, ce], axis=1), blocks


class HMatrix:
    def __init__(self, handle, ndof, cplx):
        self.handle = handle
        self.ndof = ndof
        self.cplx = cplx

    def stats(self) -> dict:
        s = HmatStats()
        _check(lib().bem_hmat_stats_get(self.handle, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in HmatStats._fields_}

    def matvec(self, x):
        dt = np.complex128 if self.cplx else np.float64
        x = np.ascontiguousarray(np.asarray(x, dtype=dt))
        y = np.zeros(self.ndof, dtype=dt)
        _check(lib().bem_hmat_matvec(self.handle, x.ctypes.data_as(_p), y.ctypes.data_as(_p)))
        return y

    def block(self, b):
        adm, m, n, rank = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        rp, cp = _i32p(), _i32p()
        _check(lib().bem_hmat_block_info(self.handle, b, ctypes.byref(adm), ctypes.byref(m), ctypes.byref(n),
                                         ctypes.byref(rank), ctypes.byref(rp), ctypes.byref(cp)))
        rows = np.ctypeslib.as_array(rp, shape=(m.value,)).copy()
        cols = np.ctypeslib.as_array(cp, shape=(n.value,)).copy()
        dense = np.zeros((m.value, n.value), dtype=np.complex128 if self.cplx else np.float64)
        _check(lib().bem_hmat_block_dense(self.handle, b, dense.ctypes.data_as(_p)))
        return bool(adm.value), rows, cols, rank.value, dense

    def destroy(self):
        if self.handle:
            lib().bem_hmat_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def hmat_assemble(mesh: Mesh, op, space, k, leaf_size=100, eta=1.0, aca_tol=1e-5, max_rank=200, n_workers=8,
                  blocks_per_worker=32, prec=FP32, dense_mode=0, max_block=0, hyps_via_slp=0) -> HMatrix:
    prm = HmatParams(leaf_size, eta, aca_tol, max_rank, n_workers, blocks_per_worker, prec, dense_mode, max_block,
                     hyps_via_slp)
    h = _p()
    _check(lib().bem_hmat_assemble(mesh.handle, op, space, float(k), ctypes.byref(prm), ctypes.byref(h)))
    return HMatrix(h, {P0: mesh.nt, P1: mesh.nv, DP1: 3 * mesh.nt}[space], is_complex(op))


class AcaPlan:
    """Handle of an ACA plan (bem_aca_plan_create): partition and resident
    lane sets of one operator, serving runs over its admissible blocks."""

    def __init__(self, handle, cplx):
        self.handle = handle
        self.cplx = cplx

    def info(self):
        nb, nd, st = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        _check(lib().bem_aca_plan_info(self.handle, ctypes.byref(nb), ctypes.byref(nd), ctypes.byref(st)))
        return {"blocks": nb.value, "ndof": nd.value, "setup_seconds": st.value}

    def block(self, b):
        m, n = ctypes.c_int64(), ctypes.c_int64()
        rp, cp = _i32p(), _i32p()
        _check(lib().bem_aca_plan_block(self.handle, int(b), ctypes.byref(m), ctypes.byref(n), ctypes.byref(rp),
                                        ctypes.byref(cp)))
        return (np.ctypeslib.as_array(rp, shape=(m.value,)).copy(),
                np.ctypeslib.as_array(cp, shape=(n.value,)).copy())

    def run(self, blocks, arrival=None, prec=FP32) -> dict:
        blocks = np.ascontiguousarray(np.asarray(blocks, dtype=np.int64).ravel())
        arr = None
        if arrival is not None:
            arr = np.ascontiguousarray(np.asarray(arrival, dtype=np.float64).ravel())
            if arr.size != blocks.size:
                raise ValueError("one arrival time per block")
        st = AcaRunStats()
        _check(lib().bem_aca_plan_run(self.handle, blocks.ctypes.data_as(_i64p),
                                      arr.ctypes.data_as(_dp) if arr is not None else None, blocks.size, prec,
                                      ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in AcaRunStats._fields_}

    def factors(self, b):
        rows, cols = self.block(b)
        r = ctypes.c_int32()
        _check(lib().bem_aca_plan_factors(self.handle, int(b), ctypes.byref(r), None, None))
        dt = np.complex128 if self.cplx else np.float64
        U = np.zeros((r.value, rows.size), dtype=dt)
        V = np.zeros((r.value, cols.size), dtype=dt)
        _check(lib().bem_aca_plan_factors(self.handle, int(b), ctypes.byref(r), U.ctypes.data_as(_p),
                                          V.ctypes.data_as(_p)))
        return U.T.copy(), V.T.copy()

    def destroy(self):
        if self.handle:
            lib().bem_aca_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def aca_plans_run(plans, plan_index, blocks, arrival=None, prec=FP32, n_workers=32, blocks_per_worker=128) -> dict:
    """bem_aca_plans_run: one served stream over blocks of several plans
    (block i is blocks[i] of plans[plan_index[i]])."""
    pidx = np.ascontiguousarray(np.asarray(plan_index, dtype=np.int64).ravel())
    blocks = np.ascontiguousarray(np.asarray(blocks, dtype=np.int64).ravel())
    if pidx.size != blocks.size:
        raise ValueError("one plan index per block")
    arr = None
    if arrival is not None:
        arr = np.ascontiguousarray(np.asarray(arrival, dtype=np.float64).ravel())
        if arr.size != blocks.size:
            raise ValueError("one arrival time per block")
    handles = (_p * len(plans))(*[pl.handle for pl in plans])
    st = AcaRunStats()
    _check(lib().bem_aca_plans_run(handles, len(plans), pidx.ctypes.data_as(_i64p), blocks.ctypes.data_as(_i64p),
                                   arr.ctypes.data_as(_dp) if arr is not None else None, blocks.size, prec,
                                   int(n_workers), int(blocks_per_worker), ctypes.byref(st)))
    return {f: getattr(st, f) for f, _ in AcaRunStats._fields_}


def aca_plan_create(mesh: Mesh, op, space, k, leaf_size=100, eta=1.0, aca_tol=1e-5, max_rank=200, n_workers=8,
                    blocks_per_worker=32, prec=FP32, max_block=0) -> AcaPlan:
    prm = HmatParams(leaf_size, eta, aca_tol, max_rank, n_workers, blocks_per_worker, prec, 0, max_block, 0)
    h = _p()
    _check(lib().bem_aca_plan_create(mesh.handle, op, space, float(k), ctypes.byref(prm), ctypes.byref(h)))
    return AcaPlan(h, is_complex(op))
