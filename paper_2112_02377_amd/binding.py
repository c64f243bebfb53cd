"""ctypes binding of libjacobi.so: the C ABI under the same names.

Argument marshalling only.  Host arrays are numpy arrays; device arrays are
torch tensors on the GPU (or raw integer addresses).  Every computation runs
in the library's HIP kernels; if the library is missing this module raises.

torch is imported before the library is opened so that the process holds one
HIP runtime (torch's); the library then binds to it by soname.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime the library binds to)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libjacobi.so")

JAC_OK, JAC_NOT_CONVERGED = 0, 1
JAC_E_INVALID, JAC_E_ZERO_DIAG, JAC_E_NOMEM, JAC_E_HIP, JAC_E_STATE, JAC_E_DIVERGED = -1, -2, -3, -4, -5, -6
JAC_BANDROW, JAC_BANDROW_SP, JAC_SUBSTRUCT = 1, 2, 3
JAC_NORM_L2_REL, JAC_NORM_INF_ABS = 0, 1
JAC_FP64, JAC_FP32_REFINE = 0, 1
(JAC_OPT_TILE_ROWS, JAC_OPT_BLOCK, JAC_OPT_LDS_ELEMS, JAC_OPT_LOOP, JAC_OPT_WG_PER_CU, JAC_OPT_INNER_TOL,
 JAC_OPT_INNER_MAX, JAC_OPT_CKPT_MEM_MB, JAC_OPT_TIMING, JAC_OPT_PARTITIONER, JAC_OPT_CACHE,
 JAC_OPT_SHIFT_TABLES, JAC_OPT_GRID) = range(1, 14)
CACHE_AUTO, CACHE_KEEP, CACHE_STREAM = 0, 1, 2
PART_ROWS, PART_NNZ, PART_GRAPH = 0, 1, 2

EXPORTS = ["jac_create", "jac_set_values", "jac_set_rhs", "jac_set_grid", "jac_partition", "jac_get_partition",
           "jac_set_x", "jac_get_x", "jac_sweep", "jac_solve", "jac_solve_batched", "jac_adjoint", "jac_autotune",
           "jac_set_option", "jac_get_option", "jac_get_info", "jac_destroy", "jac_status_string", "jac_last_error",
           "jac_graph_partition", "jac_solve_async", "jac_get_send_lists", "jac_autotune_batched",
           "jac_sweep_checkpointed", "jac_sweep_noalloc"]


class jac_info(C.Structure):
    _fields_ = [("n", C.c_int32), ("nrhs", C.c_int32), ("nparts", C.c_int32), ("mode", C.c_int32),
                ("nnz", C.c_int64), ("ell_slots", C.c_int64), ("ntiles", C.c_int32), ("nslices", C.c_int32),
                ("max_footprint", C.c_int32), ("col_bytes", C.c_int32), ("halo_entries", C.c_int64),
                ("staged_entries", C.c_int64), ("alg_bytes_per_sweep", C.c_int64),
                ("dev_bytes_per_sweep", C.c_int64), ("loop_grid", C.c_int32), ("block", C.c_int32),
                ("last_loop_ms", C.c_double), ("last_loop_sweeps", C.c_int32), ("keep_matrix", C.c_int32),
                ("state_gen", C.c_int64), ("table_slots", C.c_int64),
                ("col_format", C.c_int32), ("pad2_", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class JacError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{status_name(status)}: {msg}")
        self.status = status


_LIB = None
_i32p = C.POINTER(C.c_int32)
_i64p = C.POINTER(C.c_int64)
_f64p = C.POINTER(C.c_double)
_vp = C.c_void_p


def lib():
    """Open libjacobi.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2112_02377_amd/build.py")
        L = C.CDLL(LIB_PATH)
        sig = {
            "jac_create": [C.c_int32, _i32p, _i32p, _f64p, C.c_int32, _f64p, C.c_int32, _vp, C.POINTER(_vp)],
            "jac_set_values": [_vp, _vp],
            "jac_set_rhs": [_vp, _vp],
            "jac_set_grid": [_vp, C.c_int32, C.c_int32, C.c_int32],
            "jac_partition": [_vp, C.c_int, C.c_int32, _i32p],
            "jac_get_partition": [_vp, _i32p, _i32p, _i32p, _i32p, _i32p, _i64p],
            "jac_set_x": [_vp, _vp],
            "jac_get_x": [_vp, _vp],
            "jac_sweep": [_vp, C.c_int32, _vp],
            "jac_solve": [_vp, C.c_double, C.c_int32, C.c_int, C.c_int, _i32p, _f64p],
            "jac_solve_batched": [C.POINTER(_vp), C.c_int32, C.c_double, C.c_int32, _i32p, _f64p],
            "jac_adjoint": [_vp, C.c_int32, C.c_int32, _vp, _vp, _vp],
            "jac_autotune": [_vp, C.c_int32],
            "jac_set_option": [_vp, C.c_int, C.c_int64],
            "jac_get_option": [_vp, C.c_int, _i64p],
            "jac_get_info": [_vp, C.POINTER(jac_info)],
            "jac_graph_partition": [C.c_int32, _i32p, _i32p, C.c_int32, _i32p],
            "jac_solve_async": [_vp, C.c_double, C.c_int32, C.c_int, C.c_int32, _i32p, _f64p],
            "jac_get_send_lists": [_vp, _i32p, _i32p, _i32p, _i64p],
            "jac_autotune_batched": [C.POINTER(_vp), C.c_int32, C.c_int32],
            "jac_sweep_checkpointed": [_vp, C.c_int32, C.c_int32],
            "jac_sweep_noalloc": [_vp, C.c_int32, _vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = C.c_int
        L.jac_destroy.argtypes = [_vp]
        L.jac_destroy.restype = None
        L.jac_status_string.argtypes = [C.c_int]
        L.jac_status_string.restype = C.c_char_p
        L.jac_last_error.argtypes = []
        L.jac_last_error.restype = C.c_char_p
        _LIB = L
    return _LIB


def status_name(st: int) -> str:
    return lib().jac_status_string(int(st)).decode()


def _check(st: int, soft_ok: bool = True) -> int:
    if st < 0 or (st > 0 and not soft_ok):
        raise JacError(st, lib().jac_last_error().decode())
    return st


def _dev(t):
    """Device address of a torch tensor (checked contiguous, on the GPU) or an int."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("device arguments must be contiguous GPU tensors")
    return t.data_ptr()


def _host_i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_i32p)


def _host_f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_f64p)


def current_stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def jac_create(n, row_ptr, col_idx, vals, nrhs=1, b=None, index_base=0, stream=None):
    rp, prp = _host_i32(row_ptr)
    ci, pci = _host_i32(col_idx)
    v, pv = _host_f64(vals)
    if b is None:
        pb = C.cast(None, _f64p)
    else:
        bb, pb = _host_f64(b)
    h = _vp()
    st = lib().jac_create(int(n), prp, pci, pv, int(nrhs), pb, int(index_base),
                          current_stream() if stream is None else stream, C.byref(h))
    _check(st)
    return h


def jac_destroy(h):
    lib().jac_destroy(h)


def jac_set_values(h, vals_dev):
    return _check(lib().jac_set_values(h, _dev(vals_dev)))


def jac_set_rhs(h, b_dev):
    return _check(lib().jac_set_rhs(h, _dev(b_dev)))


def jac_set_grid(h, nx, ny, nz):
    return _check(lib().jac_set_grid(h, int(nx), int(ny), int(nz)))


def jac_partition(h, mode, nparts, sub_grid=None):
    if sub_grid is None:
        p = C.cast(None, _i32p)
    else:
        sg, p = _host_i32(sub_grid)
    return _check(lib().jac_partition(h, int(mode), int(nparts), p))


def jac_get_partition(h):
    """Returns dict(perm, bounds, recv_ptr, recv_idx) as numpy arrays."""
    L = lib()
    nb = C.c_int32(0)
    nr = C.c_int64(0)
    info = jac_get_info(h)
    _check(L.jac_get_partition(h, None, None, C.byref(nb), None, None, C.byref(nr)))
    perm = np.zeros(info["n"], np.int32)
    bounds = np.zeros(max(nb.value, 1), np.int32)
    rptr = np.zeros(info["nparts"] + 1, np.int32)
    ridx = np.zeros(max(nr.value, 1), np.int32)
    _check(L.jac_get_partition(h, perm.ctypes.data_as(_i32p), bounds.ctypes.data_as(_i32p), C.byref(nb),
                               rptr.ctypes.data_as(_i32p), ridx.ctypes.data_as(_i32p), C.byref(nr)))
    return dict(perm=perm, bounds=bounds[:nb.value], recv_ptr=rptr, recv_idx=ridx[:nr.value])


def jac_get_send_lists(h):
    """Returns dict(send_ptr, send_dest, send_idx) as numpy arrays."""
    L = lib()
    ns = C.c_int64(0)
    _check(L.jac_get_send_lists(h, None, None, None, C.byref(ns)))
    P = jac_get_info(h)["nparts"]
    sptr = np.zeros(P + 1, np.int32)
    dest = np.zeros(max(ns.value, 1), np.int32)
    idx = np.zeros(max(ns.value, 1), np.int32)
    _check(L.jac_get_send_lists(h, sptr.ctypes.data_as(_i32p), dest.ctypes.data_as(_i32p), idx.ctypes.data_as(_i32p),
                                C.byref(ns)))
    return dict(send_ptr=sptr, send_dest=dest[:ns.value], send_idx=idx[:ns.value])


def jac_set_x(h, x_dev=None):
    return _check(lib().jac_set_x(h, _dev(x_dev)))


def jac_get_x(h, x_dev):
    return _check(lib().jac_get_x(h, _dev(x_dev)))


def jac_sweep(h, nsweeps, hist_dev=None):
    return _check(lib().jac_sweep(h, int(nsweeps), _dev(hist_dev)))


def jac_sweep_noalloc(h, nsweeps, hist_dev=None):
    return _check(lib().jac_sweep_noalloc(h, int(nsweeps), _dev(hist_dev)))


def jac_solve(h, tol, maxit, norm=JAC_NORM_L2_REL, prec=JAC_FP64, nrhs=None):
    """Returns (status, sweeps[nrhs], relres[nrhs]); soft JAC_NOT_CONVERGED is returned, not raised."""
    if nrhs is None:
        nrhs = jac_get_info(h)["nrhs"]
    sw = np.zeros(nrhs, np.int32)
    rr = np.zeros(nrhs, np.float64)
    st = lib().jac_solve(h, float(tol), int(maxit), int(norm), int(prec), sw.ctypes.data_as(_i32p),
                         rr.ctypes.data_as(_f64p))
    _check(st)
    return st, sw, rr


def jac_solve_async(h, tol, maxit, norm=JAC_NORM_L2_REL, rounds_per_check=16, nrhs=None):
    """Returns (status, rounds[nrhs], relres[nrhs]); JAC_NOT_CONVERGED is returned, not raised."""
    if nrhs is None:
        nrhs = jac_get_info(h)["nrhs"]
    rounds = np.zeros(nrhs, np.int32)
    rr = np.zeros(nrhs, np.float64)
    st = lib().jac_solve_async(h, float(tol), int(maxit), int(norm), int(rounds_per_check),
                               rounds.ctypes.data_as(_i32p), rr.ctypes.data_as(_f64p))
    _check(st)
    return st, rounds, rr


def jac_solve_batched(handles, tol, maxit):
    """Returns (status, sweeps[nsys, 4], relres[nsys, 4])."""
    arr = (_vp * len(handles))(*[h.value if isinstance(h, _vp) else h for h in handles])
    sw = np.full((len(handles), 4), -1, np.int32)
    rr = np.zeros((len(handles), 4), np.float64)
    st = lib().jac_solve_batched(arr, len(handles), float(tol), int(maxit), sw.ctypes.data_as(_i32p),
                                 rr.ctypes.data_as(_f64p))
    _check(st)
    return st, sw, rr


def jac_sweep_checkpointed(h, K, ckpt_every):
    return _check(lib().jac_sweep_checkpointed(h, int(K), int(ckpt_every)))


def jac_adjoint(h, K, ckpt_every, gx_dev, gb_dev=None, gvals_dev=None):
    return _check(lib().jac_adjoint(h, int(K), int(ckpt_every), _dev(gx_dev), _dev(gb_dev), _dev(gvals_dev)))


def jac_autotune(h, sweeps_per_trial=20):
    return _check(lib().jac_autotune(h, int(sweeps_per_trial)))


def jac_autotune_batched(handles, sweeps_per_trial=32):
    arr = (_vp * len(handles))(*[h.value if isinstance(h, _vp) else h for h in handles])
    return _check(lib().jac_autotune_batched(arr, len(handles), int(sweeps_per_trial)))


def jac_graph_partition(row_ptr, col_idx, nparts):
    """Host-only weighted graph partition of a CSR pattern; returns part[n]."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = rp.shape[0] - 1
    part = np.zeros(max(n, 0), dtype=np.int32)
    _check(lib().jac_graph_partition(n, rp.ctypes.data_as(_i32p), ci.ctypes.data_as(_i32p), int(nparts),
                                     part.ctypes.data_as(_i32p)))
    return part


def jac_set_option(h, opt, value):
    return _check(lib().jac_set_option(h, int(opt), int(value)))


def jac_get_option(h, opt):
    v = C.c_int64(0)
    _check(lib().jac_get_option(h, int(opt), C.byref(v)))
    return v.value


def jac_get_info(h):
    i = jac_info()
    _check(lib().jac_get_info(h, C.byref(i)))
    return i.as_dict()
