"""ctypes wrappers around the C oracle and the references derived from it.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

What pins each function (tests/test_oracle_*.py, all CPU):

* ``sweeps`` / ``solve``: x_1 = fl(1/a_ii)*b from x_0 = 0; the 7-point
  contraction ||r_{k+1}|| <= cos(pi/(N+1)) ||r_k|| and the observed rate;
  the manufactured-solution error bound; agreement with a LAPACK dense solve
  on grids up to 6^3; the paper's 5x5 CSR example (rho(T) = 0.07^(1/3) and
  e_{k+3} = 0.07 e_k); the 1.05-dominant contraction in the infinity norm;
  the stop-rule special cases (maxit, ||b|| = 0, divergence, bad CSR).
* ``adjoint``: dL/db equals K sweeps on A^T y = g (a different code path:
  the forward sweep on the transpose); the dot-product identity; brute-force
  central differences on every stored entry of small systems.
* ``theta_grad``: central differences of the loss through the generator's
  own assembly on small grids.
* ``partition`` (``oracle/partition.py``): the paper's three-band dependency
  table exactly; hand-derived closed forms for halo and interface sizes;
  brute-force definitions on small grids.
* ``batched_solve`` and ``refine_reference`` are loops of ``solve`` (plain
  definitions) and inherit its pins.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_LIB = None

OK, NOT_CONVERGED, E_INVALID, E_ZERO_DIAG, E_NOMEM, E_DIVERGED = 0, 1, -1, -2, -3, -6
NORM_L2_REL, NORM_INF_ABS = 0, 1

_i32p = C.POINTER(C.c_int32)
_f64p = C.POINTER(C.c_double)


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        L.ref_check_csr.argtypes = [C.c_int32, _i32p, _i32p, _f64p]
        L.ref_sweeps.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p, C.c_int32, _f64p, _f64p, C.c_int]
        L.ref_solve.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p, C.c_double, C.c_int32, C.c_int,
                                _f64p, _i32p, _f64p, C.c_int]
        L.ref_adjoint.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _f64p, C.c_int32, _f64p, _f64p, _f64p, _f64p]
        L.ref_sweep_rows.argtypes = [C.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p, C.c_int32, _i32p, _f64p, _f64p]
        for f in (L.ref_check_csr, L.ref_sweeps, L.ref_solve, L.ref_adjoint, L.ref_sweep_rows):
            f.restype = C.c_int
        _LIB = L
    return _LIB


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_i32p)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_f64p)


def _null():
    return C.cast(None, _f64p)


def check_csr(row_ptr, col_idx, vals) -> int:
    rp, prp = _i32(row_ptr)
    ci, pci = _i32(col_idx)
    v, pv = _f64(vals)
    return lib().ref_check_csr(len(rp) - 1, prp, pci, pv)


def sweeps(row_ptr, col_idx, vals, b, K: int, x0=None, history: bool = True, threads: int = 1):
    """K sweeps from x0 (zeros when None).  Returns (status, x_K, hist) where
    hist[k] = ||b - A x_k||_2 for k < K."""
    rp, prp = _i32(row_ptr)
    ci, pci = _i32(col_idx)
    v, pv = _f64(vals)
    bb, pb = _f64(b)
    n = len(rp) - 1
    x0a, px0 = (None, _null()) if x0 is None else _f64(x0)
    xo = np.zeros(n)
    hist = np.zeros(max(K, 0)) if history else None
    ph = hist.ctypes.data_as(_f64p) if history else _null()
    st = lib().ref_sweeps(n, prp, pci, pv, pb, px0, int(K), xo.ctypes.data_as(_f64p), ph, int(threads))
    return st, xo, hist


def solve(row_ptr, col_idx, vals, b, tol: float, maxit: int, norm: int = NORM_L2_REL, x0=None, threads: int = 1):
    """Returns (status, x, sweeps, relres) with the stop rules of ref_solve."""
    rp, prp = _i32(row_ptr)
    ci, pci = _i32(col_idx)
    v, pv = _f64(vals)
    bb, pb = _f64(b)
    n = len(rp) - 1
    x0a, px0 = (None, _null()) if x0 is None else _f64(x0)
    xo = np.zeros(n)
    sw = C.c_int32(0)
    rr = C.c_double(0.0)
    st = lib().ref_solve(n, prp, pci, pv, pb, px0, float(tol), int(maxit), int(norm), xo.ctypes.data_as(_f64p),
                         C.byref(sw), C.byref(rr), int(threads))
    return st, xo, int(sw.value), float(rr.value)


def adjoint(row_ptr, col_idx, vals, b, K: int, g):
    """Full-storage reverse sweep.  Returns (status, dL/db, dL/dvals, x_K)."""
    rp, prp = _i32(row_ptr)
    ci, pci = _i32(col_idx)
    v, pv = _f64(vals)
    bb, pb = _f64(b)
    gg, pg = _f64(g)
    n = len(rp) - 1
    gb = np.zeros(n)
    gv = np.zeros(len(ci))
    xk = np.zeros(n)
    st = lib().ref_adjoint(n, prp, pci, pv, pb, int(K), pg, gb.ctypes.data_as(_f64p), gv.ctypes.data_as(_f64p),
                           xk.ctypes.data_as(_f64p))
    return st, gb, gv, xk


def sweep_rows(row_ptr, col_idx, vals, b, x, rows):
    """x_{k+1} at the listed rows from a given x_k (and the residual there)."""
    rp, prp = _i32(row_ptr)
    ci, pci = _i32(col_idx)
    v, pv = _f64(vals)
    bb, pb = _f64(b)
    xx, px = _f64(x)
    rr, prr = _i32(rows)
    out = np.zeros(len(rr))
    res = np.zeros(len(rr))
    st = lib().ref_sweep_rows(len(rp) - 1, prp, pci, pv, pb, px, len(rr), prr, out.ctypes.data_as(_f64p),
                              res.ctypes.data_as(_f64p))
    return st, out, res


def batched_solve(systems, tol: float, maxit: int, threads: int = 1):
    """Reference for many systems with several right-hand sides: one plain
    solve per (system, right-hand side).  Returns, per system, a list over its
    right-hand sides of (status, x, sweeps, relres)."""
    out = []
    for s in systems:
        res = [solve(s.row_ptr, s.col_idx, s.vals, s.b[c], tol, maxit, NORM_L2_REL, threads=threads)
               for c in range(s.b.shape[0])]
        out.append(res)
    return out


def refine_reference(row_ptr, col_idx, vals, b, tol: float = 1e-10, maxit: int = 1_000_000, threads: int = 1):
    """FP64 solution the mixed-precision result is measured against: a plain
    FP64 solve to ``tol``."""
    return solve(row_ptr, col_idx, vals, b, tol, maxit, NORM_L2_REL, threads=threads)


def theta_grad(theta, grid, row_ptr, slot, gvals):
    """Chain rule from dL/dvals to dL/dtheta for the two-point-flux assembly
    (interior face t = 2 th_i th_j / (th_i + th_j), boundary face t = 2 th_i,
    a_ij = -t, a_ii = sum of the cell's face terms)."""
    nx, ny, nz = grid
    n = nx * ny * nz
    th = np.asarray(theta, dtype=np.float64)
    rp = np.asarray(row_ptr, dtype=np.int64)
    slot = np.asarray(slot, dtype=np.int64)
    gv = np.asarray(gvals, dtype=np.float64)
    r = np.arange(n, dtype=np.int64)
    i, j, k = r % nx, (r // nx) % ny, r // (nx * ny)
    # entry index of (row, slot) for every row, -1 when absent
    pos = np.full((n, 7), -1, dtype=np.int64)
    rows = np.repeat(r, np.diff(rp))
    pos[rows, slot] = np.arange(len(slot))
    g_diag = gv[pos[:, 3]]
    out = np.zeros(n)
    sxy = nx * ny
    faces = [(0, k > 0, -sxy), (1, j > 0, -nx), (2, i > 0, -1), (4, i < nx - 1, 1), (5, j < ny - 1, nx),
             (6, k < nz - 1, sxy)]
    for s, inside, sh in faces:
        # boundary face: t = 2 th_i enters a_ii only
        out[~inside] += 2.0 * g_diag[~inside]
        ii = r[inside]
        jj = ii + sh
        ti, tj = th[ii], th[jj]
        den = (ti + tj) ** 2
        dti = 2.0 * tj * tj / den
        dtj = 2.0 * ti * ti / den
        g_off = gv[pos[ii, s]]
        coef = g_diag[inside] - g_off    # a_ii gets +t, a_ij gets -t
        np.add.at(out, ii, coef * dti)
        np.add.at(out, jj, coef * dtj)
    return out
