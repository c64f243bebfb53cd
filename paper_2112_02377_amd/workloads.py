"""Seeded synthetic inputs shaped like the paper's test matrices (§5, Table of
matrix statistics; §6 set-1 / set-2 problems).

This module builds inputs only: sparsity patterns, coefficients, right-hand
sides and targets.  It holds none of the Jacobi method's arithmetic, and is the
one module that both the GPU path and the CPU oracle's tests take inputs from.

Every generator draws from ``numpy.random.default_rng(SEED_BASE + c)`` (PCG64)
where ``c`` is the workload's number (1..5 below), in the draw order stated in
its docstring, so that any two callers get identical bytes.

Workloads (sizes as built here):

1. ``laplace7(20)``  7-point Laplacian on a 20^3 interior grid, n=8,000,
   nnz=53,600, ``b = A x*``, ``x* ~ U[-1,1]``.
2. ``laplace7(128)`` the same on 128^3, n=2,097,152, nnz=14,581,760.
3. ``fe27(96)``      27-point FE-like SPD matrix on 96^3 nodes with 10 % of
   the edges dropped, off-diagonals in [-1,-0.05], diagonal 1.05 x row sum.
4. ``diffusion_batch(256)`` 256 variable-coefficient 7-point diffusion
   systems, edges seeded in [16,64] per axis, 4 right-hand sides each.
5. ``diffusion_adjoint(64)`` 64^3 diffusion with conductivities, b and a
   target for the loss 0.5 ||x_K - x_target||^2, and 32 probe indices.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

SEED_BASE = 2112023770


def rng_for(workload: int) -> np.random.Generator:
    """PCG64 stream of workload ``workload`` (1..5)."""
    return np.random.default_rng(SEED_BASE + int(workload))


@dataclass
class CSRSystem:
    """A square sparse system in 0-based CSR with ascending columns per row.

    ``b`` is ``nrhs x n`` (one contiguous row per right-hand side, i.e. the
    ``n x nrhs`` column-major layout the C ABI takes)."""
    row_ptr: np.ndarray          # int32 [n+1]
    col_idx: np.ndarray          # int32 [nnz]
    vals: np.ndarray             # float64 [nnz]
    b: np.ndarray                # float64 [nrhs, n]
    grid: tuple | None = None    # (nx, ny, nz), x fastest, when the rows are grid nodes
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.row_ptr.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def nrhs(self) -> int:
        return int(self.b.shape[0])

    def scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix((self.vals, self.col_idx, self.row_ptr), shape=(self.n, self.n))


# --------------------------------------------------------------------------
# 7-point structure on an nx x ny x nz grid (x fastest), Dirichlet boundary
# eliminated: row r = i + nx*(j + ny*k); neighbours in ascending column order
# r-nx*ny, r-nx, r-1, r, r+1, r+nx, r+nx*ny when inside the grid.
# --------------------------------------------------------------------------

def _grid_coords(nx: int, ny: int, nz: int):
    r = np.arange(nx * ny * nz, dtype=np.int64)
    i = r % nx
    j = (r // nx) % ny
    k = r // (nx * ny)
    return r, i, j, k


def stencil7_pattern(nx: int, ny: int, nz: int):
    """Return (row_ptr, col_idx, slot) of the 7-point pattern.

    ``slot[p]`` in 0..6 names which neighbour entry ``p`` is, in the order
    (-z, -y, -x, self, +x, +y, +z); assembly routines use it to place
    coefficients without searching."""
    r, i, j, k = _grid_coords(nx, ny, nz)
    sxy = nx * ny
    offs = np.array([-sxy, -nx, -1, 0, 1, nx, sxy], dtype=np.int64)
    valid = np.stack([k > 0, j > 0, i > 0, np.ones_like(i, dtype=bool),
                      i < nx - 1, j < ny - 1, k < nz - 1], axis=1)
    cols = r[:, None] + offs[None, :]
    counts = valid.sum(axis=1)
    row_ptr = np.zeros(r.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    col_idx = cols[valid]
    slot = np.broadcast_to(np.arange(7), valid.shape)[valid]
    return row_ptr.astype(np.int32), col_idx.astype(np.int32), slot.astype(np.int8)


def laplace7(N: int, workload: int | None = None) -> CSRSystem:
    """7-point Laplacian on an N^3 interior grid: diagonal 6, neighbours -1.

    Draws: ``x* = U[-1,1]^n``; ``b = A x*``.  ``x*`` is kept in ``extra``."""
    row_ptr, col_idx, slot = stencil7_pattern(N, N, N)
    vals = np.where(slot == 3, 6.0, -1.0)
    rng = rng_for(workload if workload is not None else (1 if N == 20 else 2))
    n = N ** 3
    xstar = rng.uniform(-1.0, 1.0, n)
    sysm = CSRSystem(row_ptr, col_idx, vals, np.zeros((1, n)), grid=(N, N, N))
    sysm.b[0] = sysm.scipy() @ xstar
    sysm.extra["xstar"] = xstar
    return sysm


# --------------------------------------------------------------------------
# 27-point FE-like matrix (workload 3)
# --------------------------------------------------------------------------

def forward27_offsets(nx: int, ny: int):
    """The 13 neighbour offsets (dx,dy,dz) of the 27-point stencil whose linear
    offset dx + nx*dy + nx*ny*dz is positive, sorted by that linear offset."""
    offs = []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                lin = dx + nx * dy + nx * ny * dz
                if lin > 0:
                    offs.append((lin, dx, dy, dz))
    offs.sort()
    return [(dx, dy, dz) for _, dx, dy, dz in offs]


def fe27(N: int = 96, workload: int = 3, drop: float = 0.1) -> CSRSystem:
    """27-point connectivity on an N^3 node grid, each undirected edge dropped
    with probability ``drop``, off-diagonal ``-(0.05 + 0.95 u)``, diagonal
    ``1.05 * sum |off-diagonal|`` (1 for a row left without edges).

    Edges are enumerated node-ascending, then over ``forward27_offsets`` in
    order.  Draws: ``u_drop[M]``, ``u_val[M]``, then ``x* = U[-1,1]^n``;
    ``b = A x*``.  The diagonal sum runs over the row's off-diagonal entries
    in ascending column order."""
    nx = ny = nz = N
    r, i, j, k = _grid_coords(nx, ny, nz)
    src, dst = [], []
    cand_node = []
    for (dx, dy, dz) in forward27_offsets(nx, ny):
        ok = (i + dx >= 0) & (i + dx < nx) & (j + dy >= 0) & (j + dy < ny) & (k + dz >= 0) & (k + dz < nz)
        cand_node.append(ok)
    okmat = np.stack(cand_node, axis=1)                      # [n, 13] node-major
    lin = np.array([dx + nx * dy + nx * ny * dz for dx, dy, dz in forward27_offsets(nx, ny)], dtype=np.int64)
    src = np.broadcast_to(r[:, None], okmat.shape)[okmat]
    dst = (r[:, None] + lin[None, :])[okmat]
    M = src.shape[0]
    rng = rng_for(workload)
    u_drop = rng.random(M)
    u_val = rng.random(M)
    keep = u_drop >= drop
    val = -(0.05 + 0.95 * u_val[keep])
    s, d = src[keep], dst[keep]
    n = nx * ny * nz
    rows = np.concatenate([s, d])
    cols = np.concatenate([d, s])
    vv = np.concatenate([val, val])
    off = sp.csr_matrix((vv, (rows, cols)), shape=(n, n))
    off.sort_indices()
    # diagonal: 1.05 * sum |a_ij| over the row, ascending columns (sequential sum)
    absrow = np.zeros(n)
    rp = off.indptr
    data = np.abs(off.data)
    cnt = np.diff(rp)
    for slot in range(int(cnt.max()) if cnt.size else 0):
        has = cnt > slot
        absrow[has] += data[rp[:-1][has] + slot]
    diag = np.where(cnt > 0, 1.05 * absrow, 1.0)
    A = (off + sp.diags(diag)).tocsr()
    A.sort_indices()
    xstar = rng.uniform(-1.0, 1.0, n)
    sysm = CSRSystem(A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64),
                     np.zeros((1, n)), grid=(nx, ny, nz))
    sysm.b[0] = A @ xstar
    sysm.extra.update(xstar=xstar, n_edges_total=M, n_edges_kept=int(keep.sum()))
    return sysm


# --------------------------------------------------------------------------
# Trilinear (Q1) finite-element Laplacian on the unit cube: the discretisation
# behind the paper's Set-1 matrices (section 6: -Laplace(u) = f on [0,1]^3,
# u = 0 on the boundary, f = cos(x + y), uniform hexahedral mesh)
# --------------------------------------------------------------------------

def fe_q1_cube(N: int) -> CSRSystem:
    """Q1 stiffness matrix and load on an N^3 node mesh of the unit cube
    (h = 1/(N-1); N = 33 and N = 65 give the node counts of the paper's
    luf_cube-35937 and luf_cube-274625).  Deterministic (no draws).

    Rows are the N^3 nodes, x fastest.  A boundary node's row is the identity
    (u = 0 there, b = 0).  An interior node couples to the interior nodes of
    its 3x3x3 neighbourhood (boundary columns are eliminated, their values
    being 0) with the element stiffness summed over the 8 cubes around it:
    8h/3 on the diagonal, 0 for the 6 face neighbours (kept as stored zeros,
    as an assembled matrix holds them), -h/6 for the 12 edge neighbours and
    -h/12 for the 8 corner neighbours.  The load is the consistent mass
    product b_i = sum_j m_ij f(x_j) over the whole neighbourhood, with the
    tensor-product mass m_ij = w(dx) w(dy) w(dz), w(0) = 2h/3, w(+-1) = h/6,
    summed in ascending column order."""
    n = N ** 3
    h = 1.0 / (N - 1)
    r = np.arange(n, dtype=np.int64)
    i, j, k = r % N, (r // N) % N, r // (N * N)
    interior = (i > 0) & (i < N - 1) & (j > 0) & (j < N - 1) & (k > 0) & (k < N - 1)
    offs = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]   # ascending columns
    stiff = {0: 8.0 * h / 3.0, 1: 0.0, 2: -h / 6.0, 3: -h / 12.0}
    wt = {0: 2.0 * h / 3.0, 1: h / 6.0, -1: h / 6.0}
    f = np.cos(i * h + j * h)
    b = np.zeros(n)
    cols, vals, ok_all = [], [], []
    for dx, dy, dz in offs:
        nb = r + dx + N * dy + N * N * dz
        ii, jj, kk = i + dx, j + dy, k + dz
        nb_int = (ii > 0) & (ii < N - 1) & (jj > 0) & (jj < N - 1) & (kk > 0) & (kk < N - 1)
        if (dx, dy, dz) == (0, 0, 0):
            ok = np.ones(n, dtype=bool)                   # every row holds its diagonal
            vals.append(np.where(interior, stiff[0], 1.0))
        else:
            ok = interior & nb_int
            vals.append(np.full(n, stiff[abs(dx) + abs(dy) + abs(dz)]))
        ok_all.append(ok)
        cols.append(np.where(ok, nb, 0))
        w = wt[dx] * wt[dy] * wt[dz]
        b = b + np.where(interior, w * f[np.clip(nb, 0, n - 1)], 0.0)
    okm = np.stack(ok_all, axis=1)                    # [n, 27], ascending columns per row
    colm = np.stack(cols, axis=1)
    valm = np.stack(vals, axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(okm.sum(axis=1), out=row_ptr[1:])
    sysm = CSRSystem(row_ptr.astype(np.int32), colm[okm].astype(np.int32), valm[okm].astype(np.float64),
                     b[None, :].copy(), grid=(N, N, N))
    sysm.extra.update(h=h, interior=interior)
    return sysm


# --------------------------------------------------------------------------
# Variable-coefficient diffusion (workloads 4 and 5)
# --------------------------------------------------------------------------

def diffusion_values(theta: np.ndarray, nx: int, ny: int, nz: int, row_ptr: np.ndarray,
                     slot: np.ndarray) -> np.ndarray:
    """Cell-centred two-point-flux coefficients on the 7-point pattern (h = 1).

    Interior face between cells i and j: ``t = 2*th_i*th_j/(th_i + th_j)``;
    Dirichlet boundary face of cell i: ``t = 2*th_i``.  ``a_ij = -t`` and
    ``a_ii`` is the sum of the six face terms taken in the fixed order
    (-z, -y, -x, +x, +y, +z).  Returns ``vals`` in the pattern's entry order."""
    r, i, j, k = _grid_coords(nx, ny, nz)
    sxy = nx * ny
    th = theta.astype(np.float64)
    faces = []
    inside = [k > 0, j > 0, i > 0, i < nx - 1, j < ny - 1, k < nz - 1]
    shifts = [-sxy, -nx, -1, 1, nx, sxy]
    for ok, sh in zip(inside, shifts):
        nb = np.where(ok, r + sh, r)
        tj = th[nb]
        t_int = 2.0 * th * tj / (th + tj)
        t_bnd = 2.0 * th
        faces.append(np.where(ok, t_int, t_bnd))
    diag = faces[0]
    for f in faces[1:]:
        diag = diag + f
    n = r.shape[0]
    # per-row entries in slot order (-z,-y,-x,self,+x,+y,+z)
    table = np.stack([-faces[0], -faces[1], -faces[2], diag, -faces[3], -faces[4], -faces[5]], axis=1)
    row_of_entry = np.repeat(np.arange(n), np.diff(row_ptr.astype(np.int64)))
    return table[row_of_entry, slot.astype(np.int64)]


def diffusion_system(nx: int, ny: int, nz: int, theta: np.ndarray, b: np.ndarray) -> CSRSystem:
    row_ptr, col_idx, slot = stencil7_pattern(nx, ny, nz)
    vals = diffusion_values(theta, nx, ny, nz, row_ptr, slot)
    s = CSRSystem(row_ptr, col_idx, vals, np.atleast_2d(np.asarray(b, dtype=np.float64)), grid=(nx, ny, nz))
    s.extra.update(theta=theta, slot=slot)
    return s


def diffusion_batch(nsys: int = 256, workload: int = 4, lo: int = 16, hi: int = 64, nrhs: int = 4) -> list[CSRSystem]:
    """``nsys`` diffusion systems.  Per system, draws in order:
    ``(nx,ny,nz) = integers(lo, hi+1, 3)``, ``theta = 10**U[-1,1]^n``,
    ``b = U[-1,1]^(nrhs*n)`` (right-hand side c is entries [c*n, (c+1)*n))."""
    rng = rng_for(workload)
    out = []
    for _ in range(nsys):
        nx, ny, nz = (int(v) for v in rng.integers(lo, hi + 1, 3))
        n = nx * ny * nz
        theta = 10.0 ** rng.uniform(-1.0, 1.0, n)
        b = rng.uniform(-1.0, 1.0, nrhs * n).reshape(nrhs, n)
        out.append(diffusion_system(nx, ny, nz, theta, b))
    return out


def diffusion_adjoint(N: int = 64, workload: int = 5, nprobe: int = 32) -> CSRSystem:
    """Draws in order: ``theta = 10**U[-1,1]^n``, ``b = U[-1,1]^n``,
    ``x_target = U[-1,1]^n``, probe indices ``choice(n, nprobe, replace=False)``."""
    rng = rng_for(workload)
    n = N ** 3
    theta = 10.0 ** rng.uniform(-1.0, 1.0, n)
    b = rng.uniform(-1.0, 1.0, n)
    x_target = rng.uniform(-1.0, 1.0, n)
    probes = rng.choice(n, min(nprobe, n), replace=False)
    s = diffusion_system(N, N, N, theta, b)
    s.extra.update(x_target=x_target, probes=np.sort(probes))
    return s


def bytes_per_sweep(n: int, nnz: int) -> int:
    """Algorithmic bytes of one FP64 CSR sweep with int32 indices: values and
    columns (12 per entry), row pointers (4 per row + 1), and x, b, invD read
    plus x' written (32 per row)."""
    return 12 * nnz + 4 * (n + 1) + 32 * n


def lean_bytes_per_sweep(n: int, nnz: int, nrhs: int = 1) -> int:
    """The same without a D^-1 vector (the diagonal is taken from the row's
    own values): 12 per entry, 4 per row + 1, and b, x read plus x' written
    (24 per row and right-hand side)."""
    return 12 * nnz + 4 * (n + 1) + 24 * n * nrhs
