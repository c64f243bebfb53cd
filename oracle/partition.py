"""Oracle partitioner: band-row, band-row sparsity-pattern and substructuring.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).  Integer work, written
plainly with numpy; the library's own C++ partitioner must reproduce every
array here bit for bit.

Rules (paper section 4; readings where the paper is silent are marked):

* Band boundaries (section 4.2, band-row splitting: each process gets a band
  of equally sized rows).  Reading: ``bounds[p] = floor(p*n/P)``; for the
  10-row, 3-band example of section 4.2.2 this gives rows 1-3 / 4-6 / 7-10,
  which is what the paper's dependency table implies.
* Naive band-row (section 4.2.1): identity order, no dependency lists (each
  band multiplies against the whole gathered vector).
* Sparsity-pattern band-row (section 4.2.2 and its receive/send dependency
  tables): identity order; the receive list of band p is every column that a
  row of p references and that lies outside p's band, ascending and grouped
  by owning band (ascending order already groups them, as bands are
  contiguous).  Lists are structural only: no pruning of entries whose
  x value happens to be zero.  The send lists are the transpose.
* Substructuring (section 4.3, block form with the interface unknowns last).
  Reading of the part map, since METIS and the meshes are not available: with
  a grid (nx,ny,nz) and a subdomain grid (sx,sy,sz), node (i,j,k) lies in block
  (bx,by,bz) where bx is the band of i under the same floor rule with sx bands
  of nx, and so on; the block id is bx + sx*(by + sy*bz).  Without a grid the
  S = sx*sy*sz subdomains are contiguous row bands.  A node is an interface
  node iff some off-diagonal neighbour in the pattern of A or A^T lies in
  another subdomain.  New order: interiors of subdomain 0..S-1, each ascending
  by original index, then all interface nodes sorted by (subdomain, index).
  Partition q owns subdomains [floor(q*S/P), floor((q+1)*S/P)).
* Weighted variants (section 4.2.2 proposes weighting row i by its number of
  stored entries; section 4.3 takes subdomains from a graph partitioner):
  ``weights="nnz"`` puts band boundary p (and, without a grid, subdomain
  boundary s) at the largest r with nnz(rows < r) * P <= p * nnz, which is
  floor(p*n/P) when all rows hold the same count.  ``part_map`` supplies the
  part of every row for the band-row modes (new order: rows part by part,
  ascending index inside a part) and ``sub_map`` the subdomain of every node
  for substructuring; the graph partitioner that produces such maps is a
  heuristic with many valid answers and is checked by its properties, not
  here.
"""
from __future__ import annotations

import numpy as np

JB, JBO, JSS = 1, 2, 3


def band_bounds(n: int, P: int) -> np.ndarray:
    """floor(p*n/P) for p = 0..P (int64 arithmetic, no overflow)."""
    p = np.arange(P + 1, dtype=np.int64)
    return (p * int(n)) // int(P)


def nnz_bounds(row_ptr, P: int) -> np.ndarray:
    """Largest r with nnz(rows < r) * P <= p * nnz, for p = 0..P."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    W = int(rp[-1])
    out = np.zeros(P + 1, dtype=np.int64)
    for p in range(P + 1):
        # rp[r] is nnz(rows < r); rp is non-decreasing
        out[p] = np.searchsorted(rp * P, p * W, side="right") - 1
    return out


def band_of(index: np.ndarray, bounds: np.ndarray) -> np.ndarray:
    """Band holding each index: the largest p with bounds[p] <= index."""
    return np.searchsorted(bounds, index, side="right") - 1


def _rows_of_entries(row_ptr: np.ndarray) -> np.ndarray:
    n = row_ptr.shape[0] - 1
    return np.repeat(np.arange(n, dtype=np.int64), np.diff(row_ptr.astype(np.int64)))


def recv_lists(row_ptr, col_idx, owner: np.ndarray, P: int):
    """Receive lists of every part, given ``owner[row]`` in the numbering of
    ``row_ptr/col_idx``: the columns a part's rows reference that another part
    owns, unique, grouped by owner ascending and ascending within a group.
    Returns (recv_ptr[P+1], recv_idx[H])."""
    rows = _rows_of_entries(row_ptr)
    cols = col_idx.astype(np.int64)
    prow = owner[rows]
    pcol = owner[cols]
    ext = prow != pcol
    # unique (receiving part, owner, column) triples in lexicographic order
    key_part, key_owner, key_col = prow[ext], pcol[ext], cols[ext]
    order = np.lexsort((key_col, key_owner, key_part))
    key_part, key_owner, key_col = key_part[order], key_owner[order], key_col[order]
    keep = np.ones(key_col.shape[0], dtype=bool)
    keep[1:] = (key_part[1:] != key_part[:-1]) | (key_col[1:] != key_col[:-1])
    key_part, key_col = key_part[keep], key_col[keep]
    recv_ptr = np.zeros(P + 1, dtype=np.int64)
    np.add.at(recv_ptr, key_part + 1, 1)
    recv_ptr = np.cumsum(recv_ptr)
    return recv_ptr.astype(np.int32), key_col.astype(np.int32)


def send_lists(recv_ptr, recv_idx, owner: np.ndarray, P: int):
    """Transpose of the receive lists: for each owner q, the (destination p,
    index) pairs it sends, ordered by destination then index."""
    dest = np.repeat(np.arange(P, dtype=np.int64), np.diff(recv_ptr.astype(np.int64)))
    idx = recv_idx.astype(np.int64)
    src = owner[idx]
    order = np.lexsort((idx, dest, src))
    send_ptr = np.zeros(P + 1, dtype=np.int64)
    np.add.at(send_ptr, src + 1, 1)
    return np.cumsum(send_ptr).astype(np.int32), dest[order].astype(np.int32), idx[order].astype(np.int32)


def subdomain_map(n: int, grid, sub_grid) -> np.ndarray:
    """Subdomain id of every row (see the module docstring)."""
    sx, sy, sz = (int(v) for v in sub_grid)
    if grid is None:
        S = sx * sy * sz
        return band_of(np.arange(n, dtype=np.int64), band_bounds(n, S))
    nx, ny, nz = (int(v) for v in grid)
    if nx * ny * nz != n:
        raise ValueError("grid does not match n")
    r = np.arange(n, dtype=np.int64)
    i, j, k = r % nx, (r // nx) % ny, r // (nx * ny)
    bx = band_of(i, band_bounds(nx, sx))
    by = band_of(j, band_bounds(ny, sy))
    bz = band_of(k, band_bounds(nz, sz))
    return bx + sx * (by + sy * bz)


def interface_mask(row_ptr, col_idx, sub: np.ndarray) -> np.ndarray:
    """True for nodes with an off-diagonal neighbour (in A or A^T) in another
    subdomain."""
    rows = _rows_of_entries(row_ptr)
    cols = col_idx.astype(np.int64)
    cross = (rows != cols) & (sub[rows] != sub[cols])
    mask = np.zeros(sub.shape[0], dtype=bool)
    mask[rows[cross]] = True   # row i sees a foreign neighbour in A
    mask[cols[cross]] = True   # column j sees it through A^T
    return mask


def permute_csr(row_ptr, col_idx, vals, perm: np.ndarray):
    """P A P^T with new row r = old row perm[r], columns renumbered by the
    inverse permutation and re-sorted ascending within each row."""
    n = perm.shape[0]
    iperm = np.empty(n, dtype=np.int64)
    iperm[perm] = np.arange(n, dtype=np.int64)
    rp = row_ptr.astype(np.int64)
    cnt = np.diff(rp)[perm]
    new_rp = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(cnt, out=new_rp[1:])
    src = np.repeat(rp[perm] - new_rp[:-1], cnt) + np.arange(new_rp[-1], dtype=np.int64)
    new_rows = np.repeat(np.arange(n, dtype=np.int64), cnt)
    new_cols = iperm[col_idx.astype(np.int64)[src]]
    order = np.lexsort((new_cols, new_rows))
    return (new_rp.astype(np.int32), new_cols[order].astype(np.int32),
            None if vals is None else vals[src][order])


def partition(row_ptr, col_idx, mode: int, P: int, grid=None, sub_grid=None, weights: str = "rows",
              part_map=None, sub_map=None) -> dict:
    """Partition an n x n CSR pattern into P parts.

    Returns a dict with ``perm`` (new -> old), ``bounds`` (JB/JBO: band
    boundaries [P+1]; JSS: sub_int_ptr [S+1] ++ sub_ifc_ptr [S+1] ++
    part_sub_ptr [P+1]), ``owner`` (part of each new row), ``recv_ptr`` and
    ``recv_idx`` (new numbering; empty for JB) and, for JSS, ``n_interior``.
    """
    n = row_ptr.shape[0] - 1
    if P < 1 or P > max(n, 1):
        raise ValueError("nparts out of range")
    if mode in (JB, JBO):
        if part_map is not None:
            part = np.asarray(part_map, dtype=np.int64)
            perm = np.lexsort((np.arange(n), part))            # by part, then index
            bounds = np.zeros(P + 1, dtype=np.int64)
            np.cumsum(np.bincount(part, minlength=P), out=bounds[1:])
        else:
            perm = np.arange(n, dtype=np.int64)
            bounds = nnz_bounds(row_ptr, P) if weights == "nnz" else band_bounds(n, P)
        owner = band_of(np.arange(n), bounds)
        if mode == JB:
            rptr, ridx = np.zeros(P + 1, dtype=np.int32), np.zeros(0, dtype=np.int32)
        else:
            new_rp, new_ci, _ = permute_csr(row_ptr, col_idx, None, perm)
            rptr, ridx = recv_lists(new_rp, new_ci, owner, P)
        return dict(perm=perm.astype(np.int32), bounds=bounds.astype(np.int32), owner=owner,
                    recv_ptr=rptr, recv_idx=ridx)
    if mode != JSS:
        raise ValueError("unknown mode")
    if sub_grid is None:
        sub_grid = (P, 1, 1)
    S = int(np.prod(sub_grid))
    if S < P:
        raise ValueError("fewer subdomains than parts")
    if sub_map is not None:
        sub = np.asarray(sub_map, dtype=np.int64)
    elif grid is None and weights == "nnz":
        sub = band_of(np.arange(n), nnz_bounds(row_ptr, S))
    else:
        sub = subdomain_map(n, grid, sub_grid)
    ifc = interface_mask(row_ptr, col_idx, sub)
    idx = np.arange(n, dtype=np.int64)
    interior = idx[~ifc]
    interior = interior[np.argsort(sub[interior], kind="stable")]
    interface = idx[ifc]
    interface = interface[np.lexsort((interface, sub[interface]))]
    perm = np.concatenate([interior, interface])
    n_int = interior.shape[0]
    int_cnt = np.bincount(sub[~ifc], minlength=S)
    ifc_cnt = np.bincount(sub[ifc], minlength=S)
    sub_int_ptr = np.zeros(S + 1, dtype=np.int64)
    np.cumsum(int_cnt, out=sub_int_ptr[1:])
    sub_ifc_ptr = np.full(S + 1, n_int, dtype=np.int64)
    sub_ifc_ptr[1:] += np.cumsum(ifc_cnt)
    part_sub_ptr = band_bounds(S, P)
    part_of_sub = band_of(np.arange(S, dtype=np.int64), part_sub_ptr)
    owner = part_of_sub[sub[perm]]
    new_rp, new_ci, _ = permute_csr(row_ptr, col_idx, None, perm)
    rptr, ridx = recv_lists(new_rp, new_ci, owner, P)
    bounds = np.concatenate([sub_int_ptr, sub_ifc_ptr, part_sub_ptr])
    return dict(perm=perm.astype(np.int32), bounds=bounds.astype(np.int32), owner=owner,
                recv_ptr=rptr, recv_idx=ridx, n_interior=int(n_int), sub=sub, interface=ifc)
