"""CPU: the weighted partitioners.

* nnz-weighted band boundaries (oracle definition): reduce to the equal-row
  rule when every row holds the same count, balance stored entries, and are
  the rule written out by brute force.
* The library's graph partitioner (host-only entry point, no GPU): a
  heuristic with many valid answers, so it is checked by its properties --
  every part non-empty, weights within the stated bound, deterministic,
  exact on cases with one right answer (disconnected pieces, a 2x2x2 split
  of a cube whose optimum is known), and a halo within a few percent of the
  ideal block partition on grids, far below band rows."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import partition as OP
from paper_2112_02377_amd import workloads as W


def B():
    from paper_2112_02377_amd import binding
    return binding


def halo(rp, ci, part, P):
    """Total receive-list length of a part map (oracle definitions)."""
    d = OP.partition(rp, ci, OP.JBO, P, part_map=part)
    return int(d["recv_ptr"][-1])


def test_nnz_bounds_equal_rows_reduce_to_band_rule():
    rp = np.arange(0, 7 * 1000 + 1, 7)           # 1000 rows of 7 entries
    for P in (1, 3, 7, 64, 1000):
        assert np.array_equal(OP.nnz_bounds(rp, P), OP.band_bounds(1000, P))


def test_nnz_bounds_brute_force_and_balance():
    rng = np.random.default_rng(5)
    cnt = rng.integers(1, 40, 997)
    rp = np.concatenate([[0], np.cumsum(cnt)])
    W_ = int(rp[-1])
    for P in (2, 5, 16, 100):
        b = OP.nnz_bounds(rp, P)
        for p in range(P + 1):
            ok = [r for r in range(len(cnt) + 1) if rp[r] * P <= p * W_]
            assert b[p] == max(ok)
        w = np.diff(rp[b])
        assert w.max() <= W_ / P + cnt.max()


def test_graph_partition_exact_on_disconnected_pieces():
    # two 6^3 grids side by side: the 2-way split with no cut edge is unique
    s = W.laplace7(6)
    A = sp.block_diag([s.scipy(), s.scipy()]).tocsr()
    A.sort_indices()
    part = B().jac_graph_partition(A.indptr, A.indices, 2)
    assert set(part[:216]) == {part[0]} and set(part[216:]) == {part[216]} and part[0] != part[216]


def test_graph_partition_finds_the_cube_optimum():
    # 32^3 into 8: the 2x2x2 split into 16^3 cubes has the smallest halo
    s = W.laplace7(32)
    part = B().jac_graph_partition(s.row_ptr, s.col_idx, 8)
    assert halo(s.row_ptr, s.col_idx, part, 8) == 3 * 2 * 4 * 16 * 16     # 6144
    assert halo(s.row_ptr, s.col_idx, OP.band_of(np.arange(s.n), OP.band_bounds(s.n, 8)), 8) == 14336


@pytest.mark.parametrize("N,P", [(64, 64), (24, 7)])
def test_graph_partition_properties_on_grids(N, P):
    s = W.laplace7(N)
    b = B()
    part = b.jac_graph_partition(s.row_ptr, s.col_idx, P)
    assert part.min() == 0 and part.max() == P - 1
    nnz_row = np.diff(s.row_ptr)
    w = np.bincount(part, weights=nnz_row, minlength=P)
    assert np.all(w > 0)
    assert w.max() <= 1.05 * nnz_row.sum() / P + nnz_row.max()
    assert np.array_equal(part, b.jac_graph_partition(s.row_ptr, s.col_idx, P))       # deterministic
    hg = halo(s.row_ptr, s.col_idx, part, P)
    hb = halo(s.row_ptr, s.col_idx, OP.band_of(np.arange(s.n), OP.band_bounds(s.n, P)), P)
    assert hg < 0.5 * hb
    if (N, P) == (64, 64):
        # ideal 4x4x4 blocks of 16^3: 3 axes x 3 cuts x 16 blocks x 16^2 faces, both directions
        ideal = 3 * 3 * 16 * 16 * 16 * 2
        assert ideal <= hg <= 1.05 * ideal


def test_graph_partition_on_the_fe_matrices():
    b = B()
    for s in (W.fe27(20, workload=3), W.fe_q1_cube(17)):
        part = b.jac_graph_partition(s.row_ptr, s.col_idx, 8)
        nnz_row = np.diff(s.row_ptr)
        w = np.bincount(part, weights=nnz_row, minlength=8)
        assert w.max() <= 1.05 * nnz_row.sum() / 8 + nnz_row.max()
        hb = halo(s.row_ptr, s.col_idx, OP.band_of(np.arange(s.n), OP.band_bounds(s.n, 8)), 8)
        assert halo(s.row_ptr, s.col_idx, part, 8) < hb


def test_graph_partition_edge_cases():
    b = B()
    s = W.laplace7(5)
    assert np.all(b.jac_graph_partition(s.row_ptr, s.col_idx, 1) == 0)
    one_each = b.jac_graph_partition(s.row_ptr, s.col_idx, s.n)
    assert np.array_equal(np.sort(one_each), np.arange(s.n))
    # a diagonal matrix has no edges: parts only balance
    rp = np.arange(101, dtype=np.int32)
    ci = np.arange(100, dtype=np.int32)
    part = b.jac_graph_partition(rp, ci, 4)
    assert np.bincount(part, minlength=4).max() <= 1.05 * 25 + 1
    # an unsymmetric pattern: the weights are its own row counts, the edges
    # those of A + A^T (the upper triangle of the 7-point matrix has the
    # 7-point graph)
    A = sp.csr_matrix(sp.triu(s.scipy()))
    A.sort_indices()
    pu = b.jac_graph_partition(A.indptr, A.indices, 4)
    wu = np.bincount(pu, weights=np.diff(A.indptr), minlength=4)
    assert wu.max() <= 1.05 * A.nnz / 4 + np.diff(A.indptr).max()
    hb = halo(s.row_ptr, s.col_idx, OP.band_of(np.arange(s.n), OP.band_bounds(s.n, 4)), 4)
    assert halo(s.row_ptr, s.col_idx, pu, 4) < hb
    with pytest.raises(b.JacError):
        b.jac_graph_partition(s.row_ptr, s.col_idx, s.n + 1)
    with pytest.raises(b.JacError):
        b.jac_graph_partition(s.row_ptr, s.col_idx, 0)
    bad = s.col_idx.copy()
    bad[3] = s.n
    with pytest.raises(b.JacError):
        b.jac_graph_partition(s.row_ptr, bad, 2)
