"""GPU: seeded random sparse systems through every split and partitioner.

Irregular patterns that grid matrices never produce: rows holding only their
diagonal, rows of up to a few hundred entries, columns far enough apart to
need 32-bit offsets, tile footprints too large for LDS (the planner then
sweeps unstaged), one-row systems, 1, 2 or 4 right-hand sides.  Each case
checks the split bit for bit against the oracle's definitions (given the
graph partitioner's map when it is used), 9 sweeps against the oracle's
(iterates 1e-12 relative, norms 1e-12), and a solve (same stop sweep,
iterate 1e-10)."""
import numpy as np
import pytest
import scipy.sparse as sp

from gpu_util import B, get_x, make, need_gpu, rel_inf, sweep
from oracle import partition as OP
from oracle import ref
from paper_2112_02377_amd import workloads as W

pytestmark = pytest.mark.gpu


def random_system(seed):
    """Diagonally dominant random matrix (dominance 1.2) with a random
    pattern; b = U[-1,1]^(n x nrhs)."""
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.choice([1, 7, 200, 1500, 3000, 40000]))
    nrhs = int(rng.choice([1, 2, 4]))
    kind = seed % 4
    rows, cols = [], []
    for i in range(n):
        if kind == 0:
            k = int(rng.integers(0, 9))                       # short rows, local columns
            c = i + rng.integers(-40, 41, k)
        elif kind == 1:
            k = int(rng.integers(0, 4)) if rng.random() < 0.9 else int(rng.integers(50, 300))
            c = rng.integers(0, n, k)                         # a few wide rows, columns anywhere
        elif kind == 2:
            k = int(rng.integers(0, 6))
            c = np.concatenate([i + rng.integers(-3, 4, k), rng.integers(0, n, 1)]) if n > 1 else np.zeros(0)
        else:
            k = 0 if rng.random() < 0.3 else int(rng.integers(1, 12))   # diagonal-only rows
            c = i + rng.integers(-(n // 2), n // 2 + 1, k)
        c = np.asarray(c, dtype=np.int64)
        c = c[(c >= 0) & (c < n) & (c != i)]
        rows.append(np.full(c.shape[0], i))
        cols.append(c)
    r = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    c = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    off = sp.csr_matrix((-(0.1 + rng.random(r.shape[0])), (r, c)), shape=(n, n))
    off.sum_duplicates()
    off.sort_indices()
    diag = 1.2 * np.maximum(np.asarray(abs(off).sum(axis=1)).ravel(), 1e-3) + (off.getnnz(axis=1) == 0)
    A = (off + sp.diags(diag)).tocsr()
    A.sort_indices()
    b = rng.uniform(-1, 1, (nrhs, n))
    s = W.CSRSystem(A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data.astype(np.float64), b)
    mode = int(rng.integers(1, 4))
    P = int(rng.integers(1, min(n, 9) + 1))
    part = int(rng.integers(0, 3))
    sub = None
    if mode == 3:
        S = int(rng.integers(P, min(n, 3 * P) + 1))
        sub = (S, 1, 1)
    return s, mode, P, sub, part


@pytest.mark.parametrize("seed", range(24))
def test_random_system_split_sweeps_and_solve(seed):
    need_gpu()
    b = B()
    s, mode, P, sub, part = random_system(seed)
    h = make(s, grid=False, opts={b.JAC_OPT_PARTITIONER: part})
    b.jac_partition(h, mode, P, sub)
    got = b.jac_get_partition(h)
    kw = {}
    if part == 1:
        kw["weights"] = "nnz"
    elif part == 2 and mode == 3:
        kw["sub_map"] = b.jac_graph_partition(s.row_ptr, s.col_idx, int(np.prod(sub)))
    elif part == 2:
        kw["part_map"] = b.jac_graph_partition(s.row_ptr, s.col_idx, P)
    exp = OP.partition(s.row_ptr, s.col_idx, mode, P, sub_grid=sub, **kw)
    for key in ("perm", "bounds", "recv_ptr", "recv_idx"):
        assert np.array_equal(got[key], exp[key]), (seed, key)
    K = 9
    hist = sweep(h, K, s.nrhs)
    x = get_x(h, s.n, s.nrhs)
    for c in range(s.nrhs):
        _, xr, hr = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[c], K)
        assert rel_inf(x[c], xr) <= 1e-12, (seed, c)
        assert np.all(np.abs(hist[:, c] - hr) <= 1e-12 * hr + 1e-14 * hr[0]), (seed, c)
    b.jac_set_x(h, None)
    st, sw, rr = b.jac_solve(h, 1e-10, 5000)
    assert st == b.JAC_OK, seed
    x = get_x(h, s.n, s.nrhs)
    for c in range(s.nrhs):
        sto, xo, ko, _ = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[c], 1e-10, 5000)
        assert sto == ref.OK and int(sw[c]) == ko, (seed, c, int(sw[c]), ko)
        assert rel_inf(x[c], xo) <= 1e-10, (seed, c)
    b.jac_destroy(h)
