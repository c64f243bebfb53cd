"""GPU: the shift-table column formats (JAC_OPT_SHIFT_TABLES).

A split whose slices reach their columns through few distinct shifts stores
one shift per slot column instead of a column per slot.  Its slots hold the
same entries in the same order per row as the explicit layout (ascending
column), so every path gives bit-identical results with the tables on or
off; the tests check that, which format each kind of matrix gets, and the
oracle on the table path."""
import numpy as np
import pytest

from gpu_util import B, get_x, make, need_gpu, rel_inf, sweep, torch
from oracle import ref
from paper_2112_02377_amd import workloads as W

pytestmark = pytest.mark.gpu

TABG, TABL = 3, 4


def systems():
    return {"lap13": W.laplace7(13, workload=1), "fe27": W.fe27(11, workload=3), "q1": W.fe_q1_cube(9),
            "wide": W.diffusion_system(200, 190, 2, np.full(200 * 190 * 2, 1.0), np.ones(200 * 190 * 2))}


@pytest.mark.parametrize("name", ["lap13", "fe27", "q1", "wide"])
@pytest.mark.parametrize("mode,P,sub", [(1, 3, None), (2, 4, None), (3, 4, (2, 2, 1))])
def test_tables_on_and_off_are_bit_identical(name, mode, P, sub):
    need_gpu()
    b = B()
    s = systems()[name]
    K = 11
    res = {}
    for tab in (1, 0):
        h = make(s, mode, P, sub, opts={b.JAC_OPT_SHIFT_TABLES: tab})
        info = b.jac_get_info(h)
        if tab == 0:
            assert info["table_slots"] == 0 and info["col_format"] in (0, 1, 2)
        elif mode == 1:
            assert info["col_format"] == TABG and info["col_bytes"] == 0, name
        elif mode == 2 and name in ("lap13", "fe27"):   # contiguous footprints
            assert info["col_format"] == TABL and info["table_slots"] == info["ell_slots"], name
        hist = sweep(h, K)
        x = get_x(h, s.n)[0]
        b.jac_set_x(h, None)
        st, sw, rr = b.jac_solve(h, 1e-9, 20000)
        res[tab] = (hist, x, get_x(h, s.n)[0], int(sw[0]))
        b.jac_destroy(h)
    for u, v in zip(res[1], res[0]):
        assert np.array_equal(u, v), name
    _, xr, _ = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], K)
    assert rel_inf(res[1][1], xr) <= 1e-12
    sto, xo, ko, _ = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-9, 20000)
    assert res[1][3] == ko and rel_inf(res[1][2], xo) <= 1e-10


def test_random_patterns_keep_explicit_columns():
    need_gpu()
    b = B()
    rng = np.random.default_rng(77)
    n = 3000
    rows, cols = [], []
    for i in range(n):
        c = rng.integers(0, n, 5)
        c = c[c != i]
        rows.append(np.full(c.shape[0], i)), cols.append(c)
    import scipy.sparse as sp
    off = sp.csr_matrix((-np.ones(sum(len(c) for c in cols)), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    off.sum_duplicates()
    A = (off + sp.diags(1.5 * np.asarray(abs(off).sum(axis=1)).ravel() + 1.0)).tocsr()
    A.sort_indices()
    s = W.CSRSystem(A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data, rng.uniform(-1, 1, (1, n)))
    for mode in (1, 2):
        h = make(s, mode, 3, grid=False)
        info = b.jac_get_info(h)
        assert info["table_slots"] == 0 and info["col_format"] in (0, 1, 2)
        b.jac_destroy(h)


def test_batched_refinement_and_adjoint_with_tables():
    need_gpu()
    b = B()
    # batched: tables on and off give the same sweeps and iterates
    systems_b = W.diffusion_batch(5, workload=4, lo=6, hi=12)
    out = {}
    for tab in (1, 0):
        hs = [make(s, 1, 1, opts={b.JAC_OPT_SHIFT_TABLES: tab}) for s in systems_b]
        st, sw, rr = b.jac_solve_batched(hs, 1e-8, 100000)
        out[tab] = (sw.copy(), [get_x(h, s.n, 4) for h, s in zip(hs, systems_b)])
        for h in hs:
            b.jac_destroy(h)
    assert np.array_equal(out[1][0], out[0][0])
    assert all(np.array_equal(u, v) for u, v in zip(out[1][1], out[0][1]))
    # FP32 inner sweeps on the table layout
    s = W.fe27(12, workload=3)
    xs = {}
    for tab in (1, 0):
        h = make(s, 2, 3, opts={b.JAC_OPT_SHIFT_TABLES: tab})
        st, sw, rr = b.jac_solve(h, 1e-10, 100000, b.JAC_NORM_L2_REL, b.JAC_FP32_REFINE)
        xs[tab] = (int(sw[0]), get_x(h, s.n)[0])
        b.jac_destroy(h)
    assert xs[1][0] == xs[0][0] and np.array_equal(xs[1][1], xs[0][1])
    # adjoint: the gradient pass rebuilds global columns from the shifts
    s = W.diffusion_adjoint(10)
    K = 40
    _, xo, _ = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], K)
    g = torch.from_numpy(np.ascontiguousarray(xo - s.extra["x_target"])).cuda()
    grads = {}
    for mode in (1, 2):
        for tab in (1, 0):
            h = make(s, mode, 3, opts={b.JAC_OPT_SHIFT_TABLES: tab})
            assert (b.jac_get_info(h)["table_slots"] > 0) == (tab == 1)
            gb = torch.empty(s.n, dtype=torch.float64, device="cuda")
            gv = torch.empty(s.nnz, dtype=torch.float64, device="cuda")
            b.jac_adjoint(h, K, 7, g, gb, gv)
            torch.cuda.synchronize()
            grads[(mode, tab)] = (gb.cpu().numpy(), gv.cpu().numpy())
            b.jac_destroy(h)
        assert np.array_equal(grads[(mode, 1)][0], grads[(mode, 0)][0])
        assert np.array_equal(grads[(mode, 1)][1], grads[(mode, 0)][1])
    _, gbo, gvo, _ = ref.adjoint(s.row_ptr, s.col_idx, s.vals, s.b[0], K, xo - s.extra["x_target"])
    assert np.abs(grads[(1, 1)][1] - gvo).max() <= 1e-10 * np.abs(gvo).max()


def test_async_converges_on_tables():
    need_gpu()
    b = B()
    s = W.laplace7(12, workload=1)
    for mode in (1, 2):
        h = make(s, mode, 4)
        assert b.jac_get_info(h)["table_slots"] > 0
        st, rounds, rr = b.jac_solve_async(h, 1e-8, 20000)
        assert st == b.JAC_OK and rr[0] <= 1e-8
        b.jac_destroy(h)
