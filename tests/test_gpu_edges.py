"""GPU: edge cases of the sweep path through the C ABI.

Tile shapes at their limits (64-row tiles, one tile for the whole system,
more waves than slices), LDS too small to stage (the planner then sweeps
unstaged), staged tiles on both sides of the run count where the footprint
lookup changes, a one-row system, zero sweeps, maxit = 0, and the arguments
the library rejects.  Iterates are bit-identical under every tile shape: each row
accumulates its entries in the same order whatever the tiling; only the norm's
summation order changes."""
import numpy as np
import pytest

from gpu_util import B, get_x, make, need_gpu, rel_inf, set_x, sweep, torch
from oracle import ref
from paper_2112_02377_amd import workloads as W

pytestmark = pytest.mark.gpu

SHAPES = [(64, 64), (64, 512), (128, 256), (1024, 512), (1 << 20, 256)]


@pytest.mark.parametrize("mode,P,sub", [(1, 3, None), (2, 5, None), (3, 4, (2, 2, 1))])
def test_tile_shapes_and_unstaged_fallback(mode, P, sub):
    need_gpu()
    b = B()
    s = W.laplace7(13, workload=1)             # 2197 rows: ragged against every tile size
    K = 7
    _, xr, hr = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], K)
    ref_x = None
    cases = [dict(tile=t, block=k) for t, k in SHAPES] + [dict(tile=512, block=256, lds=64)]
    for c in cases:
        opts = {b.JAC_OPT_TILE_ROWS: c["tile"], b.JAC_OPT_BLOCK: c["block"]}
        if "lds" in c:
            opts[b.JAC_OPT_LDS_ELEMS] = c["lds"]
        h = make(s, mode, P, sub, opts=opts)
        info = b.jac_get_info(h)
        if "lds" in c:
            # no 64-row tile's footprint fits 64 entries: the whole plan is unstaged
            assert info["staged_entries"] == 0 and info["max_footprint"] == 0
        hist = sweep(h, K)[:, 0]
        x = get_x(h, s.n)[0]
        if ref_x is None:
            ref_x = x
        assert np.array_equal(x, ref_x), c
        assert rel_inf(x, xr) <= 1e-12, c
        assert np.all(np.abs(hist - hr) <= 1e-12 * hr), c
        b.jac_set_x(h, None)                   # the solve continues from the handle's x
        st, sw, rr = b.jac_solve(h, 1e-8, 5000)
        sto, xo, ko, _ = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-8, 5000)
        assert int(sw[0]) == ko and rel_inf(get_x(h, s.n)[0], xo) <= 1e-10, c
        b.jac_destroy(h)


def test_one_row_system():
    need_gpu()
    b = B()
    rp = np.array([0, 1], np.int32)
    ci = np.array([0], np.int32)
    h = b.jac_create(1, rp, ci, np.array([4.0]), 1, np.array([3.0]))
    hist = sweep(h, 2)[:, 0]
    assert get_x(h, 1)[0][0] == 0.75                      # x_1 = b / a exactly
    assert hist[0] == 3.0 and hist[1] == 0.0
    b.jac_set_x(h, None)
    st, sw, rr = b.jac_solve(h, 1e-12, 10)
    sto, xo, ko, rro = ref.solve(rp, ci, np.array([4.0]), np.array([3.0]), 1e-12, 10)
    assert st == b.JAC_OK and int(sw[0]) == ko == 1 and rr[0] == rro == 0.0
    b.jac_destroy(h)


def test_zero_sweeps_and_zero_maxit():
    need_gpu()
    b = B()
    s = W.laplace7(7, workload=1)
    h = make(s, 2, 3)
    x0 = np.random.default_rng(3).uniform(-1, 1, s.n)
    set_x(h, x0)
    b.jac_sweep(h, 0)
    assert np.array_equal(get_x(h, s.n)[0], x0)
    b.jac_set_x(h, None)
    st, sw, rr = b.jac_solve(h, 1e-30, 0)
    sto, xo, ko, rro = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-30, 0)
    assert st == b.JAC_NOT_CONVERGED == sto and int(sw[0]) == ko == 0
    assert np.all(get_x(h, s.n)[0] == 0.0) and abs(rr[0] - rro) <= 1e-15
    b.jac_destroy(h)


def test_rejected_arguments():
    need_gpu()
    b = B()
    rp = np.array([0, 1, 2], np.int32)
    ci = np.array([0, 1], np.int32)
    v = np.array([2.0, 2.0])
    with pytest.raises(b.JacError) as e:
        b.jac_create(0, np.zeros(1, np.int32), np.zeros(0, np.int32), np.zeros(0), 1, np.zeros(0))
    assert e.value.status == b.JAC_E_INVALID
    with pytest.raises(b.JacError) as e:
        b.jac_create(2, rp, ci, v, 3, np.ones(6))
    assert e.value.status == b.JAC_E_INVALID
    h = b.jac_create(2, rp, ci, v, 1, np.ones(2))
    for mode, P, sub in ((1, 3, None), (2, 0, None), (3, 2, (1, 1, 1)), (7, 1, None)):
        with pytest.raises(b.JacError) as e:
            b.jac_partition(h, mode, P, sub)
        assert e.value.status == b.JAC_E_INVALID, (mode, P, sub)
    for opt, val in ((b.JAC_OPT_TILE_ROWS, 100), (b.JAC_OPT_BLOCK, 1024), (b.JAC_OPT_LDS_ELEMS, 10),
                     (b.JAC_OPT_LOOP, 2), (b.JAC_OPT_TIMING, 5)):
        with pytest.raises(b.JacError) as e:
            b.jac_set_option(h, opt, val)
        assert e.value.status == b.JAC_E_INVALID, opt
    with pytest.raises(b.JacError) as e:
        b.jac_sweep(h, -1)
    assert e.value.status == b.JAC_E_INVALID
    with pytest.raises(b.JacError) as e:
        b.jac_solve(h, -1.0, 10)
    assert e.value.status == b.JAC_E_INVALID
    with pytest.raises(b.JacError) as e:
        b.jac_set_grid(h, 3, 1, 1)
    assert e.value.status == b.JAC_E_INVALID
    # the handle still works after every rejected call
    st, sw, rr = b.jac_solve(h, 1e-12, 10)
    assert st == b.JAC_OK and np.array_equal(get_x(h, 2)[0], np.array([0.5, 0.5]))
    b.jac_destroy(h)


@pytest.mark.parametrize("mode,sub", [(2, None), (3, (2, 2, 2))])
def test_lds_budget_bounds_staged_footprints_for_four_columns(mode, sub):
    # 16384 staged entries of 4 doubles would need 512 KiB of LDS per
    # workgroup: the split bounds each tile's footprint by the device's LDS
    # (160 KiB on gfx950), splitting tiles or sweeping unstaged, and the
    # sweeps equal the default budget's to rounding and the oracle's
    need_gpu()
    b = B()
    s = W.laplace7(24, workload=1)
    rng = np.random.default_rng(11)
    s = W.CSRSystem(s.row_ptr, s.col_idx, s.vals, np.vstack([s.b[0]] + [rng.uniform(-1, 1, s.n) for _ in range(3)]),
                    grid=s.grid)
    K = 9
    out = []
    for opts in ({}, {b.JAC_OPT_LDS_ELEMS: 16384, b.JAC_OPT_TILE_ROWS: 8192, b.JAC_OPT_BLOCK: 512}):
        h = make(s, mode, 2, sub, opts=opts)         # parts of 6912 rows: one tile would stage ~8000 entries
        info = b.jac_get_info(h)
        assert info["max_footprint"] * 4 * 8 <= 160 * 1024, info["max_footprint"]
        hist = sweep(h, K, 4)
        out.append((hist, get_x(h, s.n, 4)))
        b.jac_destroy(h)
    for c in range(4):
        _, xr, hr = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[c], K)
        for hist, x in out:
            assert rel_inf(x[c], xr) <= 1e-12, c
            assert np.all(np.abs(hist[:, c] - hr) <= 1e-12 * hr), c


def runs_system(T=96, stride=1024, seed=5):
    """Rows of 64-row tile t reference their neighbours i +- 1 and, for
    j = 1 .. t mod 6, column (i + j * stride) mod n: a 64-row tile's staged
    footprint is then 1 + (t mod 6) runs (its own rows with their two
    neighbours, and one block of 64 per far shift), on both sides of the
    four runs up to which the sweep keeps a tile's runs in registers."""
    n = 64 * T
    rng = np.random.default_rng(seed)
    rows, cols = [], []
    for i in range(n):
        c = [i - 1, i + 1] + [(i + j * stride) % n for j in range(1, (i // 64) % 6 + 1)]
        c = [v for v in c if 0 <= v < n]
        rows += [i] * len(c)
        cols += c
    import scipy.sparse as sp
    off = sp.csr_matrix((-rng.uniform(0.5, 1.0, len(rows)), (rows, cols)), shape=(n, n))
    off.sum_duplicates()
    A = (off + sp.diags(np.asarray(abs(off).sum(axis=1)).ravel() + 0.5)).tocsr()
    A.sort_indices()
    return W.CSRSystem(A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data, rng.uniform(-1, 1, (1, n)))


@pytest.mark.parametrize("tables", [1, 0])
def test_staged_tiles_of_one_to_six_footprint_runs(tables):
    # 64-row tiles of 1 .. 6 runs, both run lookups in one launch (registers
    # up to four runs, the chunk table beyond): sweeps bit-identical to the
    # unstaged split, whose rows add the same entries in the same order, and
    # to the oracle to rounding; the persistent loop's solve bit-identical
    # to the per-sweep launches'
    need_gpu()
    b = B()
    s = runs_system()
    K = 12
    opts = {b.JAC_OPT_TILE_ROWS: 64, b.JAC_OPT_SHIFT_TABLES: tables}
    hj = make(s, 1, 1, opts=opts)
    hs = make(s, 2, 1, opts=opts)
    info = b.jac_get_info(hs)
    assert info["ntiles"] == 96 and info["col_format"] == (4 if tables else 2)   # staged: shift table or local columns
    # footprint entries: 66 for the own rows and their neighbours (65 at the
    # two ends), plus 64 per far shift
    fp = sum(66 + 64 * (t % 6) for t in range(96)) - 2
    assert info["staged_entries"] == fp, info["staged_entries"]
    out = []
    for h in (hj, hs):
        out.append((sweep(h, K), get_x(h, s.n)[0]))
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    _, xr, hr = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], K)
    assert rel_inf(out[1][1], xr) <= 1e-12
    assert np.all(np.abs(out[1][0][:, 0] - hr) <= 1e-12 * hr)
    res = []
    for loop in (0, 1):
        b.jac_set_option(hs, b.JAC_OPT_LOOP, loop)
        b.jac_set_x(hs, None)
        st, sw, rr = b.jac_solve(hs, 1e-10, 5000)
        assert st == b.JAC_OK
        res.append((int(sw[0]), get_x(hs, s.n)[0]))
    assert res[0][0] == res[1][0] and np.array_equal(res[0][1], res[1][1])
    sto, xo, ko, _ = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-10, 5000)
    assert res[0][0] == ko and rel_inf(res[0][1], xo) <= 1e-10
    b.jac_destroy(hj)
    b.jac_destroy(hs)
