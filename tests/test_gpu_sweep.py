"""GPU parity of the fused sweep, the device loop and the partitioner against
the CPU oracle, through the C ABI."""
import numpy as np
import pytest

from gpu_util import B, get_x, make, need_gpu, rel_inf, set_x, sweep, torch
from oracle import partition as OP
from oracle import ref
from paper_2112_02377_amd import workloads as W

pytestmark = pytest.mark.gpu

MODES = [("JB", 1), ("JBO", 2), ("JSS", 3)]


@pytest.fixture(scope="module")
def c1():
    need_gpu()
    return W.laplace7(20)


def test_first_sweep_is_bit_exact(c1):
    b = B()
    for mode, P in [(b.JAC_BANDROW, 4), (b.JAC_BANDROW_SP, 4), (b.JAC_SUBSTRUCT, 4)]:
        h = make(c1, mode, P, (2, 2, 1) if mode == b.JAC_SUBSTRUCT else None)
        sweep(h, 1)
        x = get_x(h, c1.n)[0]
        _, xr, _ = ref.sweeps(c1.row_ptr, c1.col_idx, c1.vals, c1.b[0], 1)
        assert np.array_equal(x, xr), mode
        b.jac_destroy(h)


@pytest.mark.parametrize("mode,P,sub", [(1, 4, None), (2, 4, None), (3, 4, (2, 2, 1)), (3, 8, (2, 2, 2)),
                                        (2, 1, None), (1, 7, None)])
def test_sweeps_and_history_match_oracle(c1, mode, P, sub):
    b = B()
    h = make(c1, mode, P, sub)
    K = 300
    hist = sweep(h, K)[:, 0]
    x = get_x(h, c1.n)[0]
    _, xr, hr = ref.sweeps(c1.row_ptr, c1.col_idx, c1.vals, c1.b[0], K)
    assert rel_inf(x, xr) <= 1e-12
    assert np.all(np.abs(hist - hr) <= 1e-12 * hr)
    # continuing from the kept iterate equals one longer run
    hist2 = sweep(h, 7)[:, 0]
    _, xr2, hr2 = ref.sweeps(c1.row_ptr, c1.col_idx, c1.vals, c1.b[0], K + 7)
    assert rel_inf(get_x(h, c1.n)[0], xr2) <= 1e-12
    assert np.all(np.abs(hist2 - hr2[K:]) <= 1e-12 * hr2[K:])
    b.jac_destroy(h)


def _tie_zone(hist, k, thr):
    return any(abs(hist[j] / thr - 1.0) <= 1e-9 for j in (k - 1, k) if 0 <= j < len(hist))


@pytest.mark.parametrize("mode,P,sub", [(1, 4, None), (2, 4, None), (3, 4, (2, 2, 1))])
@pytest.mark.parametrize("loop", [0, 1])
def test_solve_matches_oracle(c1, mode, P, sub, loop):
    b = B()
    h = make(c1, mode, P, sub, opts={b.JAC_OPT_LOOP: loop})
    st, sw, rr = b.jac_solve(h, 1e-8, 5000)
    x = get_x(h, c1.n)[0]
    sto, xo, ko, rro = ref.solve(c1.row_ptr, c1.col_idx, c1.vals, c1.b[0], 1e-8, 5000)
    assert st == b.JAC_OK and sto == ref.OK
    _, _, hr = ref.sweeps(c1.row_ptr, c1.col_idx, c1.vals, c1.b[0], ko + 2)
    if not _tie_zone(hr, ko, 1e-8 * np.linalg.norm(c1.b[0])):
        assert sw[0] == ko
        assert rel_inf(x, xo) <= 1e-10
    assert abs(rr[0] - rro) <= 1e-6 * rro
    assert rr[0] <= 1e-8
    b.jac_destroy(h)


def test_persistent_and_per_launch_loops_are_bit_identical(c1):
    b = B()
    xs = []
    for loop in (0, 1, 0):
        for mode, P, sub in [(1, 4, None), (3, 4, (2, 2, 1))]:
            h = make(c1, mode, P, sub, opts={b.JAC_OPT_LOOP: loop})
            b.jac_solve(h, 1e-9, 3000)
            xs.append(get_x(h, c1.n)[0])
            b.jac_destroy(h)
    assert np.array_equal(xs[0], xs[2]) and np.array_equal(xs[0], xs[4])
    assert np.array_equal(xs[1], xs[3]) and np.array_equal(xs[1], xs[5])


@pytest.mark.parametrize("nrhs", [2, 4])
def test_several_right_hand_sides_stop_on_their_own(nrhs):
    need_gpu()
    b = B()
    s = W.laplace7(13, workload=1)          # 2197 rows: ragged last slice
    rng = np.random.default_rng(99)
    bb = rng.uniform(-1, 1, (nrhs, s.n))
    bb[1] *= 1e-3                           # a different scale converges on its own sweep
    s.b = bb
    h = make(s, 2, 3)
    st, sw, rr = b.jac_solve(h, 1e-9, 5000)
    x = get_x(h, s.n, nrhs)
    for c in range(nrhs):
        sto, xo, ko, rro = ref.solve(s.row_ptr, s.col_idx, s.vals, bb[c], 1e-9, 5000)
        assert sw[c] == ko
        assert rel_inf(x[c], xo) <= 1e-10
    b.jac_destroy(h)


def test_infinity_norm_absolute_mode(c1):
    b = B()
    h = make(c1, 1, 4)
    st, sw, rr = b.jac_solve(h, 1e-8, 10000, b.JAC_NORM_INF_ABS)
    sto, xo, ko, rro = ref.solve(c1.row_ptr, c1.col_idx, c1.vals, c1.b[0], 1e-8, 10000, ref.NORM_INF_ABS)
    # max |r_i| ~ 1e-8 carries the rounding of b_i - q_i, about eps * |b|
    assert sw[0] == ko and abs(rr[0] - rro) <= 1e-13 * np.abs(c1.b[0]).max()
    assert rel_inf(get_x(h, c1.n)[0], xo) <= 1e-10
    b.jac_destroy(h)


def test_partition_is_bit_exact_against_oracle(c1):
    b = B()
    cases = [(c1, 1, 4, None), (c1, 2, 4, None), (c1, 3, 4, (2, 2, 1)), (c1, 3, 5, (3, 2, 2)), (c1, 2, 7, None)]
    for s, mode, P, sub in cases:
        h = make(s, mode, P, sub)
        got = b.jac_get_partition(h)
        exp = OP.partition(s.row_ptr, s.col_idx, mode, P, grid=s.grid, sub_grid=sub)
        for key in ("perm", "bounds", "recv_ptr", "recv_idx"):
            assert np.array_equal(got[key], exp[key]), (mode, P, key)
        b.jac_destroy(h)


def test_one_based_paper_csr_example():
    need_gpu()
    from test_oracle_pins import fig_csr
    b = B()
    IA, JA, AA, dense = fig_csr()
    rng = np.random.default_rng(7)
    rhs = dense @ rng.uniform(-1, 1, 5)
    h = b.jac_create(5, IA + 1, JA + 1, AA, 1, rhs, index_base=1)
    st, sw, rr = b.jac_solve(h, 1e-13, 1000)
    sto, xo, ko, rro = ref.solve(IA, JA, AA, rhs, 1e-13, 1000)
    assert st == b.JAC_OK and sw[0] == ko
    assert rel_inf(get_x(h, 5)[0], xo) <= 1e-12
    b.jac_destroy(h)


def test_error_paths():
    need_gpu()
    b = B()
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([0, 1, 0, 1], np.int32)
    with pytest.raises(b.JacError) as e:
        b.jac_create(2, rp, ci, np.array([0.0, 2.0, 2.0, 1.0]), 1, np.ones(2))
    assert e.value.status == b.JAC_E_ZERO_DIAG
    with pytest.raises(b.JacError) as e:
        b.jac_create(2, rp, np.array([1, 0, 0, 1], np.int32), np.ones(4), 1, np.ones(2))
    assert e.value.status == b.JAC_E_INVALID
    h = b.jac_create(2, rp, ci, np.array([1.0, 2.0, 2.0, 1.0]), 1, np.ones(2))
    with pytest.raises(b.JacError) as e:
        b.jac_solve(h, 1e-8, 100000)
    assert e.value.status == b.JAC_E_DIVERGED
    b.jac_destroy(h)
    s = W.laplace7(6, workload=1)
    h = make(s, 1, 2)
    st, sw, rr = b.jac_solve(h, 1e-30, 9)
    assert st == b.JAC_NOT_CONVERGED and sw[0] == 9
    _, x9, _ = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], 9)
    assert rel_inf(get_x(h, s.n)[0], x9) <= 1e-13
    set_x(h, np.zeros(s.n))
    b.jac_set_rhs(h, torch.zeros(s.n, dtype=torch.float64, device="cuda"))
    st, sw, rr = b.jac_solve(h, 1e-8, 100)
    assert st == b.JAC_OK and sw[0] == 0 and rr[0] == 0.0
    with pytest.raises(b.JacError):
        b.jac_partition(h, 2, 0)
    b.jac_destroy(h)


def test_set_values_changes_the_system():
    need_gpu()
    b = B()
    s = W.diffusion_adjoint(9)
    h = make(s, 2, 3)
    st, sw, rr = b.jac_solve(h, 1e-10, 20000)
    sto, xo, ko, _ = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-10, 20000)
    assert sw[0] == ko and rel_inf(get_x(h, s.n)[0], xo) <= 1e-9
    v2 = s.vals * 1.5
    b.jac_set_values(h, torch.from_numpy(v2).cuda())
    set_x(h, np.zeros(s.n))
    st, sw, rr = b.jac_solve(h, 1e-10, 20000)
    sto, xo, ko, _ = ref.solve(s.row_ptr, s.col_idx, v2, s.b[0], 1e-10, 20000)
    assert sw[0] == ko and rel_inf(get_x(h, s.n)[0], xo) <= 1e-9
    bad = s.vals.copy()
    bad[np.flatnonzero(s.col_idx == np.repeat(np.arange(s.n), np.diff(s.row_ptr)))[3]] = 0.0
    with pytest.raises(b.JacError) as e:
        b.jac_set_values(h, torch.from_numpy(bad).cuda())
    assert e.value.status == b.JAC_E_ZERO_DIAG
    b.jac_destroy(h)


def test_reruns_are_bit_identical(c1):
    b = B()
    out = []
    for _ in range(2):
        h = make(c1, 3, 4, (2, 2, 1))
        hist = sweep(h, 200)
        out.append((get_x(h, c1.n), hist))
        b.jac_destroy(h)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


def test_column_formats_match_oracle():
    # 16-bit row-relative columns when every |j - i| fits, 32-bit otherwise
    need_gpu()
    b = B()
    narrow = W.laplace7(9, workload=1)
    wide = W.diffusion_system(200, 190, 2, np.full(200 * 190 * 2, 1.0), np.ones(200 * 190 * 2))
    for s, cb in ((narrow, 2), (wide, 4)):
        # explicit columns (the shift tables would take both)
        h = make(s, 1, 3, opts={b.JAC_OPT_SHIFT_TABLES: 0})
        assert b.jac_get_info(h)["col_bytes"] == cb
        hist = sweep(h, 40)[:, 0]
        _, xr, hr = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], 40)
        assert rel_inf(get_x(h, s.n)[0], xr) <= 1e-12
        # b - A x carries about eps * |b_i| per row: the norm's floor is eps * ||b||
        assert np.all(np.abs(hist - hr) <= 1e-12 * hr + 1e-14 * hr[0])
        b.jac_destroy(h)
