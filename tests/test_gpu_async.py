"""GPU: asynchronous (chaotic) relaxation, jac_solve_async.

Which values a tile reads depends on timing, so results are not
bit-reproducible and are checked by what holds at any timing: the returned x
passes the stop test (recomputed here from the matrix), its error against the
manufactured solution obeys the bound its residual gives, and the number of
passes stays within a regression guard of the oracle's synchronous sweep count
(measured: 0.66-0.73 of it on the 7-point Laplacian, where in-place updates
damp the oscillatory modes Jacobi leaves, 1.1-1.6 on the Q1 cubes)."""
import numpy as np
import pytest

from gpu_util import B, get_x, make, need_gpu, set_x
from oracle import ref
from paper_2112_02377_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c1():
    return W.laplace7(20, workload=1)


@pytest.mark.parametrize("mode,P,sub,R", [(1, 4, None, 8), (2, 4, None, 1), (3, 4, (2, 2, 1), 16), (2, 7, None, 64)])
def test_async_solve_passes_its_test_and_the_error_bound(c1, mode, P, sub, R):
    need_gpu()
    b = B()
    h = make(c1, mode, P, sub)
    st, rounds, rr = b.jac_solve_async(h, 1e-8, 20000, rounds_per_check=R)
    assert st == b.JAC_OK
    x = get_x(h, c1.n)[0]
    A = c1.scipy()
    r = np.linalg.norm(c1.b[0] - A @ x)
    bn = np.linalg.norm(c1.b[0])
    assert r / bn <= 1e-8 * (1 + 1e-9)
    assert rr[0] == pytest.approx(r / bn, rel=1e-9)
    # ||x - x*||_2 <= ||r||_2 / lambda_min, lambda_min = 6 (1 - cos(pi / 21))
    lam = 6.0 * (1.0 - np.cos(np.pi / 21))
    assert np.linalg.norm(x - c1.extra["xstar"]) <= r / lam * (1 + 1e-9)
    _, _, ko, _ = ref.solve(c1.row_ptr, c1.col_idx, c1.vals, c1.b[0], 1e-8, 20000)
    assert rounds[0] % R == 0 and rounds[0] <= 1.25 * ko + R, (rounds[0], ko)
    b.jac_destroy(h)


def test_async_set1_cube_with_the_papers_stop_test():
    need_gpu()
    b = B()
    s = W.fe_q1_cube(33)
    h = make(s, 3, 8, (2, 2, 2))
    st, rounds, rr = b.jac_solve_async(h, 1e-8, 100000, b.JAC_NORM_INF_ABS, rounds_per_check=16)
    assert st == b.JAC_OK
    x = get_x(h, s.n)[0]
    res = np.abs(s.b[0] - s.scipy() @ x).max()
    assert res < 1e-8 and rr[0] == pytest.approx(res, rel=1e-9)
    # no per-pass rate is guaranteed for chaotic relaxation; a regression guard
    # at twice the synchronous count (745 sweeps; measured 1.13-1.62 times it
    # for 4-64 passes per launch: a workgroup that runs ahead iterates on
    # stale neighbour values)
    assert rounds[0] <= 2 * 745 + 16, rounds[0]
    b.jac_destroy(h)


def test_async_two_right_hand_sides_and_edge_cases():
    need_gpu()
    b = B()
    s = W.laplace7(12, workload=1)
    rng = np.random.default_rng(4)
    s2 = W.CSRSystem(s.row_ptr, s.col_idx, s.vals, np.stack([s.b[0], rng.uniform(-1, 1, s.n)]), grid=s.grid)
    h = make(s2, 2, 3)
    st, rounds, rr = b.jac_solve_async(h, 1e-9, 50000, rounds_per_check=4)
    assert st == b.JAC_OK
    x = get_x(h, s.n, 2)
    for c in range(2):
        assert np.linalg.norm(s2.b[c] - s.scipy() @ x[c]) <= 1e-9 * np.linalg.norm(s2.b[c]) * (1 + 1e-9)
    # maxit spent: JAC_NOT_CONVERGED after exactly maxit passes
    b.jac_set_x(h, None)
    st, rounds, rr = b.jac_solve_async(h, 1e-14, 37, rounds_per_check=8)
    assert st == b.JAC_NOT_CONVERGED and rounds[0] == 37
    # a solution already in place: no pass at all
    set_x(h, x)
    st, rounds, rr = b.jac_solve_async(h, 1e-8, 100)
    assert st == b.JAC_OK and rounds[0] == 0
    with pytest.raises(b.JacError):
        b.jac_solve_async(h, 1e-8, 100, rounds_per_check=0)
    b.jac_destroy(h)


def test_async_contraction_against_the_synchronous_rate():
    # fixed passes (tol 0 never passes): the residual after m passes is at
    # most a small factor above the synchronous residual after m sweeps
    need_gpu()
    b = B()
    s = W.laplace7(24, workload=1)
    h = make(s, 2, 8)
    m = 256
    st, rounds, rr = b.jac_solve_async(h, 0.0, m, rounds_per_check=32)
    assert st == b.JAC_NOT_CONVERGED and rounds[0] == m
    _, _, hist = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], m + 1)
    sync_rel = hist[m] / np.linalg.norm(s.b[0])
    assert rr[0] <= 2.0 * sync_rel, (rr[0], sync_rel)
    b.jac_destroy(h)
