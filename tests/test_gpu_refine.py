"""GPU: FP32 inner sweeps under FP64 refinement (JAC_FP32_REFINE) against the
FP64 oracle solution."""
import numpy as np
import pytest

from gpu_util import B, get_x, make, need_gpu
from oracle import ref
from paper_2112_02377_amd import workloads as W

pytestmark = pytest.mark.gpu


def fp64_relres(s, x, c=0):
    r = s.b[c] - s.scipy() @ x
    return np.linalg.norm(r) / np.linalg.norm(s.b[c])


@pytest.mark.parametrize("mode,P,sub", [(1, 3, None), (2, 3, None), (3, 4, (2, 2, 1))])
def test_refine_reaches_fp64_tolerance_on_dominant_27pt(mode, P, sub):
    need_gpu()
    b = B()
    s = W.fe27(24, workload=3)
    h = make(s, mode, P, sub)
    st, sw, rr = b.jac_solve(h, 1e-10, 100000, b.JAC_NORM_L2_REL, b.JAC_FP32_REFINE)
    x = get_x(h, s.n)[0]
    assert st == b.JAC_OK
    # the FP64 residual of the returned x, recomputed independently
    assert fp64_relres(s, x) <= 1e-10 * 1.001
    assert rr[0] <= 1e-10
    sto, xo, ko, rro = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-10, 100000)
    err = np.abs(x - xo).max() / np.abs(xo).max()
    # both solutions carry a residual below 1e-10 ||b||; ||A^-1|| is small for a 1.05-dominant matrix
    assert err <= 1e-9, err
    # restart equivalence: inner FP32 sweeps track the FP64 sweep count
    assert ko <= sw[0] <= 1.1 * ko + 10, (sw[0], ko)
    b.jac_destroy(h)


def test_refine_on_laplacian_with_two_rhs_and_inf_norm():
    need_gpu()
    b = B()
    s = W.laplace7(12, workload=1)
    rng = np.random.default_rng(5)
    s.b = np.stack([s.b[0], rng.uniform(-1, 1, s.n)])
    h = make(s, 2, 2)
    st, sw, rr = b.jac_solve(h, 1e-10, 100000, b.JAC_NORM_L2_REL, b.JAC_FP32_REFINE)
    x = get_x(h, s.n, 2)
    assert st == b.JAC_OK
    for c in range(2):
        assert fp64_relres(s, x[c], c) <= 1e-10 * 1.001
        sto, xo, ko, _ = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[c], 1e-10, 100000)
        assert np.abs(x[c] - xo).max() <= 1e-8 * np.abs(xo).max()
        # slow Laplacian modes: FP32 rounding of each correction re-excites them, so
        # the inner sweeps exceed the FP64 count by more than on the dominant matrix
        assert ko <= sw[c] <= 1.25 * ko + 10, (c, sw[c], ko)
    b.jac_destroy(h)
    # absolute infinity-norm test, the paper's experimental criterion
    h = make(W.laplace7(12, workload=1), 1, 2)
    s1 = W.laplace7(12, workload=1)
    st, sw, rr = b.jac_solve(h, 1e-9, 100000, b.JAC_NORM_INF_ABS, b.JAC_FP32_REFINE)
    x = get_x(h, s1.n)[0]
    assert st == b.JAC_OK and np.abs(s1.b[0] - s1.scipy() @ x).max() <= 1e-9 * 1.001
    b.jac_destroy(h)


def test_refine_stops_soft_when_inner_budget_is_exhausted():
    need_gpu()
    b = B()
    s = W.laplace7(12, workload=1)
    h = make(s, 1, 2)
    st, sw, rr = b.jac_solve(h, 1e-12, 50, b.JAC_NORM_L2_REL, b.JAC_FP32_REFINE)
    assert st == b.JAC_NOT_CONVERGED and sw[0] <= 50
    x = get_x(h, s.n)[0]
    assert abs(fp64_relres(s, x) - rr[0]) <= 1e-6 * rr[0]
    b.jac_destroy(h)


def test_refine_keeps_going_on_a_slowly_converging_laplacian():
    # 64^3 7-point Laplacian to 1e-8: 256 inner sweeps cut the residual by
    # only about 0.5-0.6 per outer step, which is progress, not stagnation
    # (the FP64 ratio follows the inner one); the result is checked against
    # the FP64 oracle's solution and sweep count
    need_gpu()
    b = B()
    s = W.laplace7(64, workload=1)
    h = make(s, 2, 16)
    st, sw, rr = b.jac_solve(h, 1e-8, 1000000, b.JAC_NORM_L2_REL, b.JAC_FP32_REFINE)
    x = get_x(h, s.n)[0]
    b.jac_destroy(h)
    assert st == b.JAC_OK
    assert fp64_relres(s, x) <= 1e-8 * 1.001
    sto, xo, ko, _ = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-8, 1000000, threads=16)
    assert sto == ref.OK
    # both residuals are below 1e-8 ||b||: ||x - xo|| <= 2e-8 ||b|| / lambda_min
    lam = 6 * (1 - np.cos(np.pi / 65))
    assert np.linalg.norm(x - xo) <= 2e-8 * np.linalg.norm(s.b[0]) / lam
    assert ko <= sw[0] <= 1.25 * ko + 10, (sw[0], ko)


def test_tuned_refinement_meets_the_fp64_bars_at_full_size(tmp_path, monkeypatch):
    # the 96^3 27-point system of the refinement comparison, with the tile
    # shape and the inner stop parameters picked by jac_autotune
    need_gpu()
    b = B()
    monkeypatch.setenv("JAC_TUNE_CACHE", str(tmp_path / "tune.txt"))
    s = W.fe27(96, workload=3)
    h = make(s, 1, 64)
    b.jac_autotune(h, 20)
    tau = b.jac_get_option(h, b.JAC_OPT_INNER_TOL) * 1e-9
    mmax = b.jac_get_option(h, b.JAC_OPT_INNER_MAX)
    print(f"tuned inner tolerance {tau:g}, inner sweep cap {mmax}")
    st, sw, rr = b.jac_solve(h, 1e-10, 100000, b.JAC_NORM_L2_REL, b.JAC_FP32_REFINE)
    x = get_x(h, s.n)[0]
    b.jac_destroy(h)
    assert st == b.JAC_OK
    assert fp64_relres(s, x) <= 1e-10 * 1.001
    sto, xo, ko, _ = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-10, 100000, threads=16)
    assert sto == ref.OK
    # error bar from the arithmetic: x and xo solve A y = b up to their
    # residuals, so ||x - xo||_2 <= ||A^-1||_2 (||r|| + ||r_o||), and for this
    # symmetric diagonally dominant matrix 1/||A^-1||_2 = lambda_min is at
    # least the smallest Gershgorin margin a_ii - sum_j |a_ij|
    A = s.scipy()
    d = A.diagonal()
    off = np.asarray(abs(A).sum(axis=1)).ravel() - np.abs(d)
    margin = float((d - off).min())
    assert margin > 0
    r = np.linalg.norm(s.b[0] - A @ x)
    ro = np.linalg.norm(s.b[0] - A @ xo)
    err = np.linalg.norm(x - xo)
    assert err <= (r + ro) / margin, (err, r, ro, margin)
    print(f"max |x - x_oracle| / max |x_oracle| = {np.abs(x - xo).max() / np.abs(xo).max():.3e}")
