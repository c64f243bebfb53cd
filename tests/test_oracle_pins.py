"""Pins of the CPU oracle's sweep / solve against facts the paper and the
mathematics fix (closed forms, worked examples, direct solves, invariants).
CPU only."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from conftest import read_golden
from oracle import ref
from paper_2112_02377_amd import workloads as W


def fig_csr():
    g = read_golden("fig_csr.txt")
    AA = np.array([float(t) for t in g["AA"][0]])
    JA = np.array([int(t) for t in g["JA"][0]]) - 1
    IA = np.array([int(t) for t in g["IA"][0]]) - 1
    dense = np.array([[float(t) for t in row] for row in g["DENSE"]])
    return IA.astype(np.int32), JA.astype(np.int32), AA, dense


def test_fig_csr_arrays_encode_the_drawn_matrix():
    # section 4.1: AA/JA/IA of the 5x5 example are the drawn matrix
    IA, JA, AA, dense = fig_csr()
    A = sp.csr_matrix((AA, JA, IA), shape=(5, 5)).toarray()
    assert np.array_equal(A, dense)
    assert ref.check_csr(IA, JA, AA) == ref.OK


def test_first_sweep_is_one_rounding_of_invD_times_b():
    # correction form from x0 = 0: x_1 = D^{-1} b with D^{-1} formed once
    s = W.laplace7(6, workload=1)
    st, x1, _ = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], 1)
    assert st == ref.OK
    assert np.array_equal(x1, np.float64(1.0 / 6.0) * s.b[0])
    d = W.diffusion_adjoint(5)
    st, x1, _ = ref.sweeps(d.row_ptr, d.col_idx, d.vals, d.b[0], 1)
    diag = d.scipy().diagonal()
    assert np.array_equal(x1, (1.0 / diag) * d.b[0])


def test_laplace_residual_contracts_by_cos_pi_h():
    # section 3 error bound with rho(T) = cos(pi/(N+1)) for the 7-point
    # Laplacian (T = I - A/6 is symmetric, so ||r_{k+1}|| <= rho ||r_k||)
    N = 20
    s = W.laplace7(N)
    rho = math.cos(math.pi / (N + 1))
    K = 1700
    st, _, hist = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], K)
    assert st == ref.OK
    # rounding of the computed residual adds about eps * ||A|| ||x|| ~ eps ||b||
    slack = 1e-15 * np.linalg.norm(s.b[0])
    assert np.all(hist[1:] <= rho * hist[:-1] + slack)
    for k in (1000, 1300, 1600):
        observed = (hist[k] / hist[k - 100]) ** (1.0 / 100)
        assert abs(observed - rho) <= 1e-4 * rho


def test_manufactured_solution_error_bound():
    # ||x_k - x*||_2 <= ||r_k||_2 / lambda_min(A), lambda_min = 6 (1 - cos(pi/(N+1)))
    N = 20
    s = W.laplace7(N)
    lam = 6.0 * (1.0 - math.cos(math.pi / (N + 1)))
    xstar = s.extra["xstar"]
    for K in (1, 10, 100, 500, 1000):
        st, xk, hist = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], K + 1)
        _, xK, _ = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], K)
        err = np.linalg.norm(xK - xstar)
        assert err <= hist[K] / lam * (1 + 1e-10) + 1e-13


@pytest.mark.parametrize("N", [2, 3, 4, 5, 6])
def test_small_grids_agree_with_dense_direct_solve(N):
    for s in (W.laplace7(N, workload=1), W.diffusion_adjoint(N)):
        A = s.scipy().toarray()
        xd = np.linalg.solve(A, s.b[0])
        st, x, k, rel = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-14, 200000)
        assert st == ref.OK
        lam = np.linalg.eigvalsh(A).min()
        bound = rel * np.linalg.norm(s.b[0]) / lam
        assert np.linalg.norm(x - xd) <= bound * 1.01 + 1e-13


def test_fig_csr_matrix_converges_with_rate_0_07_cubed_root():
    # theorem of section 3: converges iff rho(T) < 1; the example is not
    # diagonally dominant (row 1) yet T has the 3-cycle 2.8 * -0.125 * -0.2 =
    # 0.07, so T^(k+3) = 0.07 T^k for k >= 2 and e_{k+3} = 0.07 e_k.
    IA, JA, AA, dense = fig_csr()
    assert abs(dense[0, 0]) < abs(dense[0, 1])           # not dominant
    D = np.diag(np.diag(dense))
    T = np.eye(5) - np.linalg.solve(D, dense)
    assert abs(max(abs(np.linalg.eigvals(T))) - 0.07 ** (1 / 3)) < 1e-12
    rng = np.random.default_rng(7)
    xstar = rng.uniform(-1, 1, 5)
    b = dense @ xstar
    xex = np.linalg.solve(dense, b)
    errs = []
    for K in range(12):
        st, xk, _ = ref.sweeps(IA, JA, AA, b, K)
        errs.append(xk - xex)
    e0 = np.linalg.norm(errs[0])
    for k in range(3, 9):
        assert np.linalg.norm(errs[k + 3] - 0.07 * errs[k]) <= 1e-13 * e0
    st, x, sweeps, rel = ref.solve(IA, JA, AA, b, 1e-13, 1000)
    assert st == ref.OK and np.allclose(x, xex, rtol=0, atol=1e-12)


def test_dominant_27pt_error_contracts_by_1_05_in_inf_norm():
    # ||T||_inf = 1/1.05 by construction, so ||e_{k+1}||_inf <= ||e_k||_inf / 1.05
    s = W.fe27(10, workload=3)
    A = s.scipy().toarray()
    xex = np.linalg.solve(A, s.b[0])
    T = np.eye(s.n) - A / np.diag(A)[:, None]
    assert np.abs(T).sum(axis=1).max() <= 1 / 1.05 * (1 + 1e-14)
    prev = None
    for K in range(0, 40):
        st, xk, _ = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], K)
        e = np.abs(xk - xex).max()
        if prev is not None:
            assert e <= prev / 1.05 * (1 + 1e-12) + 1e-14
        prev = e


def test_stop_rules_and_error_paths():
    s = W.laplace7(5, workload=1)
    b = s.b[0]
    # maxit = 0: the residual of x_0 is evaluated, nothing is updated
    st, x, k, rel = ref.solve(s.row_ptr, s.col_idx, s.vals, b, 1e-30, 0)
    assert st == ref.NOT_CONVERGED and k == 0 and np.all(x == 0)
    assert rel == pytest.approx(1.0, rel=0, abs=0)
    # maxit exhausted: returns x_maxit and its relative residual
    st, x, k, rel = ref.solve(s.row_ptr, s.col_idx, s.vals, b, 1e-30, 7)
    _, _, hist = ref.sweeps(s.row_ptr, s.col_idx, s.vals, b, 8)
    _, x7, _ = ref.sweeps(s.row_ptr, s.col_idx, s.vals, b, 7)
    assert st == ref.NOT_CONVERGED and k == 7 and np.array_equal(x, x7)
    assert rel == pytest.approx(hist[7] / np.linalg.norm(b), rel=1e-14)
    # b = 0: the relative test falls back to absolute and stops at once
    st, x, k, rel = ref.solve(s.row_ptr, s.col_idx, s.vals, np.zeros_like(b), 1e-8, 100)
    assert st == ref.OK and k == 0 and rel == 0.0
    # the stop sweep is the first k whose residual passes (<=) the test
    st, x, k, rel = ref.solve(s.row_ptr, s.col_idx, s.vals, b, 1e-6, 10000)
    _, _, hist = ref.sweeps(s.row_ptr, s.col_idx, s.vals, b, k + 1)
    nb = np.linalg.norm(b)
    assert st == ref.OK and hist[k] <= 1e-6 * nb and hist[k - 1] > 1e-6 * nb
    # infinity-norm absolute mode: stop at max|r_i| <= tol
    st, x, k, rel = ref.solve(s.row_ptr, s.col_idx, s.vals, b, 1e-8, 10000, ref.NORM_INF_ABS)
    r = b - s.scipy() @ x
    assert st == ref.OK and np.abs(r).max() == rel and rel <= 1e-8
    # divergence: [[1,2],[2,1]] has rho(T) = 2
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([0, 1, 0, 1], np.int32)
    st, *_ = ref.solve(rp, ci, np.array([1.0, 2.0, 2.0, 1.0]), np.array([1.0, 1.0]), 1e-8, 100000)
    assert st == ref.E_DIVERGED
    # zero or missing diagonal, malformed structure
    assert ref.check_csr(rp, ci, np.array([0.0, 2.0, 2.0, 1.0])) == ref.E_ZERO_DIAG
    assert ref.check_csr(np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.ones(2)) == ref.E_ZERO_DIAG
    assert ref.check_csr(rp, np.array([1, 0, 0, 1], np.int32), np.ones(4)) == ref.E_INVALID
    assert ref.check_csr(rp, np.array([0, 2, 0, 1], np.int32), np.ones(4)) == ref.E_INVALID
    assert ref.check_csr(np.array([0, 3, 2], np.int32), ci, np.ones(4)) == ref.E_INVALID


def test_thread_count_does_not_change_results():
    s = W.laplace7(20)
    _, x1, h1 = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], 50, threads=1)
    _, x4, h4 = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], 50, threads=4)
    assert np.array_equal(x1, x4) and np.array_equal(h1, h4)


def test_sweep_rows_matches_full_sweep():
    s = W.laplace7(8, workload=1)
    _, x5, _ = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], 5)
    _, x6, _ = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], 6)
    rows = np.array([0, 7, 63, 100, 511])
    st, out, _ = ref.sweep_rows(s.row_ptr, s.col_idx, s.vals, s.b[0], x5, rows)
    assert st == ref.OK and np.array_equal(out, x6[rows])


def test_batched_reference_against_an_independent_jacobi():
    # each (system, right-hand side) column: the sweep count is the first k
    # whose residual meets the relative test, with x_k and the residuals
    # recomputed by a separate numpy/scipy Jacobi iteration
    import scipy.sparse as sp
    systems = W.diffusion_batch(3, workload=4, lo=4, hi=7)
    out = ref.batched_solve(systems, 1e-8, 100000)
    assert len(out) == 3
    for s, res in zip(systems, out):
        A = sp.csr_matrix((s.vals, s.col_idx, s.row_ptr), shape=(s.n, s.n))
        d = A.diagonal()
        assert len(res) == s.b.shape[0] == 4
        for c, (st, x, k, rel) in enumerate(res):
            b = s.b[c]
            nb = np.linalg.norm(b)
            xs, prev = np.zeros(s.n), None
            for _ in range(k):
                prev = xs
                xs = xs + (b - A @ xs) / d
            assert st == ref.OK
            assert np.abs(x - xs).max() <= 1e-12 * max(1.0, np.abs(xs).max())
            r_k = np.linalg.norm(b - A @ xs) / nb
            assert r_k <= 1e-8 * (1 + 1e-9) and abs(rel - r_k) <= 1e-6 * r_k
            assert np.linalg.norm(b - A @ prev) / nb > 1e-8 * (1 - 1e-9)
