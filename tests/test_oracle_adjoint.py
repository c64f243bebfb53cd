"""Pins of the oracle's reverse-mode derivative of K Jacobi sweeps. CPU only."""
import numpy as np
import scipy.sparse as sp

from oracle import ref
from paper_2112_02377_amd import workloads as W
from test_oracle_pins import fig_csr


def loss_and_x(rp, ci, vals, b, K, target):
    st, x, _ = ref.sweeps(rp, ci, vals, b, K, history=False)
    assert st == ref.OK
    return 0.5 * np.sum((x - target) ** 2), x


def transpose_csr(rp, ci, vals, n):
    At = sp.csr_matrix((vals, ci, rp), shape=(n, n)).T.tocsr()
    At.sort_indices()
    return At.indptr.astype(np.int32), At.indices.astype(np.int32), At.data


def test_db_equals_K_sweeps_on_the_transpose():
    # x_K = S_K b with S_K = sum_{j<K} T^j D^{-1}; so dL/db = S_K^T g, which is
    # K forward sweeps on A^T y = g from y = 0 (a different code path)
    IA, JA, AA, dense = fig_csr()
    rng = np.random.default_rng(3)
    b = rng.uniform(-1, 1, 5)
    g = rng.uniform(-1, 1, 5)
    K = 17
    st, gb, gv, xk = ref.adjoint(IA, JA, AA, b, K, g)
    assert st == ref.OK
    tp, ti, tv = transpose_csr(IA, JA, AA, 5)
    _, y, _ = ref.sweeps(tp, ti, tv, g, K)
    assert np.allclose(gb, y, rtol=1e-13, atol=1e-15 * np.abs(y).max())
    # symmetric diffusion matrix: the transpose is A itself
    s = W.diffusion_adjoint(6)
    g = rng.uniform(-1, 1, s.n)
    st, gb, gv, xk = ref.adjoint(s.row_ptr, s.col_idx, s.vals, s.b[0], 40, g)
    _, y, _ = ref.sweeps(s.row_ptr, s.col_idx, s.vals, g, 40)
    assert np.allclose(gb, y, rtol=1e-12, atol=1e-14 * np.abs(y).max())


def test_dot_product_identity():
    # <S_K v, w> = <v, S_K^T w>
    s = W.diffusion_adjoint(5)
    rng = np.random.default_rng(11)
    v = rng.uniform(-1, 1, s.n)
    w = rng.uniform(-1, 1, s.n)
    K = 25
    _, Sv, _ = ref.sweeps(s.row_ptr, s.col_idx, s.vals, v, K)
    _, STw, _, _ = ref.adjoint(s.row_ptr, s.col_idx, s.vals, v, K, w)
    lhs, rhs = Sv @ w, v @ STw
    assert abs(lhs - rhs) <= 1e-13 * max(abs(lhs), 1.0)


def _fd_vals(rp, ci, vals, b, K, target, h=1e-6):
    g = np.zeros_like(vals)
    for p in range(len(vals)):
        vp = vals.copy(); vp[p] += h
        vm = vals.copy(); vm[p] -= h
        _, xp = loss_and_x(rp, ci, vp, b, K, target)
        _, xm = loss_and_x(rp, ci, vm, b, K, target)
        # (L+ - L-)/2h written without the cancellation of L+ - L-
        g[p] = np.sum((xp - xm) * (xp + xm - 2 * target)) / (4 * h)
    return g


def test_dvals_match_central_differences_on_every_entry():
    # includes the diagonal entries, whose derivative also runs through 1/a_ii
    IA, JA, AA, dense = fig_csr()
    rng = np.random.default_rng(5)
    b = rng.uniform(-1, 1, 5)
    t = rng.uniform(-1, 1, 5)
    K = 9
    _, x = loss_and_x(IA, JA, AA, b, K, t)
    st, gb, gv, xk = ref.adjoint(IA, JA, AA, b, K, x - t)
    assert np.array_equal(xk, x)
    fd = _fd_vals(IA, JA, AA, b, K, t)
    assert np.allclose(gv, fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())
    s = W.diffusion_adjoint(3)
    t = s.extra["x_target"]
    _, x = loss_and_x(s.row_ptr, s.col_idx, s.vals, s.b[0], 12, t)
    st, gb, gv, _ = ref.adjoint(s.row_ptr, s.col_idx, s.vals, s.b[0], 12, x - t)
    fd = _fd_vals(s.row_ptr, s.col_idx, s.vals, s.b[0], 12, t)
    assert np.allclose(gv, fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max())


def test_dtheta_chain_rule_matches_central_differences():
    # dL/dtheta through the generator's own two-point-flux assembly
    nx, ny, nz = 4, 3, 3
    s0 = W.diffusion_adjoint(4)          # only for draws; rebuild on a 4x3x3 grid
    rng = np.random.default_rng(17)
    theta = 10.0 ** rng.uniform(-1, 1, nx * ny * nz)
    b = rng.uniform(-1, 1, nx * ny * nz)
    t = rng.uniform(-1, 1, nx * ny * nz)
    s = W.diffusion_system(nx, ny, nz, theta, b)
    K = 15
    _, x = loss_and_x(s.row_ptr, s.col_idx, s.vals, b, K, t)
    _, gb, gv, _ = ref.adjoint(s.row_ptr, s.col_idx, s.vals, b, K, x - t)
    gth = ref.theta_grad(theta, (nx, ny, nz), s.row_ptr, s.extra["slot"], gv)
    h = 1e-6
    for m in range(0, nx * ny * nz, 5):
        tp = theta.copy(); tp[m] += h
        tm = theta.copy(); tm[m] -= h
        vp = W.diffusion_values(tp, nx, ny, nz, s.row_ptr, s.extra["slot"])
        vm = W.diffusion_values(tm, nx, ny, nz, s.row_ptr, s.extra["slot"])
        _, xp = loss_and_x(s.row_ptr, s.col_idx, vp, b, K, t)
        _, xm = loss_and_x(s.row_ptr, s.col_idx, vm, b, K, t)
        fd = np.sum((xp - xm) * (xp + xm - 2 * t)) / (4 * h)
        assert abs(gth[m] - fd) <= 1e-6 * max(abs(fd), 1e-3 * np.abs(gth).max())
    assert s0.n == 64
