"""CPU: the Set-1 stand-in (Q1 finite-element Laplacian on the unit cube) and
the oracle's stop rule against the iteration counts the paper prints.

The generator is pinned to an independent tensor-product assembly and to the
sizes of the paper's matrix table; the oracle's absolute infinity-norm solve
is pinned to the paper's p = 1 iteration counts (746 and 2,216), which count
the final iterate x_{k+1} of the test ||D (x_{k+1} - x_k)||_inf < 1e-8, i.e.
||r_k||_inf < 1e-8 with k = the oracle's sweep count."""
import numpy as np
import pytest
import scipy.sparse as sp

from conftest import read_golden
from oracle import ref
from paper_2112_02377_amd import workloads as W


def cubes():
    return [dict(name=r[0], N=int(r[1]), n=int(r[2]), nnz=int(r[3]), band=int(r[4]), maxrow=int(r[5]),
                 iters=int(r[6])) for r in read_golden("set1_cubes.txt")["CUBE"]]


def kron_assembly(N):
    """Q1 stiffness and consistent load from 1-D element matrices by Kronecker
    products (K = K1 x M1 x M1 + M1 x K1 x M1 + M1 x M1 x K1, M = M1 x M1 x M1),
    then Dirichlet elimination: boundary rows -> identity with b = 0,
    boundary columns dropped from interior rows."""
    h = 1.0 / (N - 1)
    e = np.ones(N)
    K1 = sp.diags([-e[1:], 2 * e, -e[1:]], [-1, 0, 1]) / h
    M1 = sp.diags([e[1:], 4 * e, e[1:]], [-1, 0, 1]) * (h / 6)
    K = (sp.kron(sp.kron(M1, M1), K1) + sp.kron(sp.kron(M1, K1), M1) + sp.kron(sp.kron(K1, M1), M1)).tocoo()
    M = sp.kron(sp.kron(M1, M1), M1).tocsr()
    r = np.arange(N ** 3)
    i, j, k = r % N, (r // N) % N, r // (N * N)
    bnd = (i == 0) | (i == N - 1) | (j == 0) | (j == N - 1) | (k == 0) | (k == N - 1)
    f = np.cos(i * h + j * h)
    b = M @ f
    b[bnd] = 0.0
    keep = ~bnd[K.row] & ~bnd[K.col]
    rows = np.concatenate([K.row[keep], r[bnd]])
    cols = np.concatenate([K.col[keep], r[bnd]])
    vals = np.concatenate([K.data[keep], np.ones(int(bnd.sum()))])
    return sp.csr_matrix((vals, (rows, cols)), shape=(N ** 3, N ** 3)), b


@pytest.mark.parametrize("N", [4, 7, 33])
def test_generator_equals_tensor_product_assembly(N):
    s = W.fe_q1_cube(N)
    assert ref.check_csr(s.row_ptr, s.col_idx, s.vals) == 0          # ascending, unique, diagonal present
    A = s.scipy()
    Ak, bk = kron_assembly(N)
    h = 1.0 / (N - 1)
    assert abs(A - Ak).max() <= 1e-15 * h
    np.testing.assert_allclose(s.b[0], bk, rtol=1e-13, atol=1e-18)
    # every entry the tensor-product form stores is in the generator's pattern
    pat = sp.csr_matrix((np.ones(s.nnz), s.col_idx, s.row_ptr), shape=A.shape)
    Ak.eliminate_zeros()
    assert pat.multiply(abs(Ak) > 0).nnz == Ak.nnz


@pytest.mark.parametrize("c", cubes(), ids=lambda c: c["name"])
def test_sizes_against_the_matrix_table(c):
    N = c["N"]
    s = W.fe_q1_cube(N)
    assert s.n == c["n"]
    rp = s.row_ptr.astype(np.int64)
    assert int(np.diff(rp).max()) == c["maxrow"]
    rows = np.repeat(np.arange(s.n), np.diff(rp))
    assert int(np.abs(s.col_idx - rows).max()) == c["band"] == N * N + N + 1
    # interior rows: the full 27-point pattern among interior nodes; boundary
    # rows: the diagonal alone
    m = N - 2
    assert s.nnz == (3 * m - 2) ** 3 + (N ** 3 - m ** 3)
    # the paper's files hold slightly fewer stored entries (50 and 614 of
    # 0.76 M and 6.6 M): entries whose assembled value came out as an exact
    # zero are the only candidates, and the face couplings are exactly zero
    assert abs(s.nnz - c["nnz"]) <= 1e-3 * c["nnz"]
    face = np.zeros(s.nnz, dtype=bool)
    d = np.abs(s.col_idx - rows)
    face[(d == 1) | (d == N) | (d == N * N)] = True
    assert np.all(s.vals[face] == 0.0)
    assert s.nnz - int(face.sum()) < c["nnz"]


@pytest.mark.parametrize("c", cubes(), ids=lambda c: c["name"])
def test_oracle_iteration_count_is_the_papers(c):
    s = W.fe_q1_cube(c["N"])
    A = s.scipy()
    st, x, k, res = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-8, 100000, ref.NORM_INF_ABS, threads=8)
    assert st == ref.OK
    # the paper counts the iterate x_{k+1} computed before its test passes
    assert k + 1 == c["iters"]
    assert res == pytest.approx(np.abs(s.b[0] - A @ x).max(), rel=1e-12)
    assert res < 1e-8
    # first crossing: the previous iterate's residual had not passed
    _, xprev, _ = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], k - 1, history=False, threads=8)
    assert np.abs(s.b[0] - A @ xprev).max() >= 1e-8


def test_relative_two_norm_reading_does_not_give_the_papers_count():
    # the count singles out the absolute infinity-norm reading of the stop test
    c = cubes()[0]
    s = W.fe_q1_cube(c["N"])
    _, _, k, _ = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-8, 100000, ref.NORM_L2_REL, threads=8)
    assert abs((k + 1) - c["iters"]) > 50
