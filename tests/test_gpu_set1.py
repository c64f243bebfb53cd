"""GPU: the Set-1 stand-in cubes (Q1 finite elements, 33^3 and 65^3 nodes)
solved with the paper's stop test (absolute infinity norm below 1e-8) under
each splitting, against the oracle and the iteration counts the paper prints."""
import numpy as np
import pytest

from conftest import read_golden
from gpu_util import B, get_x, make, need_gpu, rel_inf
from oracle import ref
from paper_2112_02377_amd import workloads as W

pytestmark = pytest.mark.gpu

_CACHE = {}


def cube(N):
    if N not in _CACHE:
        s = W.fe_q1_cube(N)
        st, xo, ko, rro = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-8, 100000, ref.NORM_INF_ABS, threads=8)
        assert st == ref.OK
        _CACHE[N] = (s, xo, ko, rro)
    return _CACHE[N]


def paper_iters(N):
    return {int(r[1]): int(r[6]) for r in read_golden("set1_cubes.txt")["CUBE"]}[N]


@pytest.mark.parametrize("N,mode,P,sub", [(33, 1, 8, None), (33, 2, 8, None), (33, 3, 8, (2, 2, 2)),
                                          (65, 1, 64, None), (65, 2, 64, None), (65, 3, 64, (4, 4, 4))])
def test_cube_solve_matches_oracle_and_paper_count(N, mode, P, sub):
    need_gpu()
    b = B()
    s, xo, ko, rro = cube(N)
    h = make(s, mode, P, sub)
    st, sw, rr = b.jac_solve(h, 1e-8, 100000, b.JAC_NORM_INF_ABS)
    assert st == b.JAC_OK
    assert int(sw[0]) == ko
    assert int(sw[0]) + 1 == paper_iters(N)
    x = get_x(h, s.n)[0]
    assert rel_inf(x, xo) <= 1e-10
    # the reported norm is the returned iterate's absolute residual
    assert rr[0] == pytest.approx(np.abs(s.b[0] - s.scipy() @ x).max(), rel=1e-9)
    assert rr[0] < 1e-8
    b.jac_destroy(h)
