"""GPU: the weighted partitioners inside jac_partition (JAC_OPT_PARTITIONER).

The split the library builds is compared bit for bit with the oracle's
definitions given the same part or subdomain map (the graph partitioner's own
map comes from the host-only entry point, whose properties are pinned on the
CPU), and solves on the renumbered systems match the oracle's solve on the
original one."""
import numpy as np
import pytest

from gpu_util import B, get_x, make, need_gpu, rel_inf
from oracle import partition as OP
from oracle import ref
from paper_2112_02377_amd import workloads as W

pytestmark = pytest.mark.gpu

_SYS = {}


def system(name):
    if name not in _SYS:
        s = W.fe27(16, workload=3) if name == "fe27" else W.laplace7(18, workload=1)
        st, xo, ko, _ = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-8, 20000)
        _SYS[name] = (s, xo, ko)
    return _SYS[name]


CASES = [("fe27", 1, 1, 7, None, True), ("fe27", 2, 1, 7, None, True), ("fe27", 3, 1, 6, None, False),
         ("fe27", 1, 2, 8, None, True), ("fe27", 2, 2, 8, None, True), ("fe27", 3, 2, 4, (2, 2, 2), True),
         ("lap", 2, 2, 5, None, True), ("lap", 3, 2, 3, (3, 1, 1), False)]


@pytest.mark.parametrize("name,mode,partitioner,P,sub,grid", CASES)
def test_partitioner_split_is_bit_exact_and_solves_match(name, mode, partitioner, P, sub, grid):
    need_gpu()
    b = B()
    s, xo, ko = system(name)
    h = make(s, grid=grid, opts={b.JAC_OPT_PARTITIONER: partitioner})
    b.jac_partition(h, mode, P, sub)
    got = b.jac_get_partition(h)
    kw = {}
    if partitioner == 1:
        kw["weights"] = "nnz"
    elif mode == 3:
        S = int(np.prod(sub)) if sub else P
        kw["sub_map"] = b.jac_graph_partition(s.row_ptr, s.col_idx, S)
    else:
        kw["part_map"] = b.jac_graph_partition(s.row_ptr, s.col_idx, P)
    exp = OP.partition(s.row_ptr, s.col_idx, mode, P, grid=s.grid if grid else None, sub_grid=sub, **kw)
    for key in ("perm", "bounds", "recv_ptr", "recv_idx"):
        assert np.array_equal(got[key], exp[key]), key
    st, sw, rr = b.jac_solve(h, 1e-8, 20000)
    assert st == b.JAC_OK and int(sw[0]) == ko
    assert rel_inf(get_x(h, s.n)[0], xo) <= 1e-10
    b.jac_destroy(h)


def test_graph_parts_shrink_the_halo_at_full_size():
    # 128^3, 64 parts: the graph split's lists are close to the 4x4x4 block
    # optimum (294,912 entries) and far below the band rows' (2,064,384)
    need_gpu()
    b = B()
    s = W.laplace7(128)
    h = make(s, 2, 64)
    band = b.jac_get_info(h)["halo_entries"]
    b.jac_set_option(h, b.JAC_OPT_PARTITIONER, 2)
    b.jac_partition(h, 2, 64)
    graph = b.jac_get_info(h)["halo_entries"]
    assert band == 2064384
    assert 294912 <= graph <= 1.05 * 294912
    # a few sweeps on the renumbered system equal the oracle's on the original
    hist = torch_sweeps(h, 3)
    _, x3, ho = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], 3, threads=8)
    assert rel_inf(get_x(h, s.n)[0], x3) <= 1e-12
    assert np.allclose(hist, ho, rtol=1e-12, atol=0)
    b.jac_destroy(h)


def torch_sweeps(h, K):
    from gpu_util import sweep
    B().jac_set_x(h, None)
    return sweep(h, K)[:, 0]


def test_send_lists_reproduce_the_papers_tables():
    # the 10-row, three-band example of section 4.2.2: the library's receive
    # and send lists are the paper's receiving and sending dependency tables
    need_gpu()
    from test_oracle_partition import tab_dep
    b = B()
    rp, ci, P, recv, send = tab_dep()
    n = rp.shape[0] - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    vals = np.where(ci == rows, 10.0, -1.0)
    h = b.jac_create(n, rp, ci, vals, 1, np.ones(n))
    b.jac_partition(h, b.JAC_BANDROW_SP, P)
    got = b.jac_get_partition(h)
    bounds = got["bounds"]
    owner = np.searchsorted(bounds, np.arange(n), side="right") - 1
    r = {}
    for p in range(P):
        for i in got["recv_idx"][got["recv_ptr"][p]:got["recv_ptr"][p + 1]]:
            r.setdefault((p, int(owner[i])), []).append(int(i))
    assert r == recv
    sl = b.jac_get_send_lists(h)
    s = {}
    for q in range(P):
        for d, i in zip(sl["send_dest"][sl["send_ptr"][q]:sl["send_ptr"][q + 1]],
                        sl["send_idx"][sl["send_ptr"][q]:sl["send_ptr"][q + 1]]):
            s.setdefault((q, int(d)), []).append(int(i))
    assert s == send
    b.jac_destroy(h)


@pytest.mark.parametrize("mode,partitioner,P,sub", [(2, 0, 7, None), (3, 0, 8, (2, 2, 2)), (2, 2, 6, None),
                                                    (3, 2, 4, (3, 2, 1))])
def test_send_lists_are_the_transpose_of_the_receive_lists(mode, partitioner, P, sub):
    need_gpu()
    b = B()
    s = W.laplace7(14, workload=1)
    h = make(s, opts={b.JAC_OPT_PARTITIONER: partitioner})
    b.jac_partition(h, mode, P, sub)
    got = b.jac_get_partition(h)
    bounds = got["bounds"]
    if mode == 3:
        S = int(np.prod(sub))
        sub_int, sub_ifc, part_sub = bounds[:S + 1], bounds[S + 1:2 * S + 2], bounds[2 * S + 2:]
        owner = np.zeros(s.n, dtype=np.int64)
        for q in range(P):
            for t in range(part_sub[q], part_sub[q + 1]):
                owner[sub_int[t]:sub_int[t + 1]] = q
                owner[sub_ifc[t]:sub_ifc[t + 1]] = q
    else:
        owner = np.searchsorted(bounds, np.arange(s.n), side="right") - 1
    sptr, sdest, sidx = OP.send_lists(got["recv_ptr"], got["recv_idx"], owner, P)
    sl = b.jac_get_send_lists(h)
    assert np.array_equal(sl["send_ptr"], sptr)
    assert np.array_equal(sl["send_dest"], sdest) and np.array_equal(sl["send_idx"], sidx)
    assert sl["send_ptr"][-1] == got["recv_ptr"][-1]
    b.jac_destroy(h)
