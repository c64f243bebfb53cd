"""GPU: the matrix-load policy (JAC_OPT_CACHE).  Kept (temporal) and
streamed (nontemporal) loads differ only in cache hints, so every path gives
bit-identical results under both; the automatic choice follows the documented
byte rule."""
import numpy as np
import pytest

from gpu_util import B, get_x, make, need_gpu, rel_inf, sweep, torch
from oracle import ref
from paper_2112_02377_amd import workloads as W

pytestmark = pytest.mark.gpu

KEEP_BYTES = 256 << 20


def streamed(info):
    return info["ell_slots"] * (8 + info["col_bytes"]) + 24 * info["n"] * info["nrhs"]


@pytest.mark.parametrize("mode,P,sub", [(1, 3, None), (2, 4, None), (3, 4, (2, 2, 1))])
@pytest.mark.parametrize("nrhs", [1, 2])
def test_kept_and_streamed_loads_are_bit_identical(mode, P, sub, nrhs):
    need_gpu()
    b = B()
    s = W.laplace7(14, workload=1)
    if nrhs == 2:
        s = W.CSRSystem(s.row_ptr, s.col_idx, s.vals, np.vstack([s.b[0], -0.5 * s.b[0] + 1.0]), grid=s.grid)
    out = {}
    for pol in (b.CACHE_KEEP, b.CACHE_STREAM, b.CACHE_AUTO):
        h = make(s, mode, P, sub, opts={b.JAC_OPT_CACHE: pol})
        assert b.jac_get_option(h, b.JAC_OPT_CACHE) == pol
        info = b.jac_get_info(h)
        assert info["keep_matrix"] == (0 if pol == b.CACHE_STREAM else 1)
        hist = sweep(h, 17, nrhs)
        out[pol] = (get_x(h, s.n, nrhs), hist)
        b.jac_set_x(h, None)
        st, sw, rr = b.jac_solve(h, 1e-9, 5000)
        out[pol] += (get_x(h, s.n, nrhs), sw[:nrhs].copy())
        b.jac_destroy(h)
    for pol in (b.CACHE_STREAM, b.CACHE_AUTO):
        for u, v in zip(out[b.CACHE_KEEP], out[pol]):
            assert np.array_equal(u, v), pol
    _, xr, _ = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], 17)
    assert rel_inf(out[b.CACHE_KEEP][0][0], xr) <= 1e-12


def test_bad_policy_is_rejected():
    need_gpu()
    b = B()
    s = W.laplace7(6)
    h = make(s)
    for v in (-1, 3):
        with pytest.raises(b.JacError):
            b.jac_set_option(h, b.JAC_OPT_CACHE, v)
    assert b.jac_get_option(h, b.JAC_OPT_CACHE) == b.CACHE_AUTO
    b.jac_destroy(h)


def test_batched_and_adjoint_under_both_policies():
    need_gpu()
    b = B()
    systems = W.diffusion_batch(nsys=6, lo=8, hi=14, nrhs=4)
    res = {}
    for pol in (b.CACHE_KEEP, b.CACHE_STREAM):
        hs = [make(s, 1, 1) for s in systems]
        b.jac_set_option(hs[0], b.JAC_OPT_CACHE, pol)      # the batch follows its first handle
        st, sw, rr = b.jac_solve_batched(hs, 1e-8, 20000)
        res[pol] = (sw.copy(), [get_x(h, s.n, 4) for h, s in zip(hs, systems)])
        for h in hs:
            b.jac_destroy(h)
    assert np.array_equal(res[1][0], res[2][0])
    assert all(np.array_equal(u, v) for u, v in zip(res[1][1], res[2][1]))
    s = W.diffusion_adjoint(10)
    g = torch.from_numpy(np.ascontiguousarray(s.extra["x_target"])).cuda()
    grads = {}
    for pol in (b.CACHE_KEEP, b.CACHE_STREAM):
        h = make(s, 2, 3, opts={b.JAC_OPT_CACHE: pol})
        gb = torch.empty(s.n, dtype=torch.float64, device="cuda")
        gv = torch.empty(s.nnz, dtype=torch.float64, device="cuda")
        b.jac_adjoint(h, 40, 7, g, gb, gv)
        torch.cuda.synchronize()
        grads[pol] = (gb.cpu().numpy(), gv.cpu().numpy())
        b.jac_destroy(h)
    assert np.array_equal(grads[1][0], grads[2][0]) and np.array_equal(grads[1][1], grads[2][1])


def test_async_converges_under_both_policies():
    need_gpu()
    b = B()
    s = W.laplace7(12, workload=1)
    for pol in (b.CACHE_KEEP, b.CACHE_STREAM):
        h = make(s, 2, 4, opts={b.JAC_OPT_CACHE: pol})
        st, rounds, rr = b.jac_solve_async(h, 1e-8, 20000)
        assert st == b.JAC_OK and rr[0] <= 1e-8
        b.jac_destroy(h)


def test_automatic_choice_follows_the_byte_rule():
    # 128^3 (161 MiB per sweep with shift tables) keeps the matrix, 160^3
    # (312 MiB) streams it
    need_gpu()
    b = B()
    for N, keep in ((128, 1), (160, 0)):
        s = W.laplace7(N, workload=2)
        h = make(s, 1, 64)
        info = b.jac_get_info(h)
        assert info["keep_matrix"] == keep == int(streamed(info) <= KEEP_BYTES), N
        hist = sweep(h, 3)[:, 0]
        b.jac_destroy(h)
        _, _, hr = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], 3, threads=16)
        assert np.allclose(hist, hr, rtol=1e-12, atol=0), N
