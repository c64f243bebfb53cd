"""GPU: jac_sweep_noalloc, the allocation-free variant of jac_sweep, against
jac_sweep itself through the C ABI: two calls in a row on the same device
(the second on a smaller system, so the shared scratch array still holds the
first call's larger contents), each bit-identical to jac_sweep on an
identical handle (iterate and per-sweep residual norms), and the size limit
of the scratch array refused with JAC_E_INVALID."""
import numpy as np
import pytest

from gpu_util import B, get_x, make, need_gpu, torch
from paper_2112_02377_amd import workloads as W

pytestmark = pytest.mark.gpu


def run(h, K, nrhs, noalloc):
    b = B()
    hist = torch.full((K * nrhs,), -1.0, dtype=torch.float64, device="cuda")
    (b.jac_sweep_noalloc if noalloc else b.jac_sweep)(h, K, hist)
    torch.cuda.synchronize()
    return hist.cpu().numpy()


CASES = [
    # (grid edge, split, parts, subdomain grid, right-hand sides, sweeps)
    (40, 3, 8, (2, 2, 2), 1, 57),     # larger first: staged, many tiles
    (12, 2, 3, None, 2, 23),          # then smaller, two right-hand sides
]


def test_noalloc_matches_jac_sweep_on_two_calls_in_a_row():
    need_gpu()
    b = B()
    for N, mode, P, sub, nrhs, K in CASES:
        s = W.laplace7(N, workload=1)
        if nrhs > 1:
            rng = np.random.default_rng(N)
            s.b = np.stack([s.b[0]] + [rng.uniform(-1, 1, s.n) for _ in range(nrhs - 1)])
        out = []
        for noalloc in (False, True):
            h = make(s, mode, P, sub)
            x0 = torch.from_numpy(np.random.default_rng(7).uniform(-1, 1, s.n * nrhs)).cuda()
            b.jac_set_x(h, x0)
            hist = run(h, K, nrhs, noalloc)
            out.append((hist, get_x(h, s.n, nrhs)))
            b.jac_destroy(h)
        assert np.array_equal(out[0][0], out[1][0]), (N, "hist")
        assert np.array_equal(out[0][1], out[1][1]), (N, "x")
        assert np.all(out[1][0] > 0.0)


def test_noalloc_zero_sweeps_and_repeated_calls_on_one_handle():
    need_gpu()
    b = B()
    s = W.laplace7(16, workload=1)
    h1 = make(s, 1, 4)
    h2 = make(s, 1, 4)
    b.jac_sweep_noalloc(h1, 0)
    assert np.array_equal(get_x(h1, s.n), np.zeros((1, s.n)))
    # 30 sweeps as 3 x 10 no-allocation calls equal 30 jac_sweep sweeps
    for _ in range(3):
        b.jac_sweep_noalloc(h1, 10)
    b.jac_sweep(h2, 30)
    assert np.array_equal(get_x(h1, s.n), get_x(h2, s.n))
    b.jac_destroy(h1)
    b.jac_destroy(h2)


def test_noalloc_refuses_a_split_beyond_its_scratch():
    # 128^3 with 64-row tiles: 32,768 tiles; with 4 right-hand sides the
    # partials need 2 MiB, beyond the 1 MiB array; with 1 they fit (512 KiB)
    need_gpu()
    b = B()
    s = W.laplace7(128, workload=2)
    h = make(s, 1, 64, opts={b.JAC_OPT_TILE_ROWS: 64})
    assert b.jac_get_info(h)["ntiles"] == 32768
    b.jac_sweep_noalloc(h, 2)
    b.jac_destroy(h)
    rng = np.random.default_rng(3)
    s.b = np.stack([s.b[0]] + [rng.uniform(-1, 1, s.n) for _ in range(3)])
    h = make(s, 1, 64, opts={b.JAC_OPT_TILE_ROWS: 64})
    with pytest.raises(b.JacError) as e:
        b.jac_sweep_noalloc(h, 2)
    assert e.value.status == b.JAC_E_INVALID
    # the handle stays usable
    b.jac_sweep(h, 2)
    b.jac_destroy(h)
