"""GPU: many uneven systems with several right-hand sides solved together
(one launch per global sweep, or one persistent launch), against separate
solves and the CPU oracle."""
import numpy as np
import pytest

from gpu_util import B, get_x, make, need_gpu, rel_inf, torch
from oracle import ref
from paper_2112_02377_amd import workloads as W

pytestmark = pytest.mark.gpu


def small_batch(nsys=12, lo=5, hi=14):
    return W.diffusion_batch(nsys, workload=4, lo=lo, hi=hi)


@pytest.mark.parametrize("loop", [0, 1])
def test_batched_equals_separate_solves_and_oracle(loop):
    # loop 0: one launch per global sweep over the running systems; 1: one
    # persistent launch
    need_gpu()
    b = B()
    systems = small_batch()
    hs = [make(s, 1, 1, opts={b.JAC_OPT_LOOP: loop}) for s in systems]
    st, sw, rr = b.jac_solve_batched(hs, 1e-8, 200000)
    assert st == b.JAC_OK
    xb = [get_x(h, s.n, 4) for h, s in zip(hs, systems)]
    for h in hs:
        b.jac_destroy(h)
    for si, s in enumerate(systems):
        # the same system alone through jac_solve: identical arithmetic, identical result
        h = make(s, 1, 1)
        st1, sw1, rr1 = b.jac_solve(h, 1e-8, 200000)
        x1 = get_x(h, s.n, 4)
        b.jac_destroy(h)
        assert np.array_equal(sw[si], sw1) and np.array_equal(xb[si], x1), si
        for c in range(4):
            sto, xo, ko, rro = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[c], 1e-8, 200000)
            assert sw[si, c] == ko, (si, c)
            assert rel_inf(xb[si][c], xo) <= 1e-10
            assert abs(rr[si, c] - rro) <= 1e-6 * rro


@pytest.mark.parametrize("mode", [2, 3])
def test_batched_staged_modes_and_persistent_single_system(mode):
    need_gpu()
    b = B()
    systems = small_batch(6, 6, 12)
    hs = [make(s, mode, 2, (2, 1, 1) if mode == 3 else None) for s in systems]
    st, sw, rr = b.jac_solve_batched(hs, 1e-9, 200000)
    for h, s, k in zip(hs, systems, sw):
        x = get_x(h, s.n, 4)
        for c in range(4):
            sto, xo, ko, _ = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[c], 1e-9, 200000)
            assert k[c] == ko and rel_inf(x[c], xo) <= 1e-10
        b.jac_destroy(h)


def test_persistent_loop_matches_per_launch_for_fixed_sweeps():
    need_gpu()
    b = B()
    s = W.laplace7(16, workload=1)
    out = []
    for loop in (0, 1):
        h = make(s, 2, 4, opts={b.JAC_OPT_LOOP: loop})
        hist = torch.zeros(250, dtype=torch.float64, device="cuda")
        b.jac_sweep(h, 250, hist)
        out.append((get_x(h, s.n)[0], hist.cpu().numpy()))
        b.jac_destroy(h)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("loop", [0, 1])
def test_batched_maxit_exhausted_equals_separate_solves(loop):
    # every column runs out of sweeps: statuses, counts, norms and iterates
    # equal those of separate solves with the same cap
    need_gpu()
    b = B()
    systems = small_batch(5, 8, 12)
    hs = [make(s, 1, 1, opts={b.JAC_OPT_LOOP: loop}) for s in systems]
    st, sw, rr = b.jac_solve_batched(hs, 1e-14, 150)
    assert st == b.JAC_NOT_CONVERGED
    for si, (h, s) in enumerate(zip(hs, systems)):
        xb = get_x(h, s.n, 4)
        h1 = make(s, 1, 1)
        st1, sw1, rr1 = b.jac_solve(h1, 1e-14, 150)
        assert st1 == b.JAC_NOT_CONVERGED
        assert np.array_equal(sw[si], sw1) and np.array_equal(rr[si], rr1)
        assert np.array_equal(xb, get_x(h1, s.n, 4))
        b.jac_destroy(h1)
        b.jac_destroy(h)
