"""GPU: parity at the full sizes the bench times.

The 128^3 7-point Laplacian (n = 2,097,152, b = A x* as in the bench), 64
parts under each split, the bench's default tile shape and loop:

* one sweep from the device's own state x_k, every row of x_{k+1} against
  the oracle's sweep from the same x_k: the per-sweep bar, 1e-12 relative;
* 2000 sweeps from x_0 = 0 against the oracle's 2000 sweeps.  The two sum
  each row in a different rounding (fused multiply-add on the device, and the
  substructured order permutes columns), so they drift apart by at most the
  per-sweep rounding summed over the sweeps: a row of m = 7 entries differs
  by at most about (m + 2) eps (|b_i| + sum_j |a_ij x_j|) / a_ii + eps |x_i|
  per sweep, under 40 eps max(1, max|x|) here (|b_i| <= 12, |x| ~ 1), and
  the Jacobi matrix has infinity norm 1, so after K sweeps the bound is
  K * 50 eps max(1, max|x|);
* the 192^3 control, whose band reaches past 16-bit row offsets (a shift
  table, or 32-bit columns without tables), a few sweeps against the oracle
  under the same bound;
* the 96^3 27-point FE-like system of the refinement comparison: FP64 and
  FP32-inner solves to 1e-10 against the oracle's FP64 solve;
* the 256-system, 4-right-hand-side batch of the batched comparison: every
  column bit-identical to its system solved alone and its FP64 residual
  recomputed on the host; a seeded subset of 16 systems plus the smallest and
  the largest against the oracle column by column (stop sweep exact, iterate
  within 1e-10)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import scipy.sparse as sp

from gpu_util import B, get_x, make, need_gpu, rel_inf, sweep, torch
from oracle import partition as OP
from oracle import ref
from paper_2112_02377_amd import workloads as W

pytestmark = pytest.mark.gpu

EPS = np.finfo(np.float64).eps
MODES = [(1, 64, None), (2, 64, None), (3, 64, (8, 8, 8))]
_REF = {}


@pytest.fixture(scope="module")
def big():
    return W.laplace7(128, workload=2)


def ref_sweeps(s, K):
    if K not in _REF:
        _REF[K] = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], K, threads=16)
    return _REF[K]


@pytest.mark.parametrize("mode,P,sub", MODES)
def test_one_sweep_from_device_state_every_row(big, mode, P, sub):
    need_gpu()
    b = B()
    s = big
    h = make(s, mode, P, sub)
    sweep(h, 37)
    xk = get_x(h, s.n)[0]
    hist = sweep(h, 1)[:, 0]
    xk1 = get_x(h, s.n)[0]
    st, xr, hr = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], 1, x0=xk, threads=16)
    assert st == ref.OK
    scale = max(np.abs(xk1).max(), 1.0)
    assert np.abs(xk1 - xr).max() <= 1e-12 * scale
    assert abs(hist[0] - hr[0]) <= 1e-12 * hr[0]
    # the recorded norm is that of b - A x_k
    r = np.linalg.norm(s.b[0] - s.scipy() @ xk)
    assert abs(hist[0] - r) <= 1e-12 * r
    b.jac_destroy(h)


@pytest.mark.parametrize("mode,P,sub", MODES)
def test_bench_sweeps_against_the_oracle(big, mode, P, sub):
    need_gpu()
    b = B()
    s = big
    K = 2000
    _, xr, hr = ref_sweeps(s, K)
    h = make(s, mode, P, sub)
    hist = sweep(h, K)[:, 0]
    x = get_x(h, s.n)[0]
    bound = K * 50 * EPS * max(1.0, np.abs(xr).max())
    assert np.abs(x - xr).max() <= bound
    # norms: b - A x differs by at most ||A||_inf * bound per row
    rn = np.sqrt(s.n) * 12 * bound
    assert np.all(np.abs(hist - hr) <= 1e-12 * hr + rn)
    b.jac_destroy(h)


def test_192_control_shift_table_and_32_bit_columns():
    # the band reaches past 16-bit row offsets: a shift table by default, 32-bit
    # columns without tables; both bit-identical and against the oracle
    need_gpu()
    b = B()
    s = W.laplace7(192, workload=2)
    K = 6
    out = []
    for tab, fmt, cb in ((1, 3, 0), (0, 0, 4)):
        h = make(s, 1, 64, opts={b.JAC_OPT_SHIFT_TABLES: tab})
        info = b.jac_get_info(h)
        assert info["col_format"] == fmt and info["col_bytes"] == cb
        assert info["n"] == 7077888 and info["nnz"] == 49324032
        out.append((sweep(h, K)[:, 0], get_x(h, s.n)[0]))
        b.jac_destroy(h)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    hist, x = out[0]
    _, xr, hr = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], K, threads=16)
    bound = K * 50 * EPS * max(1.0, np.abs(xr).max())
    assert np.abs(x - xr).max() <= bound
    assert np.all(np.abs(hist - hr) <= 1e-12 * hr + np.sqrt(s.n) * 12 * bound)


def test_fe27_96_fp64_and_fp32_refinement_at_full_size():
    # FP64: the oracle's stop sweep and iterate.  FP32 inner sweeps: the FP64
    # residual of the returned x (recomputed here) meets the tolerance, and x
    # lies within 1e-9 of the oracle's solution (both residuals are below
    # 1e-10 ||b|| and ||A^-1|| is small for a 1.05-dominant matrix).
    need_gpu()
    b = B()
    s = W.fe27(96, workload=3)
    h = make(s, 1, 64)
    st, sw, rr = b.jac_solve(h, 1e-10, 100000)
    x64 = get_x(h, s.n)[0]
    sto, xo, ko, rro = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-10, 100000, threads=16)
    assert st == b.JAC_OK and sto == ref.OK and int(sw[0]) == ko
    assert rel_inf(x64, xo) <= 1e-10
    b.jac_set_x(h, None)
    st, sw, rr = b.jac_solve(h, 1e-10, 100000, b.JAC_NORM_L2_REL, b.JAC_FP32_REFINE)
    x = get_x(h, s.n)[0]
    b.jac_destroy(h)
    assert st == b.JAC_OK
    A = sp.csr_matrix((s.vals, s.col_idx, s.row_ptr), shape=(s.n, s.n))
    assert np.linalg.norm(s.b[0] - A @ x) / np.linalg.norm(s.b[0]) <= 1e-10 * 1.001
    assert np.abs(x - xo).max() / np.abs(xo).max() <= 1e-9


def batch_subset(sizes):
    """The seeded 16-system subset the CPU baseline also times, plus the
    smallest and the largest system."""
    pick = set(np.random.default_rng(2112).choice(256, 16, replace=False).tolist())
    return sorted(pick | {int(sizes.argmin()), int(sizes.argmax())})


def test_full_batch_against_separate_solves_and_oracle():
    # the 256 uneven diffusion systems (edges U[16,64]) x 4 right-hand sides
    need_gpu()
    b = B()
    systems = W.diffusion_batch()
    assert len(systems) == 256 and all(s.nrhs == 4 for s in systems)
    hs = [make(s, 1, 1) for s in systems]
    st, sw, rr = b.jac_solve_batched(hs, 1e-8, 100000)
    assert st == b.JAC_OK
    xb = [get_x(h, s.n, 4) for h, s in zip(hs, systems)]
    for h in hs:
        b.jac_destroy(h)
    # every column: bit-identical to its system solved alone, and its FP64
    # residual (recomputed here) passes the test it stopped on
    for si, s in enumerate(systems):
        h = make(s, 1, 1)
        st1, sw1, rr1 = b.jac_solve(h, 1e-8, 100000)
        x1 = get_x(h, s.n, 4)
        b.jac_destroy(h)
        assert np.array_equal(sw[si, :4], sw1) and np.array_equal(xb[si], x1), si
        A = s.scipy()
        for c in range(4):
            res = np.linalg.norm(s.b[c] - A @ xb[si][c]) / np.linalg.norm(s.b[c])
            assert res <= 1e-8 * (1 + 1e-6) and abs(res - rr[si, c]) <= 1e-6 * res, (si, c)
    # a seeded subset against the oracle, column by column
    sizes = np.array([s.n for s in systems])
    jobs = [(si, c) for si in batch_subset(sizes) for c in range(4)]

    def oracle(job):
        si, c = job
        s = systems[si]
        return ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[c], 1e-8, 100000)

    with ThreadPoolExecutor(16) as ex:
        out = list(ex.map(oracle, jobs))
    for (si, c), (sto, xo, ko, rro) in zip(jobs, out):
        assert sto == ref.OK and sw[si, c] == ko, (si, c)
        assert rel_inf(xb[si][c], xo) <= 1e-10, (si, c)


@pytest.mark.parametrize("mode,sub", [(1, None), (2, None), (3, (8, 8, 8)), (3, (4, 4, 4))])
def test_split_arrays_bit_exact_at_full_size(big, mode, sub):
    # 128^3, 64 parts: order, bounds, receive lists and send lists of the
    # library's split equal the oracle partitioner's, array for array
    need_gpu()
    b = B()
    s = big
    h = make(s, mode, 64, sub)
    got = b.jac_get_partition(h)
    sl = b.jac_get_send_lists(h)
    b.jac_destroy(h)
    exp = OP.partition(s.row_ptr, s.col_idx, mode, 64, grid=(128, 128, 128), sub_grid=sub)
    for key in ("perm", "bounds", "recv_ptr", "recv_idx"):
        assert np.array_equal(got[key], exp[key]), key
    sptr, sdest, sidx = OP.send_lists(exp["recv_ptr"], exp["recv_idx"], exp["owner"], 64)
    assert np.array_equal(sl["send_ptr"], sptr)
    assert np.array_equal(sl["send_dest"], sdest) and np.array_equal(sl["send_idx"], sidx)
    halo = {1: 0, 2: 2064384, 3: 458752 if sub == (8, 8, 8) else 294912}[mode]
    assert len(got["recv_idx"]) == halo


def test_adjoint_at_full_size_against_full_storage_oracle():
    """The differentiation workload at its full size: 64^3 diffusion, K = 400
    sweeps, reverse segments of 20.  dL/db and dL/dvals from jac_adjoint
    against the oracle's full-storage reverse sweep, element by element, and
    dL/dtheta from the autograd Function against the oracle's chain rule."""
    need_gpu()
    from paper_2112_02377_amd.autograd import JacobiK, diffusion_values
    b = B()
    s = W.diffusion_adjoint(64)
    K, c = 400, 20
    t = s.extra["x_target"]
    st, xo, _ = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], K, threads=16)
    g = xo - t
    sto, gbo, gvo, xk = ref.adjoint(s.row_ptr, s.col_idx, s.vals, s.b[0], K, g)
    assert sto == ref.OK
    h = make(s, 1, 1)
    gb = torch.empty(s.n, dtype=torch.float64, device="cuda")
    gv = torch.empty(s.nnz, dtype=torch.float64, device="cuda")
    b.jac_adjoint(h, K, c, torch.from_numpy(g).cuda(), gb, gv)
    torch.cuda.synchronize()
    gb, gv = gb.cpu().numpy(), gv.cpu().numpy()
    assert np.abs(gb - gbo).max() <= 1e-10 * np.abs(gbo).max()
    assert np.abs(gv - gvo).max() <= 1e-10 * np.abs(gvo).max()
    assert rel_inf(get_x(h, s.n)[0], xk) <= 1e-12
    # through torch: theta -> values -> K sweeps -> loss
    theta = torch.from_numpy(s.extra["theta"]).cuda().requires_grad_(True)
    vals = diffusion_values(theta, s.grid, s.row_ptr, s.extra["slot"])
    x = JacobiK.apply(vals, torch.from_numpy(s.b[0]).cuda(), h, K, c)
    (0.5 * ((x - torch.from_numpy(t).cuda()) ** 2).sum()).backward()
    gth = theta.grad.cpu().numpy()
    gth_o = ref.theta_grad(s.extra["theta"], s.grid, s.row_ptr, s.extra["slot"], gvo)
    assert np.abs(gth - gth_o).max() <= 1e-10 * np.abs(gth_o).max()
    b.jac_destroy(h)
