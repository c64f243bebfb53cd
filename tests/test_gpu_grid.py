"""GPU: workgroups of the per-sweep launch (JAC_OPT_GRID).

One workgroup per tile, or one resident round of workgroups each sweeping
consecutive tiles (in both cases each XCD sweeps its share of the tiles):
every tile writes the same values and the same norm partial either way,
and the stop decision sums the partials in tile order, so sweeps, norms and
iterates are bit-identical.  The 128^3 splits have
about twice as many tiles as the device holds workgroups at once, so the
resident round really gives each workgroup several tiles."""
import numpy as np
import pytest

from gpu_util import B, get_x, make, need_gpu, rel_inf, sweep
from oracle import ref
from paper_2112_02377_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lap128():
    return W.laplace7(128, workload=2)


@pytest.mark.parametrize("name,mode,P,sub,auto_resident", [("JB", 1, 64, None, True), ("JBO", 2, 64, None, True),
                                                            ("JSS", 3, 64, (8, 8, 8), False)])
def test_grid_choices_are_bit_identical(lap128, name, mode, P, sub, auto_resident):
    need_gpu()
    b = B()
    s = lap128
    K = 12
    out, grids = {}, {}
    for g in (1, 2, 0):
        h = make(s, mode, P, sub, opts={b.JAC_OPT_GRID: g})
        assert b.jac_get_option(h, b.JAC_OPT_GRID) == g
        ntiles = b.jac_get_info(h)["ntiles"]
        hist = sweep(h, K)
        grids[g] = b.jac_get_info(h)["loop_grid"]
        x = get_x(h, s.n)[0]
        b.jac_set_x(h, None)
        st, sw, rr = b.jac_solve(h, 1e-2, 3000)
        out[g] = (hist, x, int(sw[0]), float(rr[0]), get_x(h, s.n)[0])
        b.jac_destroy(h)
    # a workgroup per tile: the XCD with the most tiles sets the count
    assert ntiles + 1 <= grids[1] <= ntiles + ntiles // 4 + 9
    assert grids[2] < ntiles + 1                      # several tiles per workgroup
    assert grids[0] == (grids[2] if auto_resident else grids[1]), name
    for g in (2, 0):
        assert np.array_equal(out[g][0], out[1][0]) and np.array_equal(out[g][1], out[1][1]), (name, g)
        assert out[g][2:4] == out[1][2:4] and np.array_equal(out[g][4], out[1][4]), (name, g)
    _, xr, _ = ref.sweeps(s.row_ptr, s.col_idx, s.vals, s.b[0], K, threads=8)
    assert rel_inf(out[2][1], xr) <= 1e-12


def test_grid_option_range():
    need_gpu()
    b = B()
    s = W.laplace7(8, workload=1)
    h = make(s, 1, 1)
    with pytest.raises(b.JacError):
        b.jac_set_option(h, b.JAC_OPT_GRID, 3)
    assert b.jac_get_option(h, b.JAC_OPT_GRID) == 0
    b.jac_destroy(h)


def test_adjoint_and_refinement_under_both_grids(lap128):
    # the adjoint's forward and recompute sweeps and the FP32 inner sweeps run
    # the same launches: several tiles per workgroup must not change a bit
    need_gpu()
    b = B()
    s = lap128
    import torch
    rng = np.random.default_rng(11)
    g = torch.from_numpy(rng.uniform(-1, 1, s.n)).cuda()
    out = {}
    for grid in (1, 2):
        h = make(s, 1, 64, None, opts={b.JAC_OPT_GRID: grid})
        gb = torch.empty(s.n, dtype=torch.float64, device="cuda")
        gv = torch.empty(s.nnz, dtype=torch.float64, device="cuda")
        b.jac_adjoint(h, 12, 4, g, gb, gv)
        torch.cuda.synchronize()
        grads = (gb.cpu().numpy(), gv.cpu().numpy())
        b.jac_set_x(h, None)
        st, sw, rr = b.jac_solve(h, 1e-12, 600, b.JAC_NORM_L2_REL, b.JAC_FP32_REFINE)
        out[grid] = (grads, int(sw[0]), float(rr[0]), get_x(h, s.n)[0], b.jac_get_info(h)["loop_grid"])
        b.jac_destroy(h)
    assert out[2][4] < out[1][4]
    assert np.array_equal(out[1][0][0], out[2][0][0]) and np.array_equal(out[1][0][1], out[2][0][1])
    assert out[1][1:3] == out[2][1:3] and np.array_equal(out[1][3], out[2][3])
