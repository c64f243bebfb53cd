"""GPU: the autotuner picks a candidate shape, keeps the iterate and the
results, and reuses its on-disk cache."""
import os

import numpy as np
import pytest

from gpu_util import B, get_x, make, need_gpu, rel_inf, set_x
from oracle import ref
from paper_2112_02377_amd import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_keeps_state_and_caches(tmp_path, monkeypatch):
    need_gpu()
    b = B()
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("JAC_TUNE_CACHE", str(cache))
    s = W.laplace7(24, workload=1)
    h = make(s, 2, 4)
    x0 = np.random.default_rng(3).uniform(-1, 1, s.n)
    set_x(h, x0)
    b.jac_autotune(h, 5)
    assert rel_inf(get_x(h, s.n)[0], x0) == 0.0          # iterate restored
    rows = b.jac_get_option(h, b.JAC_OPT_TILE_ROWS)
    block = b.jac_get_option(h, b.JAC_OPT_BLOCK)
    cands = {(64, 64), (128, 64), (128, 128), (256, 128), (256, 256), (512, 256), (1024, 256), (2048, 256),
             (512, 128), (512, 512), (1024, 512), (2048, 512), (4096, 512)}
    assert (rows, block) in cands
    lines = cache.read_text().splitlines()
    assert len(lines) == 3 and lines[0].split("|")[1].split()[:2] == [str(rows), str(block)]
    # the launch grid, tuned since it was left automatic
    grid = b.jac_get_option(h, b.JAC_OPT_GRID)
    assert grid in (1, 2) and lines[1].startswith("grid ") and lines[1].split("|")[1].split()[0] == str(grid)
    # the refinement's inner stop parameters: one of the candidate pairs
    tau = b.jac_get_option(h, b.JAC_OPT_INNER_TOL)
    mmax = b.jac_get_option(h, b.JAC_OPT_INNER_MAX)
    assert tau in (1000000, 100000, 10000, 1000) and mmax in (64, 256, 1024, 4096)
    assert lines[2].startswith("refine ") and lines[2].split("|")[1].split()[:2] == [str(tau), str(mmax)]
    set_x(h, np.zeros(s.n))
    st, sw, rr = b.jac_solve(h, 1e-8, 10000)
    sto, xo, ko, _ = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-8, 10000)
    assert sw[0] == ko and rel_inf(get_x(h, s.n)[0], xo) <= 1e-10
    b.jac_destroy(h)
    # a second handle of the same shape takes the cached choice without timing
    h2 = make(s, 2, 4)
    b.jac_autotune(h2, 5)
    assert b.jac_get_option(h2, b.JAC_OPT_TILE_ROWS) == rows and b.jac_get_option(h2, b.JAC_OPT_BLOCK) == block
    assert b.jac_get_option(h2, b.JAC_OPT_INNER_TOL) == tau and b.jac_get_option(h2, b.JAC_OPT_INNER_MAX) == mmax
    assert b.jac_get_option(h2, b.JAC_OPT_GRID) == grid
    assert len(cache.read_text().splitlines()) == 3
    b.jac_destroy(h2)


def test_autotune_batched_keeps_state_and_results(tmp_path, monkeypatch):
    need_gpu()
    b = B()
    cache = tmp_path / "tune_batch.txt"
    monkeypatch.setenv("JAC_TUNE_CACHE", str(cache))
    systems = W.diffusion_batch(6, workload=4, lo=6, hi=20)
    hs = [make(s, 1, 1) for s in systems]
    rng = np.random.default_rng(9)
    x0 = [rng.uniform(-1, 1, s.n * 4) for s in systems]
    for h, x in zip(hs, x0):
        set_x(h, x)
    b.jac_autotune_batched(hs, 8)
    shapes = {(b.jac_get_option(h, b.JAC_OPT_TILE_ROWS), b.jac_get_option(h, b.JAC_OPT_BLOCK)) for h in hs}
    assert len(shapes) == 1 and shapes.pop() in {(256, 256), (512, 256), (1024, 256), (2048, 256)}
    for h, s, x in zip(hs, systems, x0):
        assert np.array_equal(get_x(h, s.n, 4).reshape(-1), x)         # iterates restored
        set_x(h, np.zeros(s.n * 4))
    st, sw, rr = b.jac_solve_batched(hs, 1e-8, 100000)
    assert st == b.JAC_OK
    for si, (h, s) in enumerate(zip(hs, systems)):
        xb = get_x(h, s.n, 4)
        set_x(h, np.zeros(s.n * 4))
        st1, sw1, rr1 = b.jac_solve(h, 1e-8, 100000)
        assert np.array_equal(sw[si], sw1) and np.array_equal(xb, get_x(h, s.n, 4))
    assert len(cache.read_text().splitlines()) == 1 and cache.read_text().startswith("batch 6 ")
    for h in hs:
        b.jac_destroy(h)
