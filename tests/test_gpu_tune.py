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
    assert len(lines) == 1 and lines[0].split("|")[1].split()[:2] == [str(rows), str(block)]
    set_x(h, np.zeros(s.n))
    st, sw, rr = b.jac_solve(h, 1e-8, 10000)
    sto, xo, ko, _ = ref.solve(s.row_ptr, s.col_idx, s.vals, s.b[0], 1e-8, 10000)
    assert sw[0] == ko and rel_inf(get_x(h, s.n)[0], xo) <= 1e-10
    b.jac_destroy(h)
    # a second handle of the same shape takes the cached choice without timing
    h2 = make(s, 2, 4)
    b.jac_autotune(h2, 5)
    assert b.jac_get_option(h2, b.JAC_OPT_TILE_ROWS) == rows and b.jac_get_option(h2, b.JAC_OPT_BLOCK) == block
    assert len(cache.read_text().splitlines()) == 1
    b.jac_destroy(h2)
