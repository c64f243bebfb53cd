"""Helpers shared by the GPU tests: build handles from generated systems and
move vectors between numpy and the device."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def B():
    from paper_2112_02377_amd import binding
    return binding


def make(sysm, mode=None, nparts=1, sub_grid=None, grid=True, opts=None):
    b = B()
    h = b.jac_create(sysm.n, sysm.row_ptr, sysm.col_idx, sysm.vals, sysm.nrhs, sysm.b.reshape(-1))
    for k, v in (opts or {}).items():
        b.jac_set_option(h, k, v)
    if grid and sysm.grid is not None:
        b.jac_set_grid(h, *sysm.grid)
    if mode is not None:
        b.jac_partition(h, mode, nparts, sub_grid)
    return h


def get_x(h, n, nrhs=1):
    b = B()
    x = torch.empty(n * nrhs, dtype=torch.float64, device="cuda")
    b.jac_get_x(h, x)
    torch.cuda.synchronize()
    return x.cpu().numpy().reshape(nrhs, n)


def set_x(h, x):
    b = B()
    t = torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64).reshape(-1)).cuda()
    b.jac_set_x(h, t)
    torch.cuda.synchronize()


def sweep(h, K, nrhs=1):
    b = B()
    hist = torch.zeros(max(K, 1) * nrhs, dtype=torch.float64, device="cuda")
    b.jac_sweep(h, K, hist)
    torch.cuda.synchronize()
    return hist.cpu().numpy()[:K * nrhs].reshape(K, nrhs)


def rel_inf(a, b):
    s = max(np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() / s
