"""torch.autograd.Function over libjacobi's hand-written adjoint.

``JacobiK.apply(vals, b, handle, K, ckpt_every)`` returns x_K, the iterate
after K synchronous Jacobi sweeps from x_0 = 0 on A(vals) x = b, where
``vals`` are the matrix coefficients in the handle's CSR entry order.  The
forward keeps its checkpoints on the device (``jac_sweep_checkpointed``); the
backward calls ``jac_adjoint`` (checkpointed reverse sweeps on the device),
which reuses them when the handle was not touched in between, and returns
dL/dvals and dL/db.  Any differentiable torch expression producing
``vals`` (for instance ``diffusion_values`` below) then carries the gradient
on to its own parameters.

Both directions run in the library's HIP kernels; this module only moves
device pointers.
"""
from __future__ import annotations

import numpy as np
import torch

from . import binding as B


class JacobiK(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, b, handle, K, ckpt_every):
        vals = vals.detach().contiguous()
        b = b.detach().contiguous()
        B.jac_set_values(handle, vals)
        B.jac_set_rhs(handle, b)
        B.jac_sweep_checkpointed(handle, int(K), int(ckpt_every))
        x = torch.empty_like(b)
        B.jac_get_x(handle, x)
        ctx.save_for_backward(vals, b)
        ctx.handle, ctx.K, ctx.ckpt = handle, int(K), int(ckpt_every)
        ctx.state = B.jac_get_info(handle)["state_gen"]
        return x

    @staticmethod
    def backward(ctx, gx):
        vals, b = ctx.saved_tensors
        # if the handle was used since the forward, restore its system (the
        # adjoint then takes its checkpoints again)
        if B.jac_get_info(ctx.handle)["state_gen"] != ctx.state:
            B.jac_set_values(ctx.handle, vals)
            B.jac_set_rhs(ctx.handle, b)
        gb = torch.empty_like(b)
        gv = torch.empty_like(vals)
        B.jac_adjoint(ctx.handle, ctx.K, ctx.ckpt, gx.contiguous(), gb, gv)
        return gv, gb, None, None, None


def diffusion_values(theta: torch.Tensor, grid, row_ptr, slot) -> torch.Tensor:
    """Coefficients of the cell-centred two-point-flux diffusion matrix on the
    7-point pattern (h = 1), as a differentiable function of the conductivities
    ``theta``: interior face t = 2 th_i th_j / (th_i + th_j), Dirichlet face
    t = 2 th_i, a_ij = -t, a_ii = sum of the six face terms in the order
    (-z, -y, -x, +x, +y, +z).  ``slot[p]`` names entry p's neighbour
    (-z, -y, -x, self, +x, +y, +z) as in the pattern generator."""
    nx, ny, nz = (int(v) for v in grid)
    dev = theta.device
    n = nx * ny * nz
    r = torch.arange(n, device=dev)
    i, j, k = r % nx, (r // nx) % ny, r // (nx * ny)
    sxy = nx * ny
    inside = [k > 0, j > 0, i > 0, i < nx - 1, j < ny - 1, k < nz - 1]
    shifts = [-sxy, -nx, -1, 1, nx, sxy]
    faces = []
    for ok, sh in zip(inside, shifts):
        nb = torch.where(ok, r + sh, r)
        tj = theta[nb]
        t_int = 2.0 * theta * tj / (theta + tj)
        t_bnd = 2.0 * theta
        faces.append(torch.where(ok, t_int, t_bnd))
    diag = faces[0]
    for f in faces[1:]:
        diag = diag + f
    table = torch.stack([-faces[0], -faces[1], -faces[2], diag, -faces[3], -faces[4], -faces[5]], dim=1)
    rp = torch.as_tensor(np.asarray(row_ptr, dtype=np.int64), device=dev)
    rows = torch.repeat_interleave(torch.arange(n, device=dev), rp[1:] - rp[:-1])
    sl = torch.as_tensor(np.asarray(slot, dtype=np.int64), device=dev)
    return table[rows, sl]
