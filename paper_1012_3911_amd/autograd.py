"""torch.autograd binding of the split-operator run and its adjoint.

``SplitStep.apply(psi0, ebar, V0, grid)`` propagates psi0 through
``ebar.shape[0]`` Strang steps on ``grid`` (field integrals ``ebar`` of shape
(nsteps, ndim), static potential ``V0``) and returns psi(T).  Its backward
calls the library's hand-written adjoint (sfo_adjoint): the state and the
incoming gradient are walked back together with the exact inverse step (no
stored trajectory), returning the gradients with respect to psi0, ebar and
V0.  Gradients follow torch's complex convention (the incoming gradient is
2 dL/dconj(psi(T)) for a real loss).
"""
from __future__ import annotations

import torch


class SplitStep(torch.autograd.Function):
    @staticmethod
    def forward(ctx, psi0, ebar, V0, grid):
        v0 = V0.detach()
        e_host = ebar.detach().to("cpu", torch.float64).numpy().copy()
        grid.set_potential(v0)
        grid.set_field(e_host)
        nsteps = int(ebar.shape[0])
        psi = psi0.detach().to(grid.torch_dtype).clone().contiguous()
        grid.propagate(psi, 0, nsteps)
        ctx.grid = grid
        ctx.nsteps = nsteps
        ctx.ebar_meta = (ebar.device, ebar.dtype)
        ctx.v0_meta = (V0.shape, V0.dtype, V0.device)
        # the grid is mutable: keep what this run installed, so that a later
        # forward call on the same grid cannot change the tables the
        # backward of this one walks back through
        ctx.ebar_host = e_host
        ctx.tables = grid.tables_version
        ctx.save_for_backward(psi, v0)
        return psi

    @staticmethod
    def backward(ctx, gT):
        psiT, v0 = ctx.saved_tensors
        grid = ctx.grid
        if grid.tables_version != ctx.tables:
            grid.set_potential(v0)
            grid.set_field(ctx.ebar_host)
        psi = psiT.clone()
        g = gT.detach().to(grid.torch_dtype).contiguous().clone()
        want_v = ctx.needs_input_grad[2]
        de, dv = grid.adjoint(psi, g, 0, ctx.nsteps, want_dV0=want_v)
        dev, dt = ctx.ebar_meta
        vshape, vdt, vdev = ctx.v0_meta
        gpsi = g if ctx.needs_input_grad[0] else None
        gE = de.to(dev, dt) if ctx.needs_input_grad[1] else None
        gV = dv.reshape(vshape).to(vdev, vdt) if want_v else None
        return gpsi, gE, gV, None


def propagate(psi0, ebar, V0, grid):
    """Differentiable psi(T) (see SplitStep)."""
    return SplitStep.apply(psi0, ebar, V0, grid)
