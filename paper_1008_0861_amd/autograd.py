"""torch.autograd.Function over the C ABI: nsteps semi-implicit steps as a
differentiable map (T0, chi) -> T_N.  The forward runs asd_adjoint_forward
(the steps, storing a checkpoint every ckpt_every steps); the backward is the
hand-written adjoint asd_adjoint_step_stored, which recomputes each segment
from its stored checkpoint."""
import torch

from . import binding


class SemiImplicitSteps(torch.autograd.Function):
    """T_N = SemiImplicitSteps.apply(T0, chi, grid, dt, nsteps, ckpt_every)

    grid: a binding.Grid built with per_cell_chi=True and b already set.
    T0, chi: contiguous CUDA tensors of the grid's shape and dtype.
    Gradients flow to T0 and chi.
    """

    @staticmethod
    def forward(ctx, T0, chi, grid, dt, nsteps, ckpt_every):
        cur = torch.cuda.current_stream()
        grid.stream.wait_stream(cur)
        with torch.cuda.stream(grid.stream):
            chi_c = chi.detach().contiguous()
            grid.set_field("chi", chi_c)
            T = T0.detach().clone()
            grid.set_field("T", T)
            ws = grid.adjoint_forward(dt, nsteps, ckpt_every)
        cur.wait_stream(grid.stream)
        ctx.save_for_backward(chi_c)
        ctx.ws = ws  # the checkpoints (states at steps 0, k, 2k, ...)
        ctx.grid, ctx.dt, ctx.nsteps, ctx.k = grid, dt, nsteps, ckpt_every
        return T

    @staticmethod
    def backward(ctx, gT):
        (chi,) = ctx.saved_tensors
        grid = ctx.grid
        cur = torch.cuda.current_stream()
        grid.stream.wait_stream(cur)
        with torch.cuda.stream(grid.stream):
            grid.set_field("chi", chi)
            gT0, gchi = grid.adjoint_stored(ctx.dt, ctx.nsteps, ctx.k, ctx.ws, gT.contiguous(), grad_chi=True)
        cur.wait_stream(grid.stream)
        ctx.ws = None
        return gT0, gchi, None, None, None, None


def semi_implicit_steps(T0, chi, grid, dt, nsteps, ckpt_every=10):
    return SemiImplicitSteps.apply(T0, chi, grid, dt, nsteps, ckpt_every)
