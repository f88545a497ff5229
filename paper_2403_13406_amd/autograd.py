"""torch.autograd.Function over the composed time loop: U0 -> U(T).

Forward: f0 = f^eq(U0) (eslb_init_equilibrium), n composed steps (eslb_step),
U(T) = sum_k f_k (eslb_moments).  Backward: the hand-written adjoint in libeslb
(eslb_moments_adjoint, eslb_adjoint with step checkpointing, eslb_init_adjoint).
Only device memory and the stream come from PyTorch.
"""
import torch


class EslbTimeLoop(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, solver, nsteps, ckpt_every):
        u0c = u0.detach().contiguous()
        f0 = solver.init_equilibrium(u0c)
        f = f0.clone()
        solver.step(f, nsteps)
        uT = solver.moments(f)
        solver.offsets = [0] * solver.q         # f0 is stored with zero offsets
        ctx.solver, ctx.nsteps, ctx.ckpt = solver, int(nsteps), int(ckpt_every)
        ctx.save_for_backward(u0c, f0)
        return uT

    @staticmethod
    def backward(ctx, ubar):
        u0, f0 = ctx.saved_tensors
        s = ctx.solver
        s.offsets = [0] * s.q
        fbar = s.moments_adjoint(ubar.detach().contiguous())
        s.adjoint(f0, ctx.nsteps, ctx.ckpt, fbar)
        return s.init_adjoint(u0, fbar), None, None, None


def time_loop(u0, solver, nsteps, ckpt_every=50):
    """U(T) from U0 through nsteps composed steps, differentiable w.r.t. U0."""
    return EslbTimeLoop.apply(u0, solver, nsteps, ckpt_every)
