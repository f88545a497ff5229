"""torch.autograd.Function over the composed time loop: U0 -> U(T).

Forward: f0 = f^eq(U0) (eslb_init_equilibrium), n composed steps keeping the
state every ckpt_every steps (eslb_step_checkpointed), U(T) = sum_k f_k
(eslb_moments).  Backward: the hand-written adjoint in libeslb
(eslb_moments_adjoint, eslb_adjoint_checkpointed from the forward's checkpoints,
eslb_init_adjoint).
Only device memory and the stream come from PyTorch.
"""
import torch


class EslbTimeLoop(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u0, solver, nsteps, ckpt_every, tape):
        u0c = u0.detach().contiguous()
        f = solver.init_equilibrium(u0c)
        solver.offsets = [0] * solver.q          # f^eq(U0) is stored with zero offsets
        # the forward run keeps the checkpoints the backward pass starts from
        ckpt = solver.step_checkpointed(f, nsteps, ckpt_every)
        uT = solver.moments(f)
        solver.offsets = [0] * solver.q
        ctx.solver, ctx.nsteps, ctx.ckpt, ctx.tape = solver, int(nsteps), int(ckpt_every), tape
        ctx.save_for_backward(u0c, ckpt)
        return uT

    @staticmethod
    def backward(ctx, ubar):
        u0, ckpt = ctx.saved_tensors
        s = ctx.solver
        s.offsets = [0] * s.q
        fbar = s.moments_adjoint(ubar.detach().contiguous())
        s.adjoint_checkpointed(ckpt, ctx.nsteps, ctx.ckpt, fbar, tape=ctx.tape)
        return s.init_adjoint(u0, fbar), None, None, None, None


def time_loop(u0, solver, nsteps, ckpt_every=50, tape="auto"):
    """U(T) from U0 through nsteps composed steps, differentiable w.r.t. U0.

    tape: workspace choice of the backward pass (Solver.adjoint)."""
    return EslbTimeLoop.apply(u0, solver, nsteps, ckpt_every, tape)
