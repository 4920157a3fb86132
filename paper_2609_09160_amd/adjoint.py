"""Differentiable simulation: the fused step's hand-written discrete adjoint
(liblbfast.so, lbfast_adjoint) behind a torch.autograd.Function.

    mT = simulate(F, m0, tau, nsteps, every=50)       # F: [3, nz, ny, nx]
    J = 0.5 * (mT[1:4] ** 2).sum()                    # any torch objective
    J.backward()                                      # F.grad, m0.grad

The forward pass runs nsteps fused steps with the per-site force field F
(static in time), saving the state every `every` steps; the backward pass
recomputes each segment from its checkpoint and sweeps it with the adjoint
step, all on the GPU.  every=1 keeps every state (nsteps state buffers of
HBM) and the backward pass then recomputes nothing: the fastest choice when
the memory is there.  Storage F64 or F32 (the compute dtype of F and of the
gradients).  The paper itself does not treat differentiation.
"""
import torch

from .solver import Solver


class LBFastAdjoint(torch.autograd.Function):
    """(F, m0) -> m(T) through nsteps of the fused step of a Solver."""

    @staticmethod
    def forward(ctx, F, m0, solver, nsteps, every):
        solver.set_force_field(F.detach())
        solver.set_moments(m0.detach())
        ckpt = solver.forward_checkpointed(nsteps, every)
        mT = solver.moments(dtype=solver.compute_dtype)
        # The backward pass recomputes segments with this force field: save
        # it, so that later forward calls or set_force_field on the same
        # solver do not change the gradient of this call (and an in-place
        # change of F before backward raises, as for any saved tensor).
        ctx.save_for_backward(F)
        ctx.solver, ctx.ckpt, ctx.nsteps, ctx.every = solver, ckpt, int(nsteps), int(every)
        ctx.F_dtype, ctx.m0_dtype = F.dtype, m0.dtype
        ctx.F_shape, ctx.m0_shape = F.shape, m0.shape
        return mT

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g_mT):
        (F,) = ctx.saved_tensors
        ctx.solver.set_force_field(F.detach())
        gF, g0 = ctx.solver.adjoint(ctx.nsteps, ctx.every, ctx.ckpt, g_mT,
                                    want_m0=ctx.needs_input_grad[1])
        gF = gF.reshape(ctx.F_shape).to(ctx.F_dtype)
        if g0 is not None:
            g0 = g0.reshape(ctx.m0_shape).to(ctx.m0_dtype)
        return gF, g0, None, None, None


def simulate(F, m0, tau, nsteps, every=50, lattice=19, storage="f32", bc=(0, 0, 0),
             solver=None):
    """m(T) [10, nz, ny, nx] after nsteps from m0 under the force field F
    [3, nz, ny, nx]; differentiable with respect to F and m0.  A Solver of the
    matching shape may be passed in to reuse its buffers."""
    nz, ny, nx = F.shape[1:]
    if solver is None:
        solver = Solver((nx, ny, nz), tau, lattice=lattice, storage=storage, bc=bc,
                        device=F.device)
    return LBFastAdjoint.apply(F, m0, solver, nsteps, every)
