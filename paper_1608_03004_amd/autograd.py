"""Gradients of a loss on the final energy-density profile e(z) of a shock
tube with respect to tau and the initial states, through the library's
hand-written discrete adjoint.

Memory is bounded by checkpointing: the forward keeps every c-th state
(c = ceil(sqrt(nsteps)) by default); the backward walks the segments in
reverse and hands each checkpoint to rlb_adjoint_segment, which recomputes
the segment's states (with their stage states, kept in one scratch buffer of
c steps) and applies the adjoint of every step in reverse order.  The time
step is held fixed: the gradient with respect to tau is taken at constant dt.
"""
import math

import torch

from .rlb import Lattice, Tube


class SodProfile(torch.autograd.Function):
    """e(z) at the final time of one tube from (tau, P_L, n_L, P_R, n_R).

    Inputs are 0-dim FP64 tensors; the lattice (created with adjoint=True,
    one tube) is passed as a non-tensor argument together with the number of
    steps and the checkpoint interval (0: ceil(sqrt(nsteps))).
    """

    @staticmethod
    def forward(ctx, tau, P_L, n_L, P_R, n_R, lat: Lattice, nsteps: int, every: int = 0):
        every = every or max(1, math.ceil(math.sqrt(nsteps)))
        lat.set_tau(float(tau))
        lat.set_initial_state((float(P_L), float(n_L), 0.0), (float(P_R), float(n_R), 0.0))
        checkpoints = []
        k = 0
        while k < nsteps:
            checkpoints.append((k, lat.get_state().clone()))
            n = min(every, nsteps - k)
            lat.step(n)
            k += n
        final = lat.get_state().clone()
        e = lat.fields(0)[5].clone()
        lat.check()
        ctx.lat, ctx.nsteps, ctx.checkpoints, ctx.final = lat, nsteps, checkpoints, final
        return e

    @staticmethod
    def backward(ctx, de):
        lat = ctx.lat
        nx = lat.tubes[0].nx
        dfields = torch.zeros((10, nx), dtype=torch.float64, device=lat.device)
        dfields[5] = de.to(torch.float64)
        lam = torch.zeros(lat.state_elems, dtype=lat.dtype, device=lat.device)
        lat.fields_adjoint(0, ctx.final, dfields, lam)
        dtau = torch.zeros(len(lat.tubes), dtype=torch.float64, device=lat.device)
        bounds = [k for k, _ in ctx.checkpoints] + [ctx.nsteps]
        longest = max(k1 - k0 for (k0, _), k1 in zip(ctx.checkpoints, bounds[1:]))
        scratch = torch.empty(lat.adjoint_segment_size(longest), dtype=torch.uint8, device=lat.device)
        for seg in range(len(ctx.checkpoints) - 1, -1, -1):
            k0, state = ctx.checkpoints[seg]
            lat.adjoint_segment(state, bounds[seg + 1] - k0, scratch, lam, dtau)
        gl, gr = lat.initial_state_adjoint(0, lam)
        dev, f64 = lat.device, torch.float64
        g = lambda v: torch.tensor(v, dtype=f64, device=dev)
        return (dtau[0].clone(), g(gl[0]), g(gl[1]), g(gr[0]), g(gr[1]), None, None, None)


def profile_loss(tau, P_L, n_L, P_R, n_R, lat: Lattice, nsteps: int, target, every: int = 0):
    """L = sum_x dz (e_x - target_x)^2 at the final time."""
    e = SodProfile.apply(tau, P_L, n_L, P_R, n_R, lat, nsteps, every)
    t = lat.tubes[0]
    dz = (t.z_max - t.z_min) / t.nx
    return dz * torch.sum((e - target) ** 2)
