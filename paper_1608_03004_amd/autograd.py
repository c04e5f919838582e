"""Gradients of a loss on the final energy-density profile e(z) of a shock
tube with respect to tau and the initial states, through the library's
hand-written discrete adjoint.

Memory is bounded by checkpointing: the forward keeps every c-th state
(c = ceil(sqrt(nsteps)) by default); the backward walks the segments in
reverse: for each checkpoint rlb_adjoint_segment_forward recomputes the
segment's states (with their stage states, in a scratch buffer of c steps)
and rlb_adjoint_segment_reverse applies the adjoint of every step in reverse
order; the recomputation of the next segment overlaps the reverse sweep of
the current one (two buffers, two streams).  The time
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
        segs = [(state, k1 - k0) for (k0, state), k1 in zip(ctx.checkpoints, bounds[1:])][::-1]  # reverse order
        longest = max(n for _, n in segs)
        # The forward recomputation of the next segment (in reverse order) runs
        # on a side stream while the reverse sweep of the current one runs on
        # the lattice's stream: both are chains of small launches that leave
        # most of the GPU idle.  Two scratch buffers alternate; events order
        # each buffer's fill before its sweep and its sweep before its next fill.
        main = lat.stream
        side = torch.cuda.Stream(device=lat.device)
        side.wait_stream(main)
        scratch = [torch.empty(lat.adjoint_segment_size(longest), dtype=torch.uint8, device=lat.device)
                   for _ in range(2)]
        filled = [torch.cuda.Event() for _ in range(2)]
        freed = [torch.cuda.Event() for _ in range(2)]

        def refill(r):
            buf = r % 2
            if r >= 2:
                side.wait_event(freed[buf])
            lat.adjoint_segment_forward(segs[r][0], segs[r][1], scratch[buf], side)
            filled[buf].record(side)

        refill(0)
        for r, (_, n) in enumerate(segs):
            if r + 1 < len(segs):
                refill(r + 1)
            main.wait_event(filled[r % 2])
            lat.adjoint_segment_reverse(n, scratch[r % 2], lam, dtau)
            freed[r % 2].record(main)
        for s in scratch:
            s.record_stream(side)
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
