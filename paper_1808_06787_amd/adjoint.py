"""Gradients through the sweep: the library's checkpointed forward run and its
one-call adjoint (segment recomputation and the hand-written adjoint kernels),
plus a torch.autograd.Function around them.

Memory: one checkpoint (msd_state_bytes) every `every` steps, and scratch for
a recomputation stack of every-1 states, two adjoint buffers and the dL/dD
accumulator.  Cost: the forward run, one recomputation of it, and the adjoint
steps.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _ffi as F
from .sim import Sim


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def forward_with_checkpoints(sim: Sim, steps: int, every: int) -> dict:
    """Advance a sim that was just initialised (time 0) by `steps`, keeping the state
    at the start of every segment of `every` steps on the device.  Returns the
    checkpoint record that `gradients` takes."""
    steps, every = int(steps), int(every)
    if every < 1:
        raise ValueError("every must be >= 1")
    n = (steps + every - 1) // every
    buf = torch.empty(max(n, 1) * sim.state_bytes(), dtype=torch.uint8, device=sim.device) if n else None
    F.check(sim.lib.msd_forward_checkpointed(sim._h, steps, every, _p(buf)), "msd_forward_checkpointed")
    return {"buffer": buf, "steps": steps, "every": every}


def gradients(sim: Sim, ckpts: dict, T: int, dL_dxi: torch.Tensor, every: int):
    """dL/dxi(0) (N-1 FP64 planes, device) and the N x N matrix of pair derivatives
    dL/dD (numpy) for dL/dxi(T) given as N FP64 planes, after
    forward_with_checkpoints(sim, T, every).  The handle's state is left at an
    intermediate time afterwards."""
    if ckpts["steps"] != T or ckpts["every"] != every:
        raise ValueError("checkpoints were taken for another run")
    if sim.time != T:
        raise ValueError(f"sim is at time {sim.time}, expected {T}")
    g = dL_dxi.to(device=sim.device, dtype=torch.float64).contiguous()
    if tuple(g.shape) != (sim.N,) + sim.nodes_shape:
        raise ValueError("dL_dxi must hold N planes")
    nbytes = int(sim.lib.msd_adjoint_scratch_bytes(sim._h, int(every)))
    scratch = torch.empty(nbytes, dtype=torch.uint8, device=sim.device)
    dxi0 = torch.empty((sim.m,) + sim.nodes_shape, dtype=torch.float64, device=sim.device)
    dD = (C.c_double * (sim.N * sim.N))()
    F.check(sim.lib.msd_adjoint(sim._h, int(T), int(every), _p(ckpts["buffer"]), _p(g), _p(dxi0), dD, _p(scratch),
                                C.c_size_t(nbytes)), "msd_adjoint")
    return dxi0, np.array(dD[:]).reshape(sim.N, sim.N)


class MSDiffusion(torch.autograd.Function):
    """xi(T) = MSDiffusion.apply(xi0, D, spec) with spec a dict of Sim arguments plus
    'steps' and 'every'.  xi0: (N, *nodes) FP64; D: symmetric (N, N) FP64.  The
    gradient with respect to D is symmetric, half of each pair derivative in
    each of the two entries; the gradient with respect to the last species'
    initial field is zero (it is not an independent input, Eq. (2-3b))."""

    @staticmethod
    def forward(ctx, xi0, D, spec):
        spec = dict(spec)
        steps = int(spec.pop("steps"))
        every = int(spec.pop("every", 100))
        lattice = spec.pop("lattice")
        shape = spec.pop("shape")
        precision = spec.pop("precision", "f32")
        sim = Sim(lattice, D.detach().cpu().double().numpy(), shape, precision, device=xi0.device, **spec)
        sim.init(xi0.detach().double())
        ckpts = forward_with_checkpoints(sim, steps, every)
        xi, _, _ = sim.read(torch.float64, flux=False, grad=False)
        ctx.sim, ctx.ckpts, ctx.steps, ctx.every = sim, ckpts, steps, every
        ctx.D_device, ctx.D_dtype = D.device, D.dtype
        return xi

    @staticmethod
    def backward(ctx, grad_xi):
        sim = ctx.sim
        dxi0, dD = gradients(sim, ctx.ckpts, ctx.steps, grad_xi, ctx.every)
        gx = torch.zeros((sim.N,) + sim.nodes_shape, dtype=torch.float64, device=sim.device)
        gx[: sim.m] = dxi0
        gD = torch.tensor(dD / 2.0, dtype=ctx.D_dtype, device=ctx.D_device)
        ctx.sim = None
        ctx.ckpts = None
        sim.close()
        return gx, gD, None
