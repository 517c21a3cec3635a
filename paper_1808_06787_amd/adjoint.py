"""Gradients through the sweep: checkpointed forward run, segment recompute and
the hand-written adjoint kernels, plus a torch.autograd.Function around them.

Memory: one checkpoint (msd_state_bytes) every `every` steps, a recompute stack
of every-1 states, two adjoint buffers and the dL/dD accumulator.  Cost: the
forward run, one recompute of it, and one adjoint launch per step.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _ffi as F
from .sim import Sim


def _p(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


def forward_with_checkpoints(sim: Sim, steps: int, every: int) -> dict:
    """Advance an initialised sim by `steps`, saving its state at every multiple of
    `every` (from its current time) before stepping on.  Returns {time: state}."""
    if every < 1:
        raise ValueError("every must be >= 1")
    ckpts = {}
    t_end = sim.time + int(steps)
    while sim.time < t_end:
        state, t = sim.save()
        ckpts[t] = state
        sim.step(min(every, t_end - sim.time))
    return ckpts


def gradients(sim: Sim, ckpts: dict, T: int, dL_dxi: torch.Tensor, every: int):
    """dL/dxi(0) (N-1 FP64 planes, device) and the N x N matrix of pair derivatives
    dL/dD (numpy) for dL/dxi(T) given as N FP64 planes.  `ckpts` are the states
    saved by forward_with_checkpoints (starting at time 0).  The handle's state
    is left at an intermediate time afterwards."""
    lib = sim.lib
    h = sim._h
    if sim.time != T:
        raise ValueError(f"sim is at time {sim.time}, expected {T}")
    g = dL_dxi.to(device=sim.device, dtype=torch.float64).contiguous()
    if tuple(g.shape) != (sim.N,) + sim.nodes_shape:
        raise ValueError("dL_dxi must hold N planes")
    sb = sim.state_bytes()
    acc = torch.empty(int(lib.msd_adjoint_accum_bytes(h)), dtype=torch.uint8, device=sim.device)
    a_cur = torch.empty(sb, dtype=torch.uint8, device=sim.device)
    a_nxt = torch.empty(sb, dtype=torch.uint8, device=sim.device)
    stack = torch.empty(max(every - 1, 1) * sb, dtype=torch.uint8, device=sim.device)
    F.check(lib.msd_adjoint_begin(h, _p(acc)), "msd_adjoint_begin")
    F.check(lib.msd_adjoint_seed(h, _p(g), _p(a_cur)), "msd_adjoint_seed")
    starts = sorted(t for t in ckpts if t < T)
    if T > 0 and (not starts or starts[0] != 0):
        raise ValueError("checkpoints must start at time 0")
    for i in range(len(starts) - 1, -1, -1):
        t0 = starts[i]
        t1 = starts[i + 1] if i + 1 < len(starts) else T
        if t1 - t0 > every:
            raise ValueError("checkpoints further apart than `every`")
        if t1 - t0 > 1:
            sim.restore(ckpts[t0], t0)
            F.check(lib.msd_record(h, t1 - t0 - 1, _p(stack)), "msd_record")
        in_b = C.c_int32(0)
        F.check(lib.msd_adjoint_steps(h, t1, t0, _p(ckpts[t0]), _p(stack), _p(a_cur), _p(a_nxt), _p(acc),
                                      C.byref(in_b)), "msd_adjoint_steps")
        if in_b.value:
            a_cur, a_nxt = a_nxt, a_cur
    dxi0 = torch.empty((sim.m,) + sim.nodes_shape, dtype=torch.float64, device=sim.device)
    dD = (C.c_double * (sim.N * sim.N))()
    F.check(lib.msd_adjoint_finish(h, _p(a_cur), _p(acc), _p(dxi0), dD), "msd_adjoint_finish")
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
