"""Shared helpers of the GPU tests: run a case through the HIP library and
through the oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np

from oracle import lbm, ms

PREC_TOL = {
    # FP64: the sweep must match the oracle to 1e-12 relative to the field's size.
    "f64": dict(xi=1e-12, flux_rel=1e-11),
    # FP32: 1e-5 absolute on mole fractions.  Fluxes and gradients are first
    # moments of distributions of size ~w xi, so their rounding error is about
    # q * eps32 * max f per step, independent of the (small) flux itself:
    # we allow 2e-6 absolute in lattice units.
    "f32": dict(xi=1e-5, flux_abs=2e-6),
}


def rand_D(rng, n, lo=0.03, hi=0.3):
    D = np.ones((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            D[i, j] = D[j, i] = np.exp(rng.uniform(np.log(lo), np.log(hi)))
    return D


def rand_field(rng, N, nodes, lo=0.2):
    x = rng.uniform(lo, 1.0, size=(N,) + tuple(nodes))
    return x / x.sum(axis=0, keepdims=True)


def smooth_field(rng, N, nodes, amp=0.1):
    """Smooth periodic random field about 1/N (few Fourier modes per axis)."""
    grids = np.meshgrid(*[np.arange(n) / n for n in nodes], indexing="ij")
    out = np.empty((N,) + tuple(nodes))
    for i in range(N):
        p = np.zeros(nodes)
        for _ in range(4):
            k = rng.integers(-3, 4, size=len(nodes))
            p += rng.uniform(0, 1) * np.cos(2 * np.pi * sum(kk * g for kk, g in zip(k, grids)) + rng.uniform(0, 6.3))
        p *= amp / max(np.abs(p).max(), 1e-12)
        out[i] = 1.0 / N + p
    return out / out.sum(axis=0, keepdims=True)


RELAX_NAMES = {"paper": ms.RELAX_PAPER, "srt": ms.RELAX_SRT, "trt": ms.RELAX_TRT}


def oracle_problem(lattice, D, shape, bc=None, xi_wall=None, relax="paper", xi_ref=None, c_t=1.0,
                   trt_magic=ms.MAGIC_PAPER, dilute=False):
    return lbm.Problem(lattice, D, shape, bc=bc, xi_wall=xi_wall or {}, relax=RELAX_NAMES[relax],
                       magic=trt_magic, xi_ref=xi_ref, c_t=c_t, dilute=dilute)


def oracle_run(prob, xi0, steps):
    f = lbm.run(prob, xi0, steps)
    return lbm.observables(prob, f)


def gpu_run(lattice, D, shape, precision, xi0, steps, bc=None, xi_wall=None, relax="paper", xi_ref=None,
            c_t=1.0, launch=None, split=None, trt_magic=ms.MAGIC_PAPER, dilute=False):
    import torch

    from paper_1808_06787_amd.sim import Sim

    sim = Sim(lattice, D, shape, precision, bc=bc, xi_wall=xi_wall, relax=relax, c_t=c_t, xi_ref=xi_ref,
              trt_magic=trt_magic, dilute=dilute)
    if launch:
        sim.set_launch(**launch)
    sim.init(torch.from_numpy(np.ascontiguousarray(xi0)))
    if split:
        for s in split:
            sim.step(s)
    else:
        sim.step(steps)
    xi, J, g = sim.read(torch.float64)
    torch.cuda.synchronize()
    out = (xi.cpu().numpy(), J.cpu().numpy(), g.cpu().numpy())
    sim.close()
    return out


def assert_parity(gpu, orc, precision, label=""):
    xi_g, J_g, g_g = gpu
    xi_o, g_o, J_o = orc[0], orc[1], orc[2]
    tol = PREC_TOL[precision]
    scale = max(np.abs(xi_o).max(), 1e-300)
    err_xi = np.abs(xi_g - xi_o).max()
    if precision == "f64":
        assert err_xi <= tol["xi"] * scale, f"{label}: xi error {err_xi:.3e}"
        for name, a, b in (("J", J_g, J_o), ("grad", g_g, g_o)):
            s = max(np.abs(b).max(), 1e-300)
            e = np.abs(a - b).max()
            assert e <= tol["flux_rel"] * s + 1e-15, f"{label}: {name} error {e:.3e} (scale {s:.3e})"
    else:
        assert err_xi <= tol["xi"], f"{label}: xi error {err_xi:.3e}"
        for name, a, b in (("J", J_g, J_o), ("grad", g_g, g_o)):
            e = np.abs(a - b).max()
            assert e <= tol["flux_abs"], f"{label}: {name} error {e:.3e}"
    return err_xi
