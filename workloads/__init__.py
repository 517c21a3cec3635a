"""Seeded synthetic inputs for the benchmark and test workloads.

This module only draws numbers: initial mole-fraction fields, Maxwell-Stefan
diffusivity matrices, instance lists and perturbation directions.  It holds
none of the lattice Boltzmann arithmetic, so both the FP64 oracle and the HIP
path can take their inputs from here without sharing any of the method.

All randomness is numpy's PCG64 (``np.random.default_rng(seed)``).  Fields are
returned in FP64 with node arrays stored x fastest (numpy shape (N, nz, ny, nx),
(N, ny, nx) or (N, nx)); diffusivities are symmetric N x N matrices in lattice
units with an unused unit diagonal.

Workloads (the paper prints no performance workloads; these stand in for its
problem classes at production sizes):

* ``ternary_1d``       1D ternary step, D1Q3, 256 nodes, FP64, periodic.
* ``ternary_2d``       2D ternary, D2Q5, 4096^2, FP32, periodic, smooth random field.
* ``quaternary_3d``    3D quaternary, D3Q7, 512^3, FP32, zero-flux x walls, two slabs.
* ``batched_2d``       256 independent 2D mixtures with N in {3, 4, 5}, sides 64..1024.
* ``adjoint_2d``       2D ternary 1024^2 for the gradient workload.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

PERIODIC = "periodic"
ZERO_FLUX = "zero_flux"
DIRICHLET = "dirichlet"


@dataclass
class Workload:
    name: str
    lattice: str
    shape: tuple                  # (nx,), (nx, ny) or (nx, ny, nz)
    D: np.ndarray                 # (N, N), lattice units
    xi0: np.ndarray               # (N, *shape[::-1]) float64
    steps: int
    precision: str                # "f32" | "f64"
    bc: tuple = None              # per axis (low, high)
    relax: str = "paper"
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.D.shape[0]

    @property
    def nodes(self) -> int:
        return int(np.prod(self.shape))


def symmetric_loguniform(rng, n, lo, hi):
    """Symmetric n x n matrix with off-diagonal entries exp(U(ln lo, ln hi)), drawn row
    by row over the upper triangle; unit diagonal (unused)."""
    D = np.ones((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            D[i, j] = D[j, i] = np.exp(rng.uniform(np.log(lo), np.log(hi)))
    return D


def smooth_field(rng, N, shape2d, base, amplitude, modes=8, kmax=4):
    """N fields base + p_i on a periodic (nx, ny) grid; p_i is a sum of `modes` plane
    waves a cos(2 pi (k x / nx + l y / ny) + phi) with k, l ~ U{-kmax..kmax} (not both
    zero), a ~ U(0, 1), phi ~ U(0, 2 pi), scaled so that max |p_i| = amplitude; the N
    fields are then divided by their sum so that they add up to one at every node.
    Returns (N, ny, nx) float64."""
    nx, ny = shape2d
    x = np.arange(nx) / nx
    y = np.arange(ny) / ny
    out = np.empty((N, ny, nx))
    for i in range(N):
        p = np.zeros((ny, nx))
        for _ in range(modes):
            while True:
                k, l = rng.integers(-kmax, kmax + 1, size=2)
                if k or l:
                    break
            a = rng.uniform(0.0, 1.0)
            phi = rng.uniform(0.0, 2 * np.pi)
            ax = 2 * np.pi * k * x
            ay = 2 * np.pi * l * y + phi
            # cos(ax + ay) = cos(ay) cos(ax) - sin(ay) sin(ax), built as outer products
            p += a * (np.outer(np.cos(ay), np.cos(ax)) - np.outer(np.sin(ay), np.sin(ax)))
        p *= amplitude / np.abs(p).max()
        out[i] = base + p
    out /= out.sum(axis=0, keepdims=True)
    return out


def ternary_1d(nx=256):
    """1D ternary step: x < nx/2 holds (0.5, 0.5, 0.0), the rest (0.0, 0.5, 0.5);
    D12, D13, D23 = 0.45 * (0.0833, 0.680, 0.168) in lattice units (relaxation
    times between about 0.61 and 1.42); 10,000 steps; FP64; periodic."""
    D = np.ones((3, 3))
    for (i, j), v in {(0, 1): 0.0833, (0, 2): 0.680, (1, 2): 0.168}.items():
        D[i, j] = D[j, i] = 0.45 * v
    left = np.arange(nx) < nx // 2
    xi0 = np.stack([np.where(left, 0.5, 0.0), np.full(nx, 0.5), np.where(left, 0.0, 0.5)])
    return Workload("ternary_1d_d1q3", "D1Q3", (nx,), D, xi0, 10_000, "f64",
                    bc=((PERIODIC, PERIODIC),))


def ternary_2d(shape=(4096, 4096), seed=1, steps=2000):
    """2D ternary, smooth random field about 1/3 (8 modes, amplitude 0.1), D_ij
    log-uniform in [0.05, 0.5]; FP32; periodic."""
    rng = np.random.default_rng(seed)
    D = symmetric_loguniform(rng, 3, 0.05, 0.5)
    xi0 = smooth_field(rng, 3, shape, 1.0 / 3.0, 0.1)
    return Workload(f"ternary_2d_d2q5_{shape[0]}x{shape[1]}", "D2Q5", tuple(shape), D, xi0, steps, "f32",
                    bc=((PERIODIC, PERIODIC), (PERIODIC, PERIODIC)))


def quaternary_3d(shape=(512, 512, 512), seed=2, steps=500, noise_dtype=np.float32):
    """3D quaternary two-slab problem: x < nx/2 holds (0.50, 0.25, 0.15, 0.10), the rest
    (0.10, 0.25, 0.15, 0.50) (species 2 and 3 uniform, so that any flux of theirs is
    osmotic); each value multiplied by (1 + 0.01 eps), eps ~ N(0, 1) i.i.d., then
    renormalised; D_ij log-uniform in [0.02, 0.8]; zero-flux walls in x, periodic in
    y and z; FP32."""
    nx, ny, nz = shape
    rng = np.random.default_rng(seed)
    D = symmetric_loguniform(rng, 4, 0.02, 0.8)
    a = np.array([0.50, 0.25, 0.15, 0.10])
    b = np.array([0.10, 0.25, 0.15, 0.50])
    left = (np.arange(nx) < nx // 2)
    xi0 = np.empty((4, nz, ny, nx))
    for i in range(4):
        base = np.where(left, a[i], b[i])
        eps = rng.standard_normal(size=(nz, ny, nx), dtype=noise_dtype)
        xi0[i] = base * (1.0 + 0.01 * eps.astype(np.float64))
        del eps
    xi0 /= xi0.sum(axis=0, keepdims=True)
    return Workload(f"quaternary_3d_d3q7_{nx}x{ny}x{nz}", "D3Q7", tuple(shape), D, xi0, steps, "f32",
                    bc=((ZERO_FLUX, ZERO_FLUX), (PERIODIC, PERIODIC), (PERIODIC, PERIODIC)))


def batched_instance_specs(count=256, seed_base=4000, sides=tuple(range(64, 1025, 64))):
    """(N, side) of each instance: instance b draws from PCG64(seed_base + b)."""
    specs = []
    for b in range(count):
        rng = np.random.default_rng(seed_base + b)
        N = int(rng.integers(3, 6))
        side = int(sides[rng.integers(0, len(sides))])
        specs.append((N, side))
    return specs


def batched_instance(b, seed_base=4000, sides=tuple(range(64, 1025, 64)), steps=1000):
    """Instance b of the batched workload: N ~ U{3, 4, 5}, side ~ U{64, 128, ..., 1024},
    D_ij log-uniform in [0.05, 0.5], smooth field about 1/N with amplitude 0.1; D2Q5,
    FP32, periodic."""
    rng = np.random.default_rng(seed_base + b)
    N = int(rng.integers(3, 6))
    side = int(sides[rng.integers(0, len(sides))])
    D = symmetric_loguniform(rng, N, 0.05, 0.5)
    xi0 = smooth_field(rng, N, (side, side), 1.0 / N, 0.1)
    return Workload(f"batched_{b}", "D2Q5", (side, side), D, xi0, steps, "f32",
                    bc=((PERIODIC, PERIODIC), (PERIODIC, PERIODIC)))


def batched_2d(count=256, seed_base=4000, steps=1000):
    return [batched_instance(b, seed_base, steps=steps) for b in range(count)]


def adjoint_2d(shape=(1024, 1024), seed=5, steps=2000):
    """Gradient workload: 2D ternary like ``ternary_2d`` (seed 5), D^0 log-uniform in
    [0.05, 0.5]; the target is produced with D* = D^0 (1 + 0.2 U(-1, 1)) entry-wise
    (PCG64(seed * 11), symmetric); the finite-difference direction v for the
    initial field is drawn from PCG64(seed * 111) (unit-norm, zero species sum).
    Checkpoints every 100 steps."""
    rng = np.random.default_rng(seed)
    D0 = symmetric_loguniform(rng, 3, 0.05, 0.5)
    xi0 = smooth_field(rng, 3, shape, 1.0 / 3.0, 0.1)
    r2 = np.random.default_rng(seed * 11)
    Dstar = np.ones((3, 3))
    for i in range(3):
        for j in range(i + 1, 3):
            Dstar[i, j] = Dstar[j, i] = D0[i, j] * (1.0 + 0.2 * r2.uniform(-1.0, 1.0))
    r3 = np.random.default_rng(seed * 111)
    v = r3.standard_normal(size=(3,) + tuple(shape[::-1]))
    v -= v.mean(axis=0, keepdims=True)
    v /= np.linalg.norm(v)
    w = Workload(f"adjoint_2d_d2q5_{shape[0]}x{shape[1]}", "D2Q5", tuple(shape), D0, xi0, steps, "f32",
                 bc=((PERIODIC, PERIODIC), (PERIODIC, PERIODIC)))
    w.meta.update(D_target=Dstar, direction=v, checkpoint_every=100)
    return w
