"""Pins of the autograd twin: its forward pass equals the numpy oracle, and its
gradients equal central finite differences of the numpy oracle."""
import numpy as np
import pytest
import torch

from oracle import lbm, ms, twin

LATS = ["D1Q2", "D1Q3", "D2Q4", "D2Q5", "D3Q6", "D3Q7", "D2Q9", "D3Q15"]


def _rand_D(rng, n, lo=0.03, hi=0.3):
    D = np.ones((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            D[i, j] = D[j, i] = np.exp(rng.uniform(np.log(lo), np.log(hi)))
    return D


def _problem(name, rng, N, relax=ms.RELAX_PAPER, walls=True, lin=False, dilute=False):
    shape = {1: (7,), 2: (6, 5), 3: (4, 3, 3)}[int(name[1])]
    d = len(shape)
    bc = [("periodic", "periodic")] * d
    xi_wall = {}
    if walls:
        bc[0] = ("dirichlet", "zero_flux")
        x = rng.uniform(0.2, 1.0, N)
        xi_wall[(0, 0)] = x / x.sum()
    xref = None
    if lin:
        x = rng.uniform(0.2, 1.0, N)
        xref = x / x.sum()
    return lbm.Problem(name, _rand_D(rng, N), shape, bc=tuple(bc), xi_wall=xi_wall, relax=relax, xi_ref=xref,
                       magic=0.3 if relax == ms.RELAX_TRT else ms.MAGIC_PAPER, dilute=dilute)


def _field(rng, p):
    x = rng.uniform(0.2, 1.0, size=(p.N,) + p.nodes)
    return x / x.sum(axis=0, keepdims=True)


@pytest.mark.parametrize("name", LATS)
@pytest.mark.parametrize("relax", [ms.RELAX_PAPER, ms.RELAX_SRT, ms.RELAX_TRT])
@pytest.mark.parametrize("dilute", [False, True])
def test_twin_forward_equals_oracle(name, relax, dilute):
    rng = np.random.default_rng(31)
    p = _problem(name, rng, 4, relax, dilute=dilute)
    xi0 = _field(rng, p)
    f_np = lbm.run(p, xi0, 6)
    tw = twin.Twin(p)
    f_t = tw.run(torch.tensor(xi0), torch.tensor(p.D), 6).numpy()
    np.testing.assert_allclose(f_t, f_np, rtol=0, atol=1e-14)


def _loss_np(p, xi0, target, steps):
    xi = lbm.mole_fractions(lbm.run(p, xi0, steps))
    return float(((xi - target) ** 2).sum())


@pytest.mark.parametrize("name", LATS)
@pytest.mark.parametrize("lin", [False, True])
@pytest.mark.parametrize("dilute", [False, True])
def test_twin_gradients_equal_finite_differences(name, lin, dilute):
    rng = np.random.default_rng(32)
    p = _problem(name, rng, 3, lin=lin, dilute=dilute)
    xi0 = _field(rng, p)
    target = _field(rng, p)
    steps = 5
    L, gD, gx = twin.misfit_gradients(p, xi0, target, steps)
    assert abs(L - _loss_np(p, xi0, target, steps)) < 1e-12 * max(L, 1)
    h = 1e-6
    N = p.N
    for i in range(N):
        for j in range(i + 1, N):
            Dp, Dm = p.D.copy(), p.D.copy()
            Dp[i, j] = Dp[j, i] = p.D[i, j] + h
            Dm[i, j] = Dm[j, i] = p.D[i, j] - h
            pp = lbm.Problem(p.lattice, Dp, p.shape, bc=p.bc, xi_wall=p.xi_wall, relax=p.relax, xi_ref=p.xi_ref,
                             dilute=p.dilute)
            pm = lbm.Problem(p.lattice, Dm, p.shape, bc=p.bc, xi_wall=p.xi_wall, relax=p.relax, xi_ref=p.xi_ref,
                             dilute=p.dilute)
            fd = (_loss_np(pp, xi0, target, steps) - _loss_np(pm, xi0, target, steps)) / (2 * h)
            assert abs(fd - gD[i, j]) <= 1e-6 * max(abs(fd), 1e-3), (i, j, fd, gD[i, j])
    v = rng.standard_normal(size=xi0.shape)
    v[-1] = 0.0
    fd = (_loss_np(p, xi0 + h * v, target, steps) - _loss_np(p, xi0 - h * v, target, steps)) / (2 * h)
    assert abs(fd - float((gx * v[:-1]).sum())) <= 1e-6 * max(abs(fd), 1e-3)
