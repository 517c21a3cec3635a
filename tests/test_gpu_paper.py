"""The paper's benchmark problems replayed by the HIP path (FP64): second-order
convergence of the binary erf problem (Sec. 4.1), the Duncan-Toor-like ternary
problem (Sec. 4.2) and the Loschmidt tube (Sec. 4.3), each against the numbers
the paper prints (tests/golden/ternary.txt).  The ternary problems also run on a
wide lattice through the temporally blocked sweep: the field must stay uniform
along the extra axis and give the same observables."""
import os

import numpy as np
import pytest
import torch
from scipy.special import erf

from oracle import lbm

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden():
    vals = {}
    with open(os.path.join(GOLDEN, "ternary.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


def _sim(D, shape, xi0, bc, launch=None, xi_wall=None):
    from paper_1808_06787_amd.sim import Sim

    s = Sim("D2Q5", D, shape, "f64", bc=bc, xi_wall=xi_wall)
    if launch:
        s.set_launch(**launch)
    s.init(torch.from_numpy(np.ascontiguousarray(xi0)))
    return s


@pytest.mark.parametrize("lam1", [1.25, 0.8])
def test_erf_second_order_convergence_on_gpu(lam1):
    """Sec. 4.1 (Figs. 3-4): relative errors of xi_1 and J_1 at t = 5 fall with slope 2
    in dx (Dirichlet anti-bounce-back faces, D_phys = 0.05, lambda_1 given)."""
    Dphys, C0, C1, T = 0.05, 0.9, 0.1, 5.0
    ex, ej, hs = [], [], []
    for nx in (120, 240, 480):
        dx = 12.0 / nx
        d_lat = (1.0 / 3.0) * (1.0 / lam1 - 0.5)
        dt = d_lat * dx * dx / Dphys
        D = np.array([[1.0, d_lat], [d_lat, 1.0]])
        x = lbm.cell_centres(nx, -6.0, 6.0)
        x1 = np.tile(np.where(x < 0, C0, C1), (4, 1))
        walls = {(0, 0): np.array([C0, 1 - C0]), (0, 1): np.array([C1, 1 - C1])}
        s = _sim(D, (nx, 4), np.stack([x1, 1 - x1]), (("dirichlet", "dirichlet"), ("periodic", "periodic")),
                 xi_wall=walls)
        s.step(int(round(T / dt)))
        xi, J, _ = s.read()
        s.close()
        xa = (C0 + C1) / 2 + (C1 - C0) / 2 * erf(x / (2 * np.sqrt(Dphys * T)))
        Ja = -(C1 - C0) / 2 * np.sqrt(Dphys / (np.pi * T)) * np.exp(-x * x / (4 * Dphys * T))
        ex.append(lbm.rel_l2_error(xa, xi[0, 0].cpu().numpy()))
        ej.append(lbm.rel_l2_error(Ja, J[0, 0, 0].cpu().numpy() * dx / dt))
        hs.append(dx)
    sx = np.polyfit(np.log(hs), np.log(ex), 1)[0]
    sj = np.polyfit(np.log(hs), np.log(ej), 1)[0]
    assert 1.8 < sx < 2.2, (sx, ex)
    assert 1.8 < sj < 2.2, (sj, ej)


def _duncan_toor_fields(ny):
    n, dt = 200, 1e-5
    dx = 1.0 / n
    Dp = np.array([[1, 0.833, 0.833], [0.833, 1, 0.168], [0.833, 0.168, 1.0]])
    Dl = Dp * dt / dx ** 2
    np.fill_diagonal(Dl, 1.0)
    x = lbm.cell_centres(n, 0.0, 1.0)
    x1 = np.where(x < 0.25, 0.8, np.where(x < 0.75, 1.6 * (0.75 - x), 0.0))
    x2 = np.full(n, 0.2)
    xi0 = np.stack([x1, x2, 1 - x1 - x2])[:, None, :].repeat(ny, axis=1)
    return Dl, xi0, dt, (n, ny)


@pytest.mark.parametrize("ny,launch", [(1, None), (48, dict(temporal=4, seg_rows=8))])
def test_duncan_toor_on_gpu(ny, launch):
    """Sec. 4.2: the minimum of xi_2 at x = 0.72 (printed 0.1581 near t = 0.2), the
    equilibria (0.4, 0.2), and the reverse -> osmotic -> reverse -> barrier sequence
    of the cross effects."""
    g = _golden()
    D, xi0, dt, shape = _duncan_toor_fields(ny)
    s = _sim(D, shape, xi0, (("zero_flux", "zero_flux"), ("periodic", "periodic")), launch)
    t, xi2, J2, g2 = [], [], [], []
    for k in range(300):
        s.step(100)
        xi, J, G = s.read()
        xi, J, G = xi.cpu().numpy(), J.cpu().numpy(), G.cpu().numpy()
        if ny > 1 and k % 50 == 0:
            assert np.abs(xi - xi[:, :1, :]).max() <= 1e-13           # uniform along y
        pr = lambda a: 0.5 * (a[..., 143] + a[..., 144])               # noqa: E731  (x = 0.72)
        t.append(s.time * dt)
        xi2.append(pr(xi[1, 0]))
        J2.append(pr(J[1, 0, 0]))
        g2.append(pr(G[1, 0, 0]))
    mass, _, _, bad = s.diagnostics()
    s.close()
    assert bad == 0
    t, xi2, J2, g2 = map(np.array, (t, xi2, J2, g2))
    i = xi2.argmin()
    assert abs(xi2[i] - g["duncan_toor_xi2_min"]) < 2e-3
    assert abs(t[i] - g["duncan_toor_t_at_min"]) < 0.03
    nodes = shape[0] * shape[1]
    np.testing.assert_allclose(mass[:2] / nodes, [g["duncan_toor_xi1_eq"], g["duncan_toor_xi2_eq"]], atol=1e-12)
    g_flip = np.where(np.diff(np.sign(g2)) != 0)[0]
    j_flip = np.where(np.diff(np.sign(J2)) != 0)[0]
    assert len(g_flip) == 2 and len(j_flip) == 1
    t1, t2, t3 = t[g_flip[0]], t[g_flip[1]], t[j_flip[0]]
    assert t1 < t2 < t3
    reverse = -J2 * g2 < 0
    assert reverse[t < t1].all()
    assert reverse[(t > t2 + 0.002) & (t < t3 - 0.002)].all()
    assert not reverse[(t > t1 + 0.002) & (t < t2 - 0.002)].any()


@pytest.mark.parametrize("nx,launch", [(1, None), (40, dict(temporal=4, seg_rows=16))])
def test_loschmidt_tube_on_gpu(nx, launch):
    """Sec. 4.3: the bottom-half average of xi_2 peaks at t* = 0.35 h, and the species
    totals give the printed equilibria (0.2575, 0.497)."""
    g = _golden()
    n, dt = 200, 3e-5
    dx = 2.0 / n
    Dp = np.array([[1, 0.2157, 0.7716], [0.2157, 1, 0.8335], [0.7716, 0.8335, 1.0]])
    D = Dp * dt / dx ** 2
    np.fill_diagonal(D, 1.0)
    t_ref_h = (100 * np.pi * np.sqrt(1 / 60)) ** 2 / 3600.0
    y = lbm.cell_centres(n, -1.0, 1.0)
    top = y >= 0
    x1 = np.where(top, 0.515, 0.0)
    x2 = np.where(top, 0.485, 0.509)
    xi0 = np.stack([x1, x2, 1 - x1 - x2])[:, :, None].repeat(nx, axis=2)
    s = _sim(D, (nx, n), xi0, (("periodic", "periodic"), ("zero_flux", "zero_flux")), launch)
    steps = int(round(0.45 / t_ref_h / dt))
    ts, bot = [], []
    while s.time < steps:
        s.step(min(100, steps - s.time))
        xi = s.read(flux=False, grad=False)[0].cpu().numpy()
        if nx > 1 and len(ts) % 50 == 0:
            assert np.abs(xi - xi[:, :, :1]).max() <= 1e-13           # uniform along x
        ts.append(s.time * dt * t_ref_h)
        bot.append(xi[1, ~top, 0].mean())
    mass, _, _, bad = s.diagnostics()
    s.close()
    assert bad == 0
    i = int(np.argmax(bot))
    assert 0 < i < len(bot) - 1
    assert abs(ts[i] - g["loschmidt_tstar_hours"]) < 0.05
    np.testing.assert_allclose(mass[:2] / (nx * n), [g["loschmidt_xi1_eq"], g["loschmidt_xi2_eq"]], atol=1e-12)
