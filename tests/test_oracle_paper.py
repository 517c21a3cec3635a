"""Pins of the oracle against the paper's printed numbers and the continuum model.

* Table I (Sec. 4.1): relative L2 errors of xi_1 and J_1, MRT and SRT, t = 1, 5, 20;
* second-order convergence in space (Sec. 4.1, Figs. 3-4 captions: slope 2.0);
* Duncan-Toor-like ternary problem (Sec. 4.2): xi_2 minimum 0.1581 near t = 0.2 at
  x = 0.72, equilibria, and the reverse / osmotic / barrier sequence;
* Loschmidt tube (Sec. 4.3): equilibria and the time t* = 0.35 h of the extremum of
  the bottom-average xi_2;
* decay of Fourier modes against the continuum equation (2-13), binary and
  linearised multicomponent, on all three lattices (pins the Lambda_1 <-> D~ map
  of Eq. (3-26) and the sound speed of each lattice).

Expected numbers live in tests/golden/ with their citations.
"""
import os

import numpy as np
import pytest
from scipy.linalg import expm
from scipy.special import erf

from oracle import lbm, ms
from oracle import lattice as lat

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_table1():
    rows = {}
    with open(os.path.join(GOLDEN, "table1.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            model, t, e_xi, e_j = line.split()
            rows[(model, int(t))] = (float(e_xi), float(e_j))
    return rows


def _read_ternary():
    vals = {}
    with open(os.path.join(GOLDEN, "ternary.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            k, v = line.split()
            vals[k] = float(v)
    return vals


def erf_problem(relax, nx, lam1=1.25, ny=2, times=(1, 5, 20)):
    """Sec. 4.1 set-up: D = 0.05, C0 = 0.9 for x < 0, C1 = 0.1 for x >= 0 on [-6, 6],
    Dirichlet (anti-bounce-back) walls holding C0 and C1, periodic in y.  The field is
    uniform in y, so ny = 2 gives the same numbers as the paper's 40 rows.
    Returns [(t, E(xi_1), E(J_1))]."""
    Dphys, C0, C1 = 0.05, 0.9, 0.1
    dx = 12.0 / nx
    d_lat = lat.D2Q5.cs2 * (1.0 / lam1 - 0.5)          # Eq. (3-26), binary
    dt = d_lat * dx * dx / Dphys
    D = np.array([[1.0, d_lat], [d_lat, 1.0]])
    walls = {(0, 0): np.array([C0, 1 - C0]), (0, 1): np.array([C1, 1 - C1])}
    p = lbm.Problem("D2Q5", D, (nx, ny), bc=((lbm.DIRICHLET, lbm.DIRICHLET), (lbm.PERIODIC, lbm.PERIODIC)),
                    xi_wall=walls, relax=relax)
    x = lbm.cell_centres(nx, -6.0, 6.0)
    x1 = np.tile(np.where(x < 0, C0, C1), (ny, 1))
    f = lbm.init(p, np.stack([x1, 1 - x1]))
    out, t = [], 0
    for T in times:
        n = int(round(T / dt))
        while t < n:
            f = lbm.step(p, f)
            t += 1
        xi, _, J = lbm.observables(p, f)
        xa = (C0 + C1) / 2 + (C1 - C0) / 2 * erf(x / (2 * np.sqrt(Dphys * T)))           # Eq. (4-2a)
        Ja = -(C1 - C0) / 2 * np.sqrt(Dphys / (np.pi * T)) * np.exp(-x * x / (4 * Dphys * T))  # Eq. (4-2b)
        Jn = J[0, 0, 0] * dx / dt                        # lattice -> physical flux units
        out.append((T, lbm.rel_l2_error(xa, xi[0, 0]), lbm.rel_l2_error(Ja, Jn)))
    return out


@pytest.mark.parametrize("model,relax", [("MRT", ms.RELAX_PAPER), ("SRT", ms.RELAX_SRT)])
def test_table_I_errors(model, relax):
    """All twelve numbers of Table I to 0.5 % (most agree to 0.1 %)."""
    table = _read_table1()
    for t, e_xi, e_j in erf_problem(relax, 240):
        ref_xi, ref_j = table[(model, t)]
        assert abs(e_xi / ref_xi - 1) < 5e-3, (model, t, e_xi, ref_xi)
        assert abs(e_j / ref_j - 1) < 5e-3, (model, t, e_j, ref_j)


def test_mrt_beats_srt():
    """Sec. 4.1: the MRT model with Eq. (3-16) is more accurate than SRT at every time."""
    mrt = erf_problem(ms.RELAX_PAPER, 240)
    srt = erf_problem(ms.RELAX_SRT, 240)
    for a, b in zip(mrt, srt):
        assert a[1] < b[1] and a[2] < b[2]


@pytest.mark.parametrize("lam1", [1.25, 0.8, 1.6])
def test_second_order_convergence(lam1):
    """Sec. 4.1 (Figs. 3-4): errors of xi_1 and J_1 at t = 5 fall with slope 2 in dx,
    for several lambda_1^11."""
    sizes = [120, 240, 480]          # dx = 1/10, 1/20, 1/40
    ex, ej = [], []
    for nx in sizes:
        (_, e_xi, e_j), = erf_problem(ms.RELAX_PAPER, nx, lam1=lam1, ny=1, times=(5,))
        ex.append(e_xi)
        ej.append(e_j)
    h = 12.0 / np.array(sizes)
    sx = np.polyfit(np.log(h), np.log(ex), 1)[0]
    sj = np.polyfit(np.log(h), np.log(ej), 1)[0]
    assert 1.8 < sx < 2.2, sx
    assert 1.8 < sj < 2.2, sj


def _duncan_toor(t_end, every):
    """Sec. 4.2: D12 = D13 = 0.833, D23 = 0.168 on [0, 1], zero flux in x (reading of
    the boundary conditions), 200 nodes, xi_1 ramp, xi_2 = 0.2.  dt = 1e-5 gives
    relaxation times between about 0.6 and 1.5."""
    n, dt = 200, 1e-5
    dx = 1.0 / n
    Dp = np.array([[1, 0.833, 0.833], [0.833, 1, 0.168], [0.833, 0.168, 1.0]])
    Dl = Dp * dt / dx ** 2
    np.fill_diagonal(Dl, 1.0)
    p = lbm.Problem("D2Q5", Dl, (n, 1), bc=((lbm.ZERO_FLUX, lbm.ZERO_FLUX), (lbm.PERIODIC, lbm.PERIODIC)))
    x = lbm.cell_centres(n, 0.0, 1.0)
    x1 = np.where(x < 0.25, 0.8, np.where(x < 0.75, 1.6 * (0.75 - x), 0.0))
    x2 = np.full(n, 0.2)
    f = lbm.init(p, np.stack([x1, x2, 1 - x1 - x2])[:, None, :])
    # x = 0.72 lies half-way between the centres of nodes 143 and 144
    rec = []
    for s in range(1, int(round(t_end / dt)) + 1):
        f = lbm.step(p, f)
        if s % every == 0:
            xi, grad, J = lbm.observables(p, f)
            pr = lambda a: 0.5 * (a[..., 143] + a[..., 144])   # noqa: E731
            rec.append((s * dt, pr(xi[1, 0]), pr(J[1, 0, 0]), pr(grad[1, 0, 0]), xi[:, 0].mean(axis=1)))
    return rec


@pytest.mark.slow
def test_duncan_toor_minimum_and_cross_effects():
    g = _read_ternary()
    rec = _duncan_toor(0.3, 100)
    t = np.array([r[0] for r in rec])
    xi2 = np.array([r[1] for r in rec])
    J2 = np.array([r[2] for r in rec])
    g2 = np.array([r[3] for r in rec])
    i = xi2.argmin()
    assert abs(xi2[i] - g["duncan_toor_xi2_min"]) < 2e-3
    assert abs(t[i] - g["duncan_toor_t_at_min"]) < 0.03
    # species totals: the means stay at the printed equilibria
    np.testing.assert_allclose(rec[-1][4][:2], [g["duncan_toor_xi1_eq"], g["duncan_toor_xi2_eq"]], atol=1e-12)
    # Sec. 4.2: reverse diffusion (-J2 dxi2/dx < 0) on (0, t1) and (t2, t3), osmotic
    # diffusion (gradient zero, flux not) at t1 and t2, a barrier (flux zero,
    # gradient not) at t3.
    g_flip = np.where(np.diff(np.sign(g2)) != 0)[0]
    j_flip = np.where(np.diff(np.sign(J2)) != 0)[0]
    assert len(g_flip) == 2 and len(j_flip) == 1
    t1, t2, t3 = t[g_flip[0]], t[g_flip[1]], t[j_flip[0]]
    assert t1 < t2 < t3
    reverse = -J2 * g2 < 0
    assert reverse[(t < t1)].all()
    assert reverse[(t > t2 + 0.002) & (t < t3 - 0.002)].all()
    assert not reverse[(t > t1 + 0.002) & (t < t2 - 0.002)].any()
    # at the osmotic times the flux, and at the barrier the gradient, is far from zero
    for i in g_flip:
        assert abs(J2[i]) > 0.05 * np.abs(J2).max()
    assert abs(g2[j_flip[0]]) > 0.05 * np.abs(g2).max()


@pytest.mark.slow
def test_loschmidt_tube_extremum_time():
    """Sec. 4.3: reduced D = 0.2157, 0.7716, 0.8335 on [-1, 1] (y), zero flux at y = +-1,
    upper half (0.515, 0.485, 0), lower half (0, 0.509, 0.491); the bottom-half average of
    xi_2 peaks at t* = 0.35 h with t_ref = L_ref^2 s/cm^2, L_ref = 100 pi sqrt(1/60) cm.
    The average is taken over the half-domain (reading of the printed integral)."""
    g = _read_ternary()
    n, dt = 200, 3e-5
    dx = 2.0 / n
    Dp = np.array([[1, 0.2157, 0.7716], [0.2157, 1, 0.8335], [0.7716, 0.8335, 1.0]])
    Dl = Dp * dt / dx ** 2
    np.fill_diagonal(Dl, 1.0)
    t_ref_h = (100 * np.pi * np.sqrt(1 / 60)) ** 2 / 3600.0
    p = lbm.Problem("D2Q5", Dl, (1, n), bc=((lbm.PERIODIC, lbm.PERIODIC), (lbm.ZERO_FLUX, lbm.ZERO_FLUX)))
    y = lbm.cell_centres(n, -1.0, 1.0)
    top = y >= 0
    x1 = np.where(top, 0.515, 0.0)
    x2 = np.where(top, 0.485, 0.509)
    f = lbm.init(p, np.stack([x1, x2, 1 - x1 - x2])[:, :, None])
    ts, bot = [], []
    for s in range(1, int(round(0.45 / t_ref_h / dt)) + 1):
        f = lbm.step(p, f)
        if s % 100 == 0:
            xi = lbm.mole_fractions(f)
            ts.append(s * dt * t_ref_h)
            bot.append(xi[1, ~top, 0].mean())
    i = int(np.argmax(bot))
    assert 0 < i < len(bot) - 1
    assert abs(ts[i] - g["loschmidt_tstar_hours"]) < 0.05
    means = lbm.mole_fractions(f).reshape(3, -1).mean(axis=1)
    np.testing.assert_allclose(means[:2], [g["loschmidt_xi1_eq"], g["loschmidt_xi2_eq"]], atol=1e-12)


@pytest.mark.parametrize("name", ["D1Q2", "D1Q3", "D2Q4", "D2Q5", "D3Q6", "D3Q7", "D2Q9", "D3Q15"])
def test_binary_fourier_decay_matches_continuum(name):
    """Eq. (2-13) with constant D (Remark I): a mode cos(k x) decays as exp(-D k^2 t)."""
    L = lat.get(name)
    # D1Q2 (c_s^2 = 1) runs this D at lambda_1 = 1.82, where the O(k^2) lattice
    # correction is about twice that of the other lattices: a longer wave
    n = 96 if name == "D1Q2" else 64
    shape = {1: (n,), 2: (n, 2), 3: (n, 2, 2)}[int(name[1])]
    d_lat = 0.05
    p = lbm.Problem(name, np.array([[1, d_lat], [d_lat, 1.0]]), shape)
    k = 2 * np.pi / n
    x = np.arange(n)
    A = 0.1
    x1 = np.broadcast_to(0.5 + A * np.cos(k * x), p.nodes)
    steps = 400
    f = lbm.run(p, np.stack([x1, 1 - x1]), steps)
    xi = lbm.mole_fractions(f)[0].reshape(-1, n)[0]
    amp = 2 * np.mean((xi - 0.5) * np.cos(k * x))
    # O(k^2) lattice corrections: k^2 = 0.0096 here; a wrong sound speed would be off by 30 %
    assert abs(amp / (A * np.exp(-d_lat * k * k * steps)) - 1) < 2e-3
    del L


@pytest.mark.parametrize("name", ["D1Q2", "D1Q3", "D2Q4", "D2Q5", "D3Q6", "D3Q7", "D2Q9", "D3Q15"])
@pytest.mark.parametrize("relax", [ms.RELAX_PAPER, ms.RELAX_SRT, ms.RELAX_TRT])
def test_linearised_multicomponent_decay_matches_eigen_decomposition(name, relax):
    """Linearised Eq. (2-13) (D~ frozen at a reference composition): a mode with
    amplitude vector a0 evolves as a(t) = exp(-k^2 D~ t) a0, coupling included."""
    n = 64 if name == "D1Q2" else 48      # D1Q2: larger O(k^2) correction (see above)
    shape = {1: (n,), 2: (n, 2), 3: (n, 2, 2)}[int(name[1])]
    D = np.array([[1, 0.02, 0.09, 0.05], [0.02, 1, 0.04, 0.08], [0.09, 0.04, 1, 0.03], [0.05, 0.08, 0.03, 1.0]])
    xref = np.array([0.3, 0.2, 0.1, 0.4])
    # TRT: the even parameter does not enter the continuum limit (only lambda_1 sets D~)
    p = lbm.Problem(name, D, shape, xi_ref=xref, relax=relax, magic=0.45)
    k = 2 * np.pi / n
    x = np.arange(n)
    a0 = np.array([0.02, -0.03, 0.01])
    xi0 = np.empty((4,) + p.nodes)
    for i in range(3):
        xi0[i] = np.broadcast_to(xref[i] + a0[i] * np.cos(k * x), p.nodes)
    xi0[3] = 1 - xi0[:3].sum(0)
    steps = 300
    xi = lbm.mole_fractions(lbm.run(p, xi0, steps))[:3].reshape(3, -1, n)[:, 0]
    amp = 2 * np.mean((xi - xref[:3, None]) * np.cos(k * x)[None], axis=1)
    Dt = np.linalg.inv(ms.ms_B(xref, D))
    expect = expm(-k * k * Dt * steps) @ a0
    # lattice corrections are O(k^2) = 2e-3 relative; a transposed D~ is off by ~5e-2
    np.testing.assert_allclose(amp, expect, rtol=0, atol=3e-3 * np.abs(a0).max())


def test_small_amplitude_nonlinear_decay_matches_linearised_theory():
    """Full nonlinear model with a 1e-4 perturbation about xi_bar evolves like the
    linearised theory about xi_bar (Sec. 1) to O(amplitude)."""
    n = 48
    D = np.array([[1, 0.02, 0.09], [0.02, 1, 0.04], [0.09, 0.04, 1.0]])
    xbar = np.array([0.3, 0.5, 0.2])
    p = lbm.Problem("D2Q5", D, (n, 2))
    k = 2 * np.pi / n
    x = np.arange(n)
    a0 = np.array([1e-4, -2e-4])
    xi0 = np.empty((3,) + p.nodes)
    for i in range(2):
        xi0[i] = np.broadcast_to(xbar[i] + a0[i] * np.cos(k * x), p.nodes)
    xi0[2] = 1 - xi0[:2].sum(0)
    steps = 300
    xi = lbm.mole_fractions(lbm.run(p, xi0, steps))[:2].reshape(2, -1, n)[:, 0]
    amp = 2 * np.mean((xi - xbar[:2, None]) * np.cos(k * x)[None], axis=1)
    expect = expm(-k * k * np.linalg.inv(ms.ms_B(xbar, D)) * steps) @ a0
    np.testing.assert_allclose(amp, expect, rtol=0, atol=5e-3 * np.abs(a0).max())


_ORIGINAL_LAMBDA2 = ms.lambda2_from_lambda1


def _lambda2_rule_dropped(L1, rule=ms.RELAX_PAPER, magic=ms.MAGIC_PAPER):
    return np.array(L1, dtype=np.float64, copy=True)


def _lambda2_wrong_product(L1, rule=ms.RELAX_PAPER, magic=ms.MAGIC_PAPER):
    return _ORIGINAL_LAMBDA2(L1, ms.RELAX_TRT if rule == ms.RELAX_PAPER else rule, 0.25)


@pytest.mark.parametrize("mistake", [_lambda2_rule_dropped, _lambda2_wrong_product])
def test_table_I_pin_catches_planted_mistakes(monkeypatch, mistake):
    """The Table I pin of the MRT model fails when the oracle's Lambda_2 carries a
    plausible mistake: Eq. (3-16) dropped (Lambda_2 = Lambda_1, the SRT model), or
    the product rule taken with 1/4 instead of 3/16."""
    monkeypatch.setattr(ms, "lambda2_from_lambda1", mistake)
    with pytest.raises(AssertionError):
        test_table_I_errors("MRT", ms.RELAX_PAPER)


_ORIGINAL_LAMBDA1 = ms.lambda1_from_fick


def _lambda1_with_one_third_on_d3q7(Dt, cs2, dt=1.0):
    # Eq. (3-26) inverted with c_s^2 = 1/3 where the D3Q7 lattice has 1/4
    return _ORIGINAL_LAMBDA1(Dt, 1.0 / 3.0 if cs2 == 0.25 else cs2, dt)


def test_continuum_decay_pin_catches_a_planted_sound_speed(monkeypatch):
    """The continuum-decay pin on D3Q7 fails when the oracle inverts Eq. (3-26)
    with the c_s^2 = 1/3 of the other lattices instead of the D3Q7 lattice's own
    second moment of the weights, 1/4."""
    monkeypatch.setattr(ms, "lambda1_from_fick", _lambda1_with_one_third_on_d3q7)
    with pytest.raises(AssertionError):
        test_binary_fourier_decay_matches_continuum("D3Q7")
    test_binary_fourier_decay_matches_continuum("D2Q5")   # lattices with 1/3 are unaffected


_ORIGINAL_FICK = ms.fick_matrix


def _fick_matrix_transposed(B):
    return np.swapaxes(_ORIGINAL_FICK(B), -1, -2).copy()


def test_linearised_decay_pin_catches_a_transposed_fick_matrix(monkeypatch):
    """The linearised-decay pin fails when the oracle's D~ = B^-1 of Eq. (2-11)
    is transposed (the cross terms then couple the wrong pairs)."""
    monkeypatch.setattr(ms, "fick_matrix", _fick_matrix_transposed)
    with pytest.raises(AssertionError):
        test_linearised_multicomponent_decay_matches_eigen_decomposition("D2Q5", ms.RELAX_PAPER)
