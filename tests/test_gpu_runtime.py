"""GPU tests of the runtime around the sweep: conservation diagnostics,
checkpoint/restore, error paths, and the paper's binary benchmark (Table I)
reproduced by the HIP path with Dirichlet faces."""
import os

import numpy as np
import pytest
import torch

from gpu_cases import gpu_run, oracle_problem, rand_D, smooth_field
from oracle import lbm

pytestmark = pytest.mark.gpu


def _sim(lattice, D, shape, precision, xi0, **kw):
    from paper_1808_06787_amd.sim import Sim

    s = Sim(lattice, D, shape, precision, **kw)
    s.init(torch.from_numpy(np.ascontiguousarray(xi0)))
    return s


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("lattice,shape,bc", [
    ("D2Q5", (120, 77), None),
    ("D3Q7", (40, 21, 13), (("zero_flux", "zero_flux"), ("periodic", "periodic"), ("periodic", "periodic"))),
])
def test_diagnostics_match_oracle_and_conserve(precision, lattice, shape, bc):
    rng = np.random.default_rng(12)
    N = 4
    D = rand_D(rng, N)
    xi0 = smooth_field(rng, N, shape[::-1], 0.15)
    s = _sim(lattice, D, shape, precision, xi0, bc=bc)
    mass0, mn0, mx0, bad0 = s.diagnostics()
    s.step(80)
    mass, mn, mx, bad = s.diagnostics()
    p = oracle_problem(lattice, D, shape, bc=bc)
    f = lbm.run(p, xi0, 80)
    om, omn, omx, obad = lbm.diagnostics(p, f)
    total = xi0.reshape(N, -1).sum(1)
    rel = 1e-12 if precision == "f64" else 2e-6
    np.testing.assert_allclose(mass0, total, rtol=rel)
    np.testing.assert_allclose(mass, total, rtol=rel)       # Eq. (2-1): closed domain
    np.testing.assert_allclose(mass, om, rtol=rel)
    tol = 1e-12 if precision == "f64" else 1e-5
    np.testing.assert_allclose(mn, omn, atol=tol)
    np.testing.assert_allclose(mx, omx, atol=tol)
    assert bad == 0 and bad0 == 0
    s.close()


def test_diagnostics_flag_non_finite_input():
    from paper_1808_06787_amd._ffi import MsdError

    rng = np.random.default_rng(13)
    D = rand_D(rng, 3)
    xi0 = smooth_field(rng, 3, (30, 40), 0.1)
    xi0[0, 3, 5] = np.nan
    s = _sim("D2Q5", D, (40, 30), "f32", xi0)
    s.step(3)
    with pytest.raises(MsdError) as e:
        s.diagnostics()
    assert e.value.status == -6
    _, _, _, bad = s.diagnostics(raise_on_diverged=False)
    assert bad > 0
    s.close()


def test_diagnostics_flag_negative_mole_fractions():
    """A mole fraction below -neg_tol (default 1e-2) is divergence; the check can
    be loosened or turned off."""
    from paper_1808_06787_amd._ffi import MsdError

    rng = np.random.default_rng(14)
    D = rand_D(rng, 3)
    xi0 = smooth_field(rng, 3, (30, 40), 0.1)
    xi0[0, 3, 5] = -0.2
    xi0[1, 3, 5] = 1.2 - xi0[2, 3, 5]
    s = _sim("D2Q5", D, (40, 30), "f32", xi0)
    with pytest.raises(MsdError) as e:
        s.diagnostics()
    assert e.value.status == -6 and "species 1" in str(e.value)
    s.set_health(neg_tol=0.5)
    s.diagnostics()
    s.set_health(neg_tol=-1.0)
    s.diagnostics()
    s.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_diagnostics_flag_species_total_drift(precision):
    """Species totals are conserved with periodic and zero-flux faces (Eq. (2-1));
    restoring a state with other totals (forced from the host) is drift past
    mass_rtol per node.  With a Dirichlet face, which exchanges species with the
    outside, the drift check is off."""
    from paper_1808_06787_amd._ffi import MsdError

    rng = np.random.default_rng(15)
    D = rand_D(rng, 3)
    shape = (40, 30)
    a = _sim("D2Q5", D, shape, precision, smooth_field(rng, 3, shape[::-1], 0.1))
    other = smooth_field(rng, 3, shape[::-1], 0.1)
    other[0] *= 0.9
    other[1] = 1.0 - other[0] - other[2]
    b = _sim("D2Q5", D, shape, precision, other)
    a.step(7)
    a.diagnostics()                  # conserved: no error
    state, t = b.save()
    a.restore(state, t)
    with pytest.raises(MsdError) as e:
        a.diagnostics()
    assert e.value.status == -6 and "drifted" in str(e.value)
    a.set_health(mass_rtol=-1.0)
    a.diagnostics()
    a.close()
    b.close()
    bc = (("dirichlet", "zero_flux"), ("periodic", "periodic"))
    walls = {(0, 0): np.array([0.8, 0.1, 0.1])}
    c = _sim("D2Q5", D, shape, precision, smooth_field(rng, 3, shape[::-1], 0.1), bc=bc, xi_wall=walls)
    c.step(200)
    c.diagnostics()                  # totals change through the Dirichlet face
    c.close()


def test_create_warns_where_the_relaxation_does_not_damp():
    """A Dirichlet face at a composition where Eq. (3-16) gives rho(I - Lambda_2) > 1."""
    from paper_1808_06787_amd.sim import Sim
    from test_stability_cpu import UNSTABLE_D, UNSTABLE_XI

    bc = (("dirichlet", "zero_flux"), ("periodic", "periodic"), ("periodic", "periodic"))
    with pytest.warns(RuntimeWarning, match="does not damp"):
        s = Sim("D3Q7", UNSTABLE_D, (8, 8, 8), "f32", bc=bc, xi_wall={(0, 0): UNSTABLE_XI})
    r1, r2 = s.stability()
    assert r2 > 1.0
    s.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_checkpoint_restore_is_bitwise(precision):
    rng = np.random.default_rng(14)
    D = rand_D(rng, 3)
    shape = (90, 50)
    xi0 = smooth_field(rng, 3, shape[::-1], 0.1)
    a = _sim("D2Q5", D, shape, precision, xi0)
    a.step(40)
    ref, _, _ = a.read()
    b = _sim("D2Q5", D, shape, precision, xi0)
    b.step(20)
    state, t = b.save()
    assert t == 20
    b.step(5)                       # wander off, then come back
    b.restore(state, t)
    assert b.time == 20
    b.step(20)
    got, _, _ = b.read()
    torch.testing.assert_close(got, ref, rtol=0, atol=0)
    # restore into a fresh handle
    c = _sim("D2Q5", D, shape, precision, np.full_like(xi0, 1 / 3))
    c.restore(state, 20)
    c.step(20)
    got2, _, _ = c.read()
    torch.testing.assert_close(got2, ref, rtol=0, atol=0)
    for s in (a, b, c):
        s.close()


def test_step_before_init_is_an_error():
    from paper_1808_06787_amd._ffi import MsdError
    from paper_1808_06787_amd.sim import Sim

    s = Sim("D1Q3", np.array([[1, 0.1], [0.1, 1.0]]), (16,), "f64")
    with pytest.raises(MsdError) as e:
        s.step(1)
    assert e.value.status == -9
    with pytest.raises(MsdError):
        s.read()
    s.close()


def test_table_I_on_the_gpu():
    """The binary erf problem of Sec. 4.1 (240 x 40 D2Q5, Dirichlet anti-bounce-back
    walls, lambda_1 = 1.25) run by the HIP path in FP64: matches the oracle to 1e-12
    and reproduces the printed MRT and SRT errors of Table I to 0.5 %."""
    from scipy.special import erf

    golden = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "table1.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                mdl, t, a, b = line.split()
                golden[(mdl, int(t))] = (float(a), float(b))
    Dphys, C0, C1, nx, ny = 0.05, 0.9, 0.1, 240, 40
    dx = 12.0 / nx
    d_lat = (1.0 / 3.0) * (1.0 / 1.25 - 0.5)
    dt = d_lat * dx * dx / Dphys
    D = np.array([[1.0, d_lat], [d_lat, 1.0]])
    x = lbm.cell_centres(nx, -6.0, 6.0)
    x1 = np.tile(np.where(x < 0, C0, C1), (ny, 1))
    xi0 = np.stack([x1, 1 - x1])
    bc = (("dirichlet", "dirichlet"), ("periodic", "periodic"))
    walls = {(0, 0): [C0, 1 - C0], (0, 1): [C1, 1 - C1]}
    from paper_1808_06787_amd.sim import Sim

    for model, relax in (("MRT", "paper"), ("SRT", "srt")):
        s = Sim("D2Q5", D, (nx, ny), "f64", bc=bc, xi_wall=walls, relax=relax)
        s.init(torch.from_numpy(xi0))
        p = oracle_problem("D2Q5", D, (nx, 4), bc=bc, xi_wall={k: np.array(v) for k, v in walls.items()},
                           relax=relax)
        f = lbm.init(p, xi0[:, :4])
        for T in (1, 5, 20):
            n = int(round(T / dt))
            s.step(n - s.time)
            xi, J, _ = s.read()
            xi = xi.cpu().numpy()
            J = J.cpu().numpy()
            assert np.abs(xi[0] - xi[0, :1]).max() == 0.0        # uniform in y
            xa = (C0 + C1) / 2 + (C1 - C0) / 2 * erf(x / (2 * np.sqrt(Dphys * T)))
            Ja = -(C1 - C0) / 2 * np.sqrt(Dphys / (np.pi * T)) * np.exp(-x * x / (4 * Dphys * T))
            e_xi = lbm.rel_l2_error(xa, xi[0, 0])
            e_j = lbm.rel_l2_error(Ja, J[0, 0, 0] * dx / dt)
            ref_xi, ref_j = golden[(model, T)]
            assert abs(e_xi / ref_xi - 1) < 5e-3, (model, T, e_xi, ref_xi)
            assert abs(e_j / ref_j - 1) < 5e-3, (model, T, e_j, ref_j)
            if T == 1:
                for _ in range(n):
                    f = lbm.step(p, f)
                oxi, _, oJ = lbm.observables(p, f)
                np.testing.assert_allclose(xi[:, :4], oxi, rtol=0, atol=1e-12)
                np.testing.assert_allclose(J[:, :, :4], oJ, rtol=0, atol=1e-12 * np.abs(oJ).max())
        s.close()


@pytest.mark.parametrize("lattice,shape", [("D2Q9", (200, 90)), ("D3Q15", (40, 30, 20))])
def test_sim_autotuner_on_diagonal_lattices(tmp_path, lattice, shape):
    """The library's candidate list on lattices with diagonal directions has no
    vector widths (that kernel is axial only); the tuned run continues as if untuned."""
    from paper_1808_06787_amd import autotune

    rng = np.random.default_rng(77)
    D = rand_D(rng, 3)
    xi0 = smooth_field(rng, 3, shape[::-1], 0.1)
    ref = _sim(lattice, D, shape, "f64", xi0)
    ref.step(9)
    want = ref.read()[0].cpu().numpy()
    ref.close()
    s = _sim(lattice, D, shape, "f64", xi0)
    s.step(4)
    res = autotune.tune_sim(s, cache_path=str(tmp_path / "tune.txt"), steps=2)
    # 5 tile shapes x XCD remapping on/off x streaming hints on/off, no vector widths
    assert len(res["trials"]) == 20 and res["best"]["vec"] == 0
    assert s.time == 4 and s.get_launch() == res["best"]
    s.step(5)
    np.testing.assert_allclose(s.read()[0].cpu().numpy(), want, rtol=0, atol=1e-14)
    s.close()


def test_sim_autotuner_keeps_state_and_caches(tmp_path):
    """msd_tune times candidate launches from a saved state and restores it: the
    run continues as if untuned (to FP32 rounding: the chosen launch may take
    passes of another length); a second call is served by the cache."""
    from paper_1808_06787_amd import autotune

    rng = np.random.default_rng(76)
    D = rand_D(rng, 3)
    shape = (600, 300)
    xi0 = smooth_field(rng, 3, shape[::-1], 0.1)
    ref = _sim("D2Q5", D, shape, "f32", xi0)
    ref.step(17)
    want = ref.read()[0].cpu().numpy()
    ref.close()
    s = _sim("D2Q5", D, shape, "f32", xi0)
    s.step(5)
    cache = str(tmp_path / "tune.txt")
    res = autotune.tune_sim(s, cache_path=cache, steps=2)
    assert s.time == 5 and len(res["trials"]) > 20 and s.get_launch() == res["best"]
    s.step(12)
    np.testing.assert_allclose(s.read()[0].cpu().numpy(), want, rtol=0, atol=2e-6)
    res2 = autotune.tune_sim(s, cache_path=cache)
    assert res2["best"] == res["best"] and res2["trials"] == []
    res3 = autotune.tune_sim(s, cache_path=cache, steps=2, force=True,
                             candidates=[dict(temporal=0, block_x=128, block_y=2), dict(temporal=2, seg_rows=8)])
    assert len(res3["trials"]) == 2 and s.get_launch() == res3["best"]
    s.close()
