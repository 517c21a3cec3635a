"""Pins of the dilute-species approximation of B (Remark III, Eqs. (2-16), (2-17))
in the oracle: the exact limit it approximates, its continuum dynamics on the
lattice, agreement with the full model for a trace species, and brute force."""
import numpy as np
import pytest

from oracle import lattice as lat
from oracle import lbm, ms, naive

LATS = ["D1Q3", "D2Q5", "D3Q7", "D1Q2", "D2Q4", "D3Q6", "D2Q9", "D3Q15"]


def _rand_D(rng, N, lo=0.05, hi=0.3):
    D = np.ones((N, N))
    for i in range(N):
        for j in range(i + 1, N):
            D[i, j] = D[j, i] = rng.uniform(lo, hi)
    return D


def _shape(name, full):
    return full[: lat.get(name).d]


@pytest.mark.parametrize("N", [3, 4, 6])
def test_exact_fick_row_of_a_vanishing_species_tends_to_the_effective_diffusivity(N):
    """Remark III: as xi_i -> 0 the row i of the exact D~ = B^-1 (Eq. (2-10))
    becomes D_eff,i e_i, with D_eff,i = 1 / B_ii of the dilute B.  The error is
    linear in xi_i (checked at two values a factor 100 apart)."""
    rng = np.random.default_rng(500 + N)
    D = _rand_D(rng, N)
    for i in range(N - 1):
        errs = []
        for eps in (1e-4, 1e-6):
            x = rng.uniform(0.2, 1.0, N)
            x[i] = 0.0
            x *= (1 - eps) / x.sum()
            x[i] = eps
            exact = np.linalg.inv(ms.ms_B(x, D))
            dil = np.linalg.inv(ms.ms_B_dilute(x, D))
            d_eff = dil[i, i]
            row = exact[i].copy()
            errs.append(max(abs(row[i] / d_eff - 1), np.abs(np.delete(row, i)).max() / d_eff))
            # the dilute matrix is diagonal
            assert np.count_nonzero(dil - np.diag(np.diag(dil))) == 0
        assert errs[1] < 1e-4, errs
        assert errs[1] < errs[0] / 20, errs


@pytest.mark.parametrize("name", ["D1Q3", "D2Q5", "D3Q7", "D2Q9", "D3Q15"])
def test_dilute_mode_mode_decays_with_effective_diffusivity(name):
    """Dilute mode on the lattice: a small cosine mode of species 1 on a uniform
    background (balanced by the last species) decays as exp(-D_eff k^2 t) with
    D_eff = 1 / sum_k xbar_k / D_1k; the other evolved species stay uniform
    (each species relaxes alone)."""
    n = 48
    shape = {1: (n,), 2: (n, 2), 3: (n, 2, 2)}[lat.get(name).d]
    D = np.array([[1, 0.02, 0.09, 0.05], [0.02, 1, 0.04, 0.08], [0.09, 0.04, 1, 0.03], [0.05, 0.08, 0.03, 1.0]])
    xbar = np.array([0.3, 0.2, 0.1, 0.4])
    p = lbm.Problem(name, D, shape, dilute=True)
    k = 2 * np.pi / n
    x = np.arange(n)
    A = 1e-4
    xi0 = np.empty((4,) + p.nodes)
    for i in range(4):
        xi0[i] = xbar[i]
    xi0[0] = np.broadcast_to(xbar[0] + A * np.cos(k * x), p.nodes)
    xi0[3] = 1 - xi0[:3].sum(0)
    steps = 300
    xi = lbm.mole_fractions(lbm.run(p, xi0, steps))
    row = xi[0].reshape(-1, n)[0]
    amp = 2 * np.mean((row - xbar[0]) * np.cos(k * x))
    d_eff = 1.0 / (xbar[1] / D[0, 1] + xbar[2] / D[0, 2] + xbar[3] / D[0, 3])
    # O(k^2) lattice corrections (~2e-3) and O(A) nonlinearity; the full model's
    # D~_11 differs from D_eff by 10 % here
    assert abs(amp / (A * np.exp(-d_eff * k * k * steps)) - 1) < 5e-3
    np.testing.assert_allclose(xi[1], xbar[1], rtol=0, atol=1e-15)
    np.testing.assert_allclose(xi[2], xbar[2], rtol=0, atol=1e-15)


@pytest.mark.parametrize("name", ["D2Q5", "D3Q7", "D2Q9"])
def test_dilute_mode_matches_full_model_for_a_trace_species(name):
    """A trace species (background 1e-6, perturbation 1e-8) evolves the same in
    the dilute and the full model up to O(1e-6) relative: the regime Remark III
    is stated for."""
    rng = np.random.default_rng(17)
    N = 4
    D = _rand_D(rng, N)
    shape = _shape(name, (24, 10, 6))
    p_full = lbm.Problem(name, D, shape, bc=tuple((lbm.ZERO_FLUX, lbm.ZERO_FLUX) for _ in shape))
    p_dil = lbm.Problem(name, D, shape, bc=p_full.bc, dilute=True)
    xi0 = np.empty((N,) + p_full.nodes)
    xi0[1] = 0.3
    xi0[2] = 0.25
    xi0[0] = 1e-6 + 1e-8 * rng.uniform(-1, 1, p_full.nodes)
    xi0[3] = 1 - xi0[:3].sum(0)
    a = lbm.mole_fractions(lbm.run(p_full, xi0, 40))[0]
    b = lbm.mole_fractions(lbm.run(p_dil, xi0, 40))[0]
    pert = a - 1e-6
    assert np.abs(pert).max() > 1e-10          # the perturbation is still there
    assert np.abs(b - a).max() <= 1e-5 * np.abs(pert).max()


@pytest.mark.parametrize("name", LATS)
def test_dilute_vectorised_matches_scalar_loops(name):
    """Brute force in dilute mode, every face kind, also with the linearised theory."""
    rng = np.random.default_rng(len(name) + 40)
    N = 4
    shape = _shape(name, (5, 4, 3))
    d = len(shape)
    kinds = [(lbm.ZERO_FLUX, lbm.DIRICHLET), (lbm.PERIODIC, lbm.PERIODIC), (lbm.DIRICHLET, lbm.ZERO_FLUX)]
    bc = tuple(kinds[a] for a in range(d))
    walls = {(a, s): rng.dirichlet(np.ones(N)) for a in range(d) for s in (0, 1) if bc[a][s] == lbm.DIRICHLET}
    D = _rand_D(rng, N)
    xi0 = rng.dirichlet(np.ones(N), size=tuple(reversed(shape))).transpose((d,) + tuple(range(d)))
    for xref in (None, np.array([0.2, 0.3, 0.1, 0.4])):
        p = lbm.Problem(name, D, shape, bc=bc, xi_wall=walls, dilute=True, xi_ref=xref)
        np.testing.assert_allclose(lbm.run(p, xi0, 4), naive.run(p, xi0, 4), rtol=0, atol=1e-14)
