"""Pins of the oracle's full collide-and-stream step.

* brute force: the vectorised oracle against the scalar-loop one on tiny grids;
* exact reductions: SRT with Lambda = I is the explicit weighted-average scheme;
* exact discrete Fourier evolution of linear cases, built from the odd/even
  projector form of the collision (an algebraically different route from the
  oracle's moment-matrix one);
* exact symmetries: half-way bounce-back equals a mirrored periodic domain;
  anti-bounce-back equals an antisymmetric periodic extension (linear case);
  relabelling the eliminated species is invisible under SRT;
* conservation of every species' total (Eq. (2-1)) and the steady state.
"""
import dataclasses

import numpy as np
import pytest

from oracle import lbm, ms, naive
from oracle import lattice as lat

LATS = ["D1Q2", "D1Q3", "D2Q4", "D2Q5", "D3Q6", "D3Q7", "D2Q9", "D3Q15"]
# lattices whose moving directions each follow one axis: there half-way bounce-back
# is a mirror, so a walled domain equals a mirrored periodic one
AXIAL = ["D1Q2", "D1Q3", "D2Q4", "D2Q5", "D3Q6", "D3Q7"]


def _rand_D(rng, n, lo, hi):
    D = np.ones((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            D[i, j] = D[j, i] = np.exp(rng.uniform(np.log(lo), np.log(hi)))
    return D


def _rand_field(rng, N, nodes, base_lo=0.2):
    x = rng.uniform(base_lo, 1.0, size=(N,) + tuple(nodes))
    return x / x.sum(axis=0, keepdims=True)


def _shape(name, sizes):
    return sizes[: int(name[1])]


@pytest.mark.parametrize("name", LATS)
@pytest.mark.parametrize("relax", [ms.RELAX_PAPER, ms.RELAX_SRT])
def test_vectorised_matches_scalar_loops(name, relax):
    """Brute force: both oracle implementations agree on tiny grids with every face kind."""
    rng = np.random.default_rng(hash((name, relax)) % 2**32)
    N = 4
    shape = _shape(name, (5, 4, 3))
    d = len(shape)
    kinds = [(lbm.ZERO_FLUX, lbm.DIRICHLET), (lbm.PERIODIC, lbm.PERIODIC), (lbm.DIRICHLET, lbm.ZERO_FLUX)]
    bc = tuple(kinds[a] for a in range(d))
    walls = {}
    for a in range(d):
        for s in (0, 1):
            if bc[a][s] == lbm.DIRICHLET:
                walls[(a, s)] = _rand_field(rng, N, ())
    D = _rand_D(rng, N, 0.05, 0.3)
    p = lbm.Problem(name, D, shape, bc=bc, xi_wall=walls, relax=relax)
    xi0 = _rand_field(rng, N, p.nodes)
    a = lbm.run(p, xi0, 4)
    b = naive.run(p, xi0, 4)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)


@pytest.mark.parametrize("name", LATS)
@pytest.mark.parametrize("magic", [0.1, 0.6])
def test_vectorised_matches_scalar_loops_trt(name, magic):
    """TRT: the vectorised oracle (closed form of lambda_2) and the scalar loops (lambda_2
    solved from the defining product) agree."""
    rng = np.random.default_rng(int(magic * 1000) + len(name))
    N = 3
    shape = _shape(name, (5, 4, 3))
    d = len(shape)
    kinds = [(lbm.ZERO_FLUX, lbm.DIRICHLET), (lbm.PERIODIC, lbm.PERIODIC), (lbm.DIRICHLET, lbm.ZERO_FLUX)]
    bc = tuple(kinds[a] for a in range(d))
    walls = {(a, s): _rand_field(rng, N, ()) for a in range(d) for s in (0, 1) if bc[a][s] == lbm.DIRICHLET}
    D = _rand_D(rng, N, 0.05, 0.3)
    p = lbm.Problem(name, D, shape, bc=bc, xi_wall=walls, relax=ms.RELAX_TRT, magic=magic)
    xi0 = _rand_field(rng, N, p.nodes)
    np.testing.assert_allclose(lbm.run(p, xi0, 4), naive.run(p, xi0, 4), rtol=0, atol=1e-14)


@pytest.mark.parametrize("name", LATS)
def test_vectorised_matches_scalar_loops_linearised(name):
    rng = np.random.default_rng(7)
    N = 3
    D = _rand_D(rng, N, 0.05, 0.3)
    p = lbm.Problem(name, D, _shape(name, (4, 3, 3)), xi_ref=np.array([0.2, 0.5, 0.3]))
    xi0 = _rand_field(rng, N, p.nodes)
    np.testing.assert_allclose(lbm.run(p, xi0, 3), naive.run(p, xi0, 3), rtol=0, atol=1e-14)


@pytest.mark.parametrize("name", LATS)
def test_srt_unit_relaxation_is_weighted_average_scheme(name):
    """SRT with Lambda_1 = I (all D_ij = cs2/2, so that Eq. (3-26) gives Lambda_1 = I)
    relaxes f fully to w xi (Eq. (3-3)); after streaming
    xi(x, t+1) = sum_k w_k xi(x - c_k, t) exactly, for every species."""
    L = lat.get(name)
    N = 4
    D = np.full((N, N), L.cs2 / 2)
    p = lbm.Problem(name, D, _shape(name, (9, 7, 5)), relax=ms.RELAX_SRT)
    rng = np.random.default_rng(3)
    xi = _rand_field(rng, N, p.nodes)
    f = lbm.init(p, xi)
    for _ in range(6):
        f = lbm.step(p, f)
        nxt = np.zeros_like(xi)
        for k in range(L.q):
            shifted = xi
            for a in range(L.d):
                if L.c[k, a]:
                    shifted = np.roll(shifted, int(L.c[k, a]), axis=1 + (L.d - 1 - a))
            nxt += L.w[k] * shifted
        xi = nxt
        np.testing.assert_allclose(lbm.mole_fractions(f), xi, rtol=0, atol=2e-15)


def _trt_collision_matrix(L, L1, L2):
    """Collision as a (m q) x (m q) matrix from the odd/even projectors:
    f+ = f - L1 . odd(f - w xi) - L2 . even(f - w xi)."""
    q = L.q
    m = L1.shape[0]
    opp = L.opposite
    Pk = np.eye(q)[opp]
    Po = 0.5 * (np.eye(q) - Pk)
    Pe = 0.5 * (np.eye(q) + Pk)
    E = np.eye(q) - np.outer(L.w, np.ones(q))      # f -> f - w sum(f)
    return np.eye(m * q) - np.kron(L1, Po @ E) - np.kron(L2, Pe @ E)


@pytest.mark.parametrize("name", LATS)
@pytest.mark.parametrize("relax", [ms.RELAX_PAPER, ms.RELAX_SRT, ms.RELAX_TRT])
def test_exact_discrete_fourier_evolution_linear(name, relax):
    """Linearised (constant-B) case: a single Fourier mode evolves exactly by the
    amplification matrix G = S(k) C, S = diag(exp(-i k.c_k)) (Eq. (3-2) with pull
    propagation), C the collision matrix in projector form."""
    L = lat.get(name)
    rng = np.random.default_rng(21)
    N = 4
    D = _rand_D(rng, N, 0.03, 0.3)
    xref = np.array([0.1, 0.2, 0.3, 0.4])
    shape = _shape(name, (12, 8, 6))
    magic = 0.07       # TRT case: a parameter far from Eq. (3-16)'s 3/16
    p = lbm.Problem(name, D, shape, relax=relax, xi_ref=xref, magic=magic)
    B = ms.ms_B(xref, D)
    L1 = ms.lambda1_from_fick(np.linalg.inv(B), L.cs2)
    L2 = ms.lambda2_from_lambda1(L1, relax, magic)
    C = _trt_collision_matrix(L, L1, L2)
    kvec = np.array([2 * np.pi * (a + 1) / shape[a] for a in range(L.d)])
    S = np.kron(np.eye(N - 1), np.diag(np.exp(-1j * (L.c[:, : L.d] @ kvec))))
    G = S @ C
    amp = rng.uniform(-0.05, 0.05, N - 1)
    grids = np.meshgrid(*[np.arange(s) for s in shape[::-1]], indexing="ij")   # (z, y, x)
    phase = sum(kvec[a] * grids[L.d - 1 - a] for a in range(L.d))
    xi0 = np.empty((N,) + p.nodes)
    for i in range(N - 1):
        xi0[i] = xref[i] + amp[i] * np.cos(phase)
    xi0[-1] = 1 - xi0[:-1].sum(0)
    a = np.kron(amp, L.w).astype(complex)
    f = lbm.init(p, xi0)
    for _ in range(15):
        f = lbm.step(p, f)
        a = G @ a
    fk = np.real(a.reshape(N - 1, L.q)[:, :, None] * np.exp(1j * phase.ravel())[None, None])
    expect = xref[: N - 1, None, None] * L.w[None, :, None] + fk
    np.testing.assert_allclose(f.reshape(N - 1, L.q, -1), expect, rtol=0, atol=1e-13)


@pytest.mark.parametrize("name", AXIAL)
def test_zero_flux_wall_equals_mirrored_periodic_domain(name):
    """Half-way bounce-back (Sec. 4) at both x faces is exactly a periodic domain of
    twice the length holding the mirror image (nonlinear, paper relaxation rule)."""
    rng = np.random.default_rng(5)
    N = 4
    D = _rand_D(rng, N, 0.03, 0.3)
    shape = _shape(name, (7, 4, 3))
    bc_w = ((lbm.ZERO_FLUX, lbm.ZERO_FLUX),) + ((lbm.PERIODIC, lbm.PERIODIC),) * (len(shape) - 1)
    pw = lbm.Problem(name, D, shape, bc=bc_w)
    pp = lbm.Problem(name, D, (2 * shape[0],) + tuple(shape[1:]))
    xi0 = _rand_field(rng, N, pw.nodes)
    xi0m = np.concatenate([xi0, xi0[..., ::-1]], axis=-1)
    fw = lbm.run(pw, xi0, 25)
    fp = lbm.run(pp, xi0m, 25)
    np.testing.assert_allclose(lbm.mole_fractions(fw), lbm.mole_fractions(fp)[..., : shape[0]],
                               rtol=0, atol=1e-14)


@pytest.mark.parametrize("name", AXIAL)
def test_dirichlet_wall_equals_antisymmetric_extension_linear(name):
    """Half-way anti-bounce-back (Sec. 4) with wall value xi_b at both x faces equals a
    periodic domain of twice the length holding 2 xi_b - (mirror image), for the
    binary (linear) model."""
    rng = np.random.default_rng(6)
    D = np.array([[1.0, 0.11], [0.11, 1.0]])
    shape = _shape(name, (9, 4, 3))
    xb = 0.3
    bc_w = ((lbm.DIRICHLET, lbm.DIRICHLET),) + ((lbm.PERIODIC, lbm.PERIODIC),) * (len(shape) - 1)
    walls = {(0, 0): np.array([xb, 1 - xb]), (0, 1): np.array([xb, 1 - xb])}
    for relax in (ms.RELAX_PAPER, ms.RELAX_SRT):
        pw = lbm.Problem(name, D, shape, bc=bc_w, xi_wall=walls, relax=relax)
        pp = lbm.Problem(name, D, (2 * shape[0],) + tuple(shape[1:]), relax=relax)
        x1 = rng.uniform(0.0, 0.6, size=pw.nodes)
        ext = np.concatenate([x1, 2 * xb - x1[..., ::-1]], axis=-1)
        fw = lbm.run(pw, np.stack([x1, 1 - x1]), 30)
        fp = lbm.run(pp, np.stack([ext, 1 - ext]), 30)
        np.testing.assert_allclose(lbm.mole_fractions(fw)[0], lbm.mole_fractions(fp)[0][..., : shape[0]],
                                   rtol=0, atol=1e-14)


@pytest.mark.parametrize("name", LATS)
def test_srt_relabelling_the_eliminated_species(name):
    """With Lambda_2 = Lambda_1, choosing a different species as the eliminated one
    (Eq. (2-8a) removes J_n) must give the same mixture evolution: B of Eq. (2-10)
    transforms by similarity under that change of basis.  Nonlinear, N = 4."""
    rng = np.random.default_rng(8)
    N = 4
    D = _rand_D(rng, N, 0.03, 0.3)
    shape = _shape(name, (6, 5, 4))
    p = lbm.Problem(name, D, shape, relax=ms.RELAX_SRT)
    xi0 = _rand_field(rng, N, p.nodes)
    base = lbm.mole_fractions(lbm.run(p, xi0, 20))
    for perm in ([1, 2, 3, 0], [0, 3, 2, 1], [3, 1, 0, 2]):
        perm = np.array(perm)
        pp = lbm.Problem(name, D[np.ix_(perm, perm)], shape, relax=ms.RELAX_SRT)
        got = lbm.mole_fractions(lbm.run(pp, xi0[perm], 20))
        np.testing.assert_allclose(got, base[perm], rtol=0, atol=1e-13)


@pytest.mark.parametrize("name", LATS)
@pytest.mark.parametrize("wall", [lbm.PERIODIC, lbm.ZERO_FLUX])
def test_species_totals_conserved(name, wall):
    """Eq. (2-1) with closed boundaries: every species' total is constant in time."""
    rng = np.random.default_rng(9)
    N = 5
    D = _rand_D(rng, N, 0.03, 0.3)
    shape = _shape(name, (10, 6, 5))
    bc = ((wall, wall),) * len(shape)
    p = lbm.Problem(name, D, shape, bc=bc)
    xi0 = _rand_field(rng, N, p.nodes)
    f = lbm.run(p, xi0, 40)
    mass, mn, mx, bad = lbm.diagnostics(p, f)
    np.testing.assert_allclose(mass, xi0.reshape(N, -1).sum(1), rtol=1e-14)
    assert bad == 0 and np.all(mn > 0) and np.all(mx < 1)


def test_species_totals_conserved_over_long_runs():
    """No systematic rounding drift of the totals: 10,000 steps of a 1D ternary step
    problem keep every total to within 1e-13 of its initial value."""
    rng = np.random.default_rng(19)
    D = _rand_D(rng, 3, 0.03, 0.3)
    p = lbm.Problem("D1Q3", D, (64,))
    x = np.arange(64) < 32
    xi0 = np.stack([np.where(x, 0.5, 0.0), np.full(64, 0.5), np.where(x, 0.0, 0.5)])
    f = lbm.init(p, xi0)
    for _ in range(10_000):
        f = lbm.step(p, f)
    mass = lbm.diagnostics(p, f)[0]
    np.testing.assert_allclose(mass, xi0.sum(1), rtol=0, atol=1e-13)


def test_steady_state_is_the_mean_composition():
    """Closed domain: the long-time state is uniform at the initial mean (Secs. 4.2-4.3)."""
    rng = np.random.default_rng(10)
    D = _rand_D(rng, 3, 0.1, 0.3)
    p = lbm.Problem("D1Q3", D, (16,), bc=((lbm.ZERO_FLUX, lbm.ZERO_FLUX),))
    xi0 = _rand_field(rng, 3, p.nodes)
    xi = lbm.mole_fractions(lbm.run(p, xi0, 6000))
    np.testing.assert_allclose(xi, np.broadcast_to(xi0.mean(axis=1, keepdims=True), xi.shape), atol=1e-12)


@pytest.mark.parametrize("name", ["D1Q3", "D2Q5"])
def test_dirichlet_steady_state_is_linear_with_exact_flux(name):
    """Binary diffusion between two Dirichlet walls (anti-bounce-back, Sec. 4) settles on
    the straight line through the wall values at the half-way wall positions, with the
    uniform Fick flux J = -D (xi_hi - xi_lo) / n (Eq. (2-12a)) read by Eq. (3-27)."""
    n = 16
    Dv = 0.12
    lo, hi = 0.9, 0.1
    shape = (n,) if name == "D1Q3" else (n, 3)
    bc = ((lbm.DIRICHLET, lbm.DIRICHLET),) + ((lbm.PERIODIC, lbm.PERIODIC),) * (len(shape) - 1)
    p = lbm.Problem(name, np.array([[1, Dv], [Dv, 1.0]]), shape, bc=bc,
                    xi_wall={(0, 0): np.array([lo, 1 - lo]), (0, 1): np.array([hi, 1 - hi])})
    xi0 = np.full((2,) + p.nodes, 0.5)
    f = lbm.run(p, xi0, 8000)
    xi, grad, J = lbm.observables(p, f)
    xj = (np.arange(n) + 0.5) / n
    expect = lo + (hi - lo) * xj
    np.testing.assert_allclose(xi[0].reshape(-1, n), np.broadcast_to(expect, (xi[0].size // n, n)), atol=1e-12)
    np.testing.assert_allclose(J[0, 0], -Dv * (hi - lo) / n, atol=1e-13)
    np.testing.assert_allclose(grad[0, 0], (hi - lo) / n, atol=1e-12)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q15"])
def test_diagonal_lattice_walls_conserve_and_keep_equilibria(name):
    """Walls crossed by diagonal directions (Sec. 4 face rules at edges and corners):
    zero-flux faces on every side conserve every species total exactly; a uniform
    field stays uniform under zero-flux walls, and under Dirichlet walls that hold the
    field's own composition (both rules return w_k xi for an equilibrium)."""
    rng = np.random.default_rng(90)
    N = 3
    D = _rand_D(rng, N, 0.05, 0.3)
    shape = _shape(name, (7, 6, 5))
    d = len(shape)
    p = lbm.Problem(name, D, shape, bc=tuple((lbm.ZERO_FLUX, lbm.ZERO_FLUX) for _ in range(d)))
    xi0 = _rand_field(rng, N, p.nodes)
    xi = lbm.mole_fractions(lbm.run(p, xi0, 25))
    np.testing.assert_allclose(xi.reshape(N, -1).sum(1), xi0.reshape(N, -1).sum(1), rtol=1e-13)
    assert np.abs(xi - xi0).max() > 1e-3          # the field did move
    u = np.array([0.2, 0.5, 0.3])
    xu = np.broadcast_to(u.reshape((N,) + (1,) * d), (N,) + p.nodes).copy()
    np.testing.assert_allclose(lbm.mole_fractions(lbm.run(p, xu, 7)), xu, rtol=0, atol=1e-15)
    walls = {(a, s): u for a in range(d) for s in (0, 1)}
    pd = lbm.Problem(name, D, shape, bc=tuple((lbm.DIRICHLET, lbm.DIRICHLET) for _ in range(d)), xi_wall=walls)
    np.testing.assert_allclose(lbm.mole_fractions(lbm.run(pd, xu, 7)), xu, rtol=0, atol=1e-15)


@pytest.mark.parametrize("name", ["D2Q9", "D3Q15"])
def test_diagonal_lattice_dirichlet_walls_reach_linear_steady_state(name):
    """Binary mixture between two Dirichlet faces in x (periodic elsewhere): the steady
    state of Eq. (2-13) is linear in x; half-way anti-bounce-back puts the faces half a
    spacing outside the end nodes.  The lattice solution matches that line to O(10^-3)
    (the Eq. (3-16) relaxation puts the walls at the half-way points)."""
    n = 12
    shape = _shape(name, (n, 3, 3))
    d = len(shape)
    D = np.array([[1.0, 0.15], [0.15, 1.0]])
    bc = ((lbm.DIRICHLET, lbm.DIRICHLET),) + ((lbm.PERIODIC, lbm.PERIODIC),) * (d - 1)
    lo, hi = 0.8, 0.2
    p = lbm.Problem(name, D, shape, bc=bc, xi_wall={(0, 0): np.array([lo, 1 - lo]), (0, 1): np.array([hi, 1 - hi])})
    xi0 = np.full((2,) + p.nodes, 0.5)
    xi = lbm.mole_fractions(lbm.run(p, xi0, 4000))[0].reshape(-1, n)
    x = np.arange(n) + 0.5
    expect = lo + (hi - lo) * x / n
    np.testing.assert_allclose(xi, np.broadcast_to(expect, xi.shape), rtol=0, atol=1e-3)


@pytest.mark.parametrize("lattice,shape,bc", [
    ("D2Q5", (24, 20), ((lbm.PERIODIC, lbm.PERIODIC), (lbm.ZERO_FLUX, lbm.ZERO_FLUX))),
    ("D1Q3", (64,), ((lbm.ZERO_FLUX, lbm.ZERO_FLUX),)),
])
def test_absent_species_reduces_to_the_binary_mixture(lattice, shape, bc):
    """Eq. (2-10): with xi_2 = 0 everywhere the row of B for species 2 has only
    its diagonal, so species 2 stays absent, and species 1 sees
    B_11 = (xi_1 + xi_3)/D_13 = 1/D_13: the ternary run equals the binary
    mixture of species 1 and 3 with D = D_13 (Remark I)."""
    _absent_species_check(lattice, shape, bc)


def _ms_B_without_xi_factor(xi, D):
    B = _ORIGINAL_MS_B(xi, D)
    n = D.shape[0]
    for i in range(n - 1):
        for j in range(n - 1):
            if i != j:
                B[..., i, j] = 1.0 / D[i, n - 1] - 1.0 / D[i, j]
    return B


def _ms_B_transposed(xi, D):
    return np.swapaxes(_ORIGINAL_MS_B(xi, D), -1, -2).copy()


def _ms_B_wrong_last_species(xi, D):
    # the diagonal's own term divided by D_i,N-1 instead of D_iN
    B = _ORIGINAL_MS_B(xi, D)
    n = D.shape[0]
    for i in range(n - 1):
        B[..., i, i] += xi[..., i] * (1.0 / D[i, n - 2 if i != n - 2 else n - 3] - 1.0 / D[i, n - 1])
    return B


_ORIGINAL_MS_B = ms.ms_B


@pytest.mark.parametrize("mistake", [_ms_B_without_xi_factor, _ms_B_transposed, _ms_B_wrong_last_species])
def test_absent_species_pin_catches_planted_mistakes(monkeypatch, mistake):
    """The absent-species pin fails when B of Eq. (2-10) in the oracle carries
    a plausible mistake: the off-diagonal terms without their xi_i factor, B
    transposed, or the diagonal's own term over the wrong pair's D."""
    monkeypatch.setattr(ms, "ms_B", mistake)
    with pytest.raises(AssertionError):
        _absent_species_check("D1Q3", (64,), ((lbm.ZERO_FLUX, lbm.ZERO_FLUX),))


def _absent_species_check(lattice, shape, bc):
    rng = np.random.default_rng(61)
    D3 = _rand_D(rng, 3, 0.05, 0.5)
    nodes = tuple(reversed(shape))
    two = _rand_field(rng, 2, nodes)
    three = np.stack([two[0], np.zeros(nodes), two[1]])
    steps = 40
    pt = lbm.Problem(lattice, D3, shape, bc=bc)
    pb = lbm.Problem(lattice, np.array([[1.0, D3[0, 2]], [D3[0, 2], 1.0]]), shape, bc=bc)
    xt, _, Jt = lbm.observables(pt, lbm.run(pt, three, steps))
    xb, _, Jb = lbm.observables(pb, lbm.run(pb, two, steps))
    assert np.abs(xt[1]).max() <= 1e-15
    assert np.abs(Jt[1]).max() <= 1e-15
    np.testing.assert_allclose(xt[0], xb[0], rtol=0, atol=1e-13)
    np.testing.assert_allclose(xt[2], xb[1], rtol=0, atol=1e-13)
    np.testing.assert_allclose(Jt[0], Jb[0], rtol=0, atol=1e-13)
    # the binary field is not stationary: the test compares evolved states
    assert np.abs(xb[0] - two[0]).max() > 1e-3


_ORIGINAL_STREAM = lbm.stream


def _stream_wall_term_without_factor_two(prob, fpost):
    # the anti-bounce-back wall term w_kbar xi_b instead of 2 w_kbar xi_b
    halved = dataclasses.replace(prob, xi_wall={k: 0.5 * np.asarray(v) for k, v in prob.xi_wall.items()})
    return _ORIGINAL_STREAM(halved, fpost)


def test_dirichlet_pin_catches_a_planted_mistake(monkeypatch):
    """The antisymmetric-extension pin fails when the oracle's anti-bounce-back
    (Sec. 4) takes its wall term without the factor 2."""
    monkeypatch.setattr(lbm, "stream", _stream_wall_term_without_factor_two)
    with pytest.raises(AssertionError):
        test_dirichlet_wall_equals_antisymmetric_extension_linear("D1Q3")
