"""Pins of the oracle's Maxwell-Stefan algebra against closed forms printed in the paper.

Each test states the passage it checks.  None of them re-derives a value with
the oracle's own formula: the expected values are the paper's explicit
expressions (Remarks I-IV, Eq. (SD), the equilibrium moments and the streaming
operator in moment space of Sec. 3.2) typed in independently.
"""
import numpy as np
import pytest

from oracle import lattice as lat
from oracle import ms

pytestmark = pytest.mark.filterwarnings("error")


def _rand_D(rng, n, lo=0.05, hi=0.9):
    D = np.ones((n, n))
    for i in range(n):
        for j in range(i + 1, n):
            D[i, j] = D[j, i] = np.exp(rng.uniform(np.log(lo), np.log(hi)))
    return D


def _rand_xi(rng, n, size):
    x = rng.uniform(0.0, 1.0, size=(size, n))
    return x / x.sum(axis=1, keepdims=True)


def test_ternary_B_and_determinant_remark_IV():
    """Remark IV: explicit 2x2 B and |B| (Eq. (2-18)) of a three-component mixture."""
    rng = np.random.default_rng(11)
    for _ in range(200):
        D = _rand_D(rng, 3)
        x1, x2, x3 = _rand_xi(rng, 3, 1)[0]
        D12, D13, D23 = D[0, 1], D[0, 2], D[1, 2]
        expect = np.array(
            [
                [1 / D13 + x2 * (1 / D12 - 1 / D13), x1 * (1 / D13 - 1 / D12)],
                [x2 * (1 / D23 - 1 / D12), 1 / D23 + x1 * (1 / D12 - 1 / D23)],
            ]
        )
        B = ms.ms_B(np.array([x1, x2, x3]), D)
        np.testing.assert_allclose(B, expect, rtol=1e-13, atol=1e-13)
        det = x1 / (D12 * D13) + x2 / (D12 * D23) + x3 / (D13 * D23)
        assert det > 0
        np.testing.assert_allclose(np.linalg.det(B), det, rtol=1e-12)


def test_ternary_fick_matrix_both_forms_remark_IV():
    """Remark IV: the two printed forms of D~ = B^-1 (Eq. (2-19), both versions)."""
    rng = np.random.default_rng(12)
    for _ in range(200):
        D = _rand_D(rng, 3)
        x1, x2, x3 = _rand_xi(rng, 3, 1)[0]
        D12, D13, D23 = D[0, 1], D[0, 2], D[1, 2]
        det = x1 / (D12 * D13) + x2 / (D12 * D23) + x3 / (D13 * D23)
        form1 = np.array(
            [
                [1 / D23 + x1 * (1 / D12 - 1 / D23), x1 * (1 / D12 - 1 / D13)],
                [x2 * (1 / D12 - 1 / D23), 1 / D13 + x2 * (1 / D12 - 1 / D13)],
            ]
        ) / det
        s = x1 * D23 + x2 * D13 + x3 * D12
        form2 = np.array(
            [
                [D13 * (x1 * D23 + (1 - x1) * D12), x1 * D23 * (D13 - D12)],
                [x2 * D13 * (D23 - D12), D23 * (x2 * D13 + (1 - x2) * D12)],
            ]
        ) / s
        Dt = ms.fick_matrix(ms.ms_B(np.array([x1, x2, x3]), D))
        np.testing.assert_allclose(Dt, form1, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(Dt, form2, rtol=1e-12, atol=1e-14)


def test_equal_D12_D13_structure():
    """Sec. 4.2, Eq. (SD): with D12 = D13, D~ = [[D12, 0], [beta xi2 (1 - D12/D23), beta]]."""
    rng = np.random.default_rng(13)
    for _ in range(100):
        D12 = np.exp(rng.uniform(np.log(0.05), np.log(1.0)))
        D23 = np.exp(rng.uniform(np.log(0.05), np.log(1.0)))
        D = np.array([[1, D12, D12], [D12, 1, D23], [D12, D23, 1.0]])
        x1, x2, x3 = _rand_xi(rng, 3, 1)[0]
        beta = 1.0 / (1 / D23 + x1 * (1 / D12 - 1 / D23))
        expect = np.array([[D12, 0.0], [beta * x2 * (1 - D12 / D23), beta]])
        Dt = ms.fick_matrix(ms.ms_B(np.array([x1, x2, x3]), D))
        np.testing.assert_allclose(Dt, expect, rtol=1e-12, atol=1e-14)


def test_binary_remark_I():
    """Remark I: a binary mixture has B = 1/D (Fick's law with D~ = D)."""
    for Dv in (0.01, 0.3, 2.0):
        for x1 in (0.0, 0.3, 1.0):
            B = ms.ms_B(np.array([x1, 1 - x1]), np.array([[1.0, Dv], [Dv, 1.0]]))
            np.testing.assert_allclose(B, [[1.0 / Dv]], rtol=1e-15)


@pytest.mark.parametrize("n", [3, 4, 5, 8])
def test_equal_diffusivities_remark_II(n):
    """Remark II: all D_ij equal to one value => B = I/D, D~ = D I (Eq. (2-15))."""
    rng = np.random.default_rng(n)
    Dv = 0.37
    D = np.full((n, n), Dv)
    xi = _rand_xi(rng, n, 50)
    B = ms.ms_B(xi, D)
    np.testing.assert_allclose(B, np.broadcast_to(np.eye(n - 1) / Dv, B.shape), rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(ms.fick_matrix(B), np.broadcast_to(np.eye(n - 1) * Dv, B.shape),
                               rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("n", [3, 4, 5])
def test_dilute_species_remark_III(n):
    """Remark III: as xi_i -> 0, row i of D~ tends to D_eff e_i with D_eff = 1/sum_k xi_k/D_ik."""
    rng = np.random.default_rng(100 + n)
    D = _rand_D(rng, n)
    for i in range(n - 1):
        for eps in (1e-4, 1e-6):
            xi = _rand_xi(rng, n, 1)[0]
            xi[i] = 0.0
            xi *= (1 - eps) / xi.sum()
            xi[i] = eps
            Dt = ms.fick_matrix(ms.ms_B(xi, D))
            d_eff = 1.0 / sum(xi[k] / D[i, k] for k in range(n) if k != i)
            expect = np.zeros(n - 1)
            expect[i] = d_eff
            # the neglected terms are O(xi_i)
            np.testing.assert_allclose(Dt[i], expect, atol=50 * eps * d_eff)


def test_fick_matrix_eigenvalues_real_positive():
    """Sec. 2 assumes B invertible; for positive D_ij and xi on the simplex the
    spectrum of D~ is real, positive and bounded by the extreme D_ij."""
    rng = np.random.default_rng(14)
    for n in (3, 4, 5):
        D = _rand_D(rng, n)
        off = D[~np.eye(n, dtype=bool)]
        for xi in _rand_xi(rng, n, 200):
            ev = np.linalg.eigvals(ms.fick_matrix(ms.ms_B(xi, D)))
            assert np.all(np.abs(ev.imag) < 1e-10)
            assert np.all(ev.real >= off.min() * (1 - 1e-10))
            assert np.all(ev.real <= off.max() * (1 + 1e-10))


def test_lambda1_roundtrip_eq_3_26():
    """Eq. (3-26) as printed maps the oracle's Lambda_1 back to D~ (self-consistency only;
    the physics of the map is pinned by the continuum-decay tests)."""
    rng = np.random.default_rng(15)
    for name in ("D1Q2", "D1Q3", "D2Q4", "D2Q5", "D3Q6", "D3Q7", "D2Q9", "D3Q15"):
        cs2 = lat.get(name).cs2
        D = _rand_D(rng, 4, 0.02, 0.3)
        Dt = ms.fick_matrix(ms.ms_B(_rand_xi(rng, 4, 30), D))
        L1 = ms.lambda1_from_fick(Dt, cs2)
        np.testing.assert_allclose(ms.fick_from_lambda1(L1, cs2), Dt, rtol=1e-12, atol=1e-14)


def test_lambda2_rule_eq_3_16():
    """Eq. (3-16): off-diagonal lambda_2 = lambda_1; diagonal 8(l-2)/(l-8); the product
    (1/l1 - 1/2)(1/l2 - 1/2) is then 3/16 on the diagonal."""
    L1 = np.array([[1.25, 0.1], [-0.2, 0.7]])
    L2 = ms.lambda2_from_lambda1(L1)
    assert L2[0, 1] == 0.1 and L2[1, 0] == -0.2
    np.testing.assert_allclose(L2[0, 0], 8 * (1.25 - 2) / (1.25 - 8), rtol=1e-15)
    for i in range(2):
        np.testing.assert_allclose((1 / L1[i, i] - 0.5) * (1 / L2[i, i] - 0.5), 3 / 16, rtol=1e-13)
    np.testing.assert_array_equal(ms.lambda2_from_lambda1(L1, ms.RELAX_SRT), L1)


@pytest.mark.parametrize("magic", [1 / 12, 3 / 16, 1 / 4, 1 / 2, 2.0])
def test_trt_rule_product_and_paper_special_case(magic):
    """TRT (odd moments with lambda_1, even ones with lambda_2, Sec. 3.1 after Eq. (3-14)):
    the diagonal lambda_2 solves (1/l1 - 1/2)(1/l2 - 1/2) = magic for every l1 in (0, 2),
    off-diagonals stay lambda_1, and magic = 3/16 is Eq. (3-16) exactly."""
    rng = np.random.default_rng(8)
    l1 = rng.uniform(0.05, 1.95, size=(50, 3))
    L1 = np.zeros((50, 3, 3))
    for i in range(3):
        L1[:, i, i] = l1[:, i]
    L1[:, 0, 1] = rng.uniform(-0.2, 0.2, 50)
    L2 = ms.lambda2_from_lambda1(L1, ms.RELAX_TRT, magic)
    np.testing.assert_array_equal(L2[:, 0, 1], L1[:, 0, 1])
    for i in range(3):
        np.testing.assert_allclose((1 / L1[:, i, i] - 0.5) * (1 / L2[:, i, i] - 0.5), magic, rtol=1e-12)
        assert np.all((L2[:, i, i] > 0) & (L2[:, i, i] < 2))       # stable even relaxation
    if magic == 3 / 16:
        np.testing.assert_allclose(L2, ms.lambda2_from_lambda1(L1, ms.RELAX_PAPER), rtol=1e-14, atol=1e-15)


def test_trt_rejects_non_positive_parameter():
    with pytest.raises(ValueError):
        ms.lambda2_from_lambda1(np.eye(2), ms.RELAX_TRT, 0.0)


def test_lattice_weights_and_sound_speed():
    """Eqs. (3-5), (3-7), (3-10): weights sum to one, velocity sets are symmetric,
    and sum_k w_k c_k c_k = cs2 I with cs2 = 1/3, 1/3, 1/4."""
    for name, cs2 in (("D1Q2", 1.0), ("D1Q3", 1 / 3), ("D2Q4", 1 / 2), ("D2Q5", 1 / 3), ("D3Q6", 1 / 3),
                      ("D3Q7", 1 / 4)):
        L = lat.get(name)
        np.testing.assert_allclose(L.w.sum(), 1.0, rtol=1e-15)
        d = L.d
        c = L.c[:, :d].astype(float)
        np.testing.assert_allclose((L.w[:, None] * c).sum(0), 0.0, atol=1e-15)
        np.testing.assert_allclose(np.einsum("k,ka,kb->ab", L.w, c, c), cs2 * np.eye(d), atol=1e-15)
        opp = L.opposite
        np.testing.assert_array_equal(L.c[opp], -L.c)
        np.testing.assert_allclose(L.w[opp], L.w)


def test_d2q5_equilibrium_moments():
    """Sec. 3.2 (Eq. (m0A)): M f^eq = xi (1, 0, 0, 0, -2/3 c^2) on D2Q5 with c = 1."""
    L = lat.D2Q5
    np.testing.assert_allclose(L.M0 @ L.w, [1, 0, 0, 0, -2.0 / 3.0], atol=1e-15)


def test_d2q5_streaming_operator_in_moment_space():
    """Sec. 3.2 (Eq. (MCM)): M diag(c_k . grad) M^-1 as printed, with c = 1."""
    L = lat.D2Q5
    Minv = np.linalg.inv(L.M0)
    cx = L.M0 @ np.diag(L.c[:, 0].astype(float)) @ Minv
    cy = L.M0 @ np.diag(L.c[:, 1].astype(float)) @ Minv
    expect_x = np.array(
        [
            [0, 1, 0, 0, 0],
            [2 / 5, 0, 0, 1 / 2, 1 / 10],
            [0, 0, 0, 0, 0],
            [0, 1, 0, 0, 0],
            [0, 1, 0, 0, 0],
        ]
    )
    expect_y = np.array(
        [
            [0, 0, 1, 0, 0],
            [0, 0, 0, 0, 0],
            [2 / 5, 0, 0, -1 / 2, 1 / 10],
            [0, 0, -1, 0, 0],
            [0, 0, 1, 0, 0],
        ]
    )
    np.testing.assert_allclose(cx, expect_x, atol=1e-14)
    np.testing.assert_allclose(cy, expect_y, atol=1e-14)


@pytest.mark.parametrize("name", ["D1Q2", "D1Q3", "D2Q4", "D2Q5", "D3Q6", "D3Q7", "D2Q9", "D3Q15"])
def test_moment_rows_have_definite_parity(name):
    """Every M0 row is even or odd under k -> kbar, odd rows are exactly those of odd
    order (first order on the lattices of Eq. (3-14)'s kind, also third order on D2Q9
    and D3Q15), which relax with Lambda_1, and M0 is invertible (needed for Eq. (3-13b))."""
    L = lat.get(name)
    opp = L.opposite
    for r, order in enumerate(L.row_order):
        row = L.M0[r]
        if order % 2:
            np.testing.assert_array_equal(row[opp], -row)
            assert lat.relaxation_family(order) == 1
        else:
            np.testing.assert_array_equal(row[opp], row)
            assert lat.relaxation_family(order) == (0 if order == 0 else 2)
    assert abs(np.linalg.det(L.M0)) > 1e-6
    np.testing.assert_array_equal(L.M0[0], np.ones(L.q))
