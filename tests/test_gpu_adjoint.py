"""Hand-written adjoint of the sweep (through the C ABI) against the autograd
twin of the oracle and against central finite differences of the GPU forward
run in FP64."""
import ctypes as C

import numpy as np
import pytest
import torch

from gpu_cases import assert_parity, oracle_problem, oracle_run, rand_D, rand_field, smooth_field
from oracle import twin

pytestmark = pytest.mark.gpu


def _gpu_grads(lattice, D, shape, precision, xi0, target, steps, every, launch=None, **kw):
    from paper_1808_06787_amd import adjoint
    from paper_1808_06787_amd.sim import Sim

    sim = Sim(lattice, D, shape, precision, **kw)
    if launch:
        sim.set_launch(**launch)
    sim.init(torch.from_numpy(xi0))
    ckpts = adjoint.forward_with_checkpoints(sim, steps, every)
    xi, _, _ = sim.read(torch.float64, flux=False, grad=False)
    tgt = torch.from_numpy(target).to(xi.device)
    L = float(((xi - tgt) ** 2).sum())
    dxi0, dD = adjoint.gradients(sim, ckpts, steps, 2.0 * (xi - tgt), every)
    sim.close()
    return L, dD, dxi0.cpu().numpy()


def _compare(ref, got, rel, label):
    L0, gD0, gx0 = ref
    L1, gD1, gx1 = got
    assert abs(L1 - L0) <= rel * max(abs(L0), 1e-30), (label, L0, L1)
    sD = np.abs(gD0).max()
    assert np.abs(gD1 - gD0).max() <= rel * sD, (label, gD0, gD1)
    sx = np.abs(gx0).max()
    assert np.abs(gx1 - gx0).max() <= rel * sx, (label, np.abs(gx1 - gx0).max(), sx)


CASES = [
    ("D2Q5", (13, 9), 3, (("dirichlet", "zero_flux"), ("periodic", "periodic"))),
    ("D2Q5", (17, 6), 4, (("periodic", "periodic"), ("zero_flux", "zero_flux"))),
    ("D1Q3", (23,), 4, (("zero_flux", "dirichlet"),)),
    ("D3Q7", (6, 5, 4), 3, (("zero_flux", "zero_flux"), ("periodic", "periodic"), ("dirichlet", "dirichlet"))),
    ("D1Q2", (19,), 3, (("dirichlet", "zero_flux"),)),
    ("D2Q4", (11, 8), 4, (("zero_flux", "dirichlet"), ("periodic", "periodic"))),
    ("D3Q6", (5, 6, 4), 3, (("periodic", "periodic"), ("zero_flux", "dirichlet"), ("zero_flux", "zero_flux"))),
    ("D2Q9", (12, 9), 3, (("dirichlet", "zero_flux"), ("zero_flux", "dirichlet"))),
    ("D2Q9", (10, 11), 4, (("periodic", "periodic"), ("dirichlet", "zero_flux"))),
    ("D3Q15", (6, 5, 4), 3, (("zero_flux", "dirichlet"), ("periodic", "periodic"), ("dirichlet", "zero_flux"))),
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("relax", ["paper", "srt", "trt"])
def test_adjoint_matches_autograd_twin_fp64(case, relax):
    lattice, shape, N, bc = CASES[case]
    rng = np.random.default_rng(60 + case)
    D = rand_D(rng, N)
    walls = {}
    for a, (lo, hi) in enumerate(bc):
        for s, kind in enumerate((lo, hi)):
            if kind == "dirichlet":
                walls[(a, s)] = rand_field(rng, N, ())
    xi0 = smooth_field(rng, N, shape[::-1], 0.15)
    target = smooth_field(rng, N, shape[::-1], 0.15)
    steps, every = 20, 6
    magic = 0.35     # TRT: away from Eq. (3-16)'s 3/16 (ignored by the other rules)
    p = oracle_problem(lattice, D, shape, bc=bc, xi_wall=walls, relax=relax, trt_magic=magic)
    ref = twin.misfit_gradients(p, xi0, target, steps)
    got = _gpu_grads(lattice, D, shape, "f64", xi0, target, steps, every, bc=bc, xi_wall=walls, relax=relax,
                     trt_magic=magic)
    _compare(ref, got, 1e-10, f"{lattice} {relax}")


def test_adjoint_linearised_mode_fp64():
    rng = np.random.default_rng(66)
    N, shape = 4, (11, 10)
    D = rand_D(rng, N)
    xref = rand_field(rng, N, ())
    xi0 = smooth_field(rng, N, shape[::-1], 0.1)
    target = smooth_field(rng, N, shape[::-1], 0.1)
    p = oracle_problem("D2Q5", D, shape, xi_ref=xref)
    ref = twin.misfit_gradients(p, xi0, target, 15)
    got = _gpu_grads("D2Q5", D, shape, "f64", xi0, target, 15, 4, xi_ref=xref)
    _compare(ref, got, 1e-10, "linearised")


@pytest.mark.parametrize("steps,every", [(0, 5), (1, 5), (7, 7), (7, 1), (12, 100)])
def test_adjoint_segmenting_edge_cases(steps, every):
    rng = np.random.default_rng(67)
    N, shape = 3, (9, 7)
    D = rand_D(rng, N)
    xi0 = smooth_field(rng, N, shape[::-1], 0.1)
    target = smooth_field(rng, N, shape[::-1], 0.1)
    p = oracle_problem("D2Q5", D, shape)
    ref = twin.misfit_gradients(p, xi0, target, steps)
    got = _gpu_grads("D2Q5", D, shape, "f64", xi0, target, steps, every)
    if steps <= 1:
        # no step, or one step from f(0) = w xi(0), whose non-equilibrium part is
        # zero: L does not depend on D (both sides hold rounding noise at most)
        assert np.abs(got[1]).max() <= 1e-15 and np.abs(ref[1]).max() <= 1e-15
        np.testing.assert_allclose(got[2], ref[2], rtol=0, atol=1e-13 * np.abs(ref[2]).max())
    else:
        _compare(ref, got, 1e-10, f"{steps}/{every}")


def test_adjoint_fp32_close_to_fp64_reference():
    rng = np.random.default_rng(68)
    N, shape = 3, (40, 33)
    D = rand_D(rng, N, 0.05, 0.5)
    xi0 = smooth_field(rng, N, shape[::-1], 0.1)
    target = smooth_field(rng, N, shape[::-1], 0.1)
    ref = _gpu_grads("D2Q5", D, shape, "f64", xi0, target, 60, 16)
    got = _gpu_grads("D2Q5", D, shape, "f32", xi0, target, 60, 16)
    _compare(ref, got, 2e-4, "fp32")


def test_adjoint_agrees_with_central_differences():
    """Central differences with h = 1e-4 of the FP64 forward run (a 64 x 48 ternary
    problem, 300 steps) against the adjoint: every D_ij pair and one random
    direction of the initial field agree to 1e-4 relative."""
    from paper_1808_06787_amd.sim import Sim

    rng = np.random.default_rng(69)
    N, shape, steps = 3, (64, 48), 300
    D = rand_D(rng, N, 0.05, 0.5)
    xi0 = smooth_field(rng, N, shape[::-1], 0.1)
    target = smooth_field(rng, N, shape[::-1], 0.1)
    L, gD, gx = _gpu_grads("D2Q5", D, shape, "f64", xi0, target, steps, 50)

    def loss(Dm, x0):
        s = Sim("D2Q5", Dm, shape, "f64")
        s.init(torch.from_numpy(x0))
        s.step(steps)
        xi, _, _ = s.read(torch.float64, flux=False, grad=False)
        s.close()
        return float(((xi.cpu().numpy() - target) ** 2).sum())

    h = 1e-4
    for i in range(N):
        for j in range(i + 1, N):
            Dp, Dm = D.copy(), D.copy()
            Dp[i, j] = Dp[j, i] = D[i, j] + h
            Dm[i, j] = Dm[j, i] = D[i, j] - h
            fd = (loss(Dp, xi0) - loss(Dm, xi0)) / (2 * h)
            assert abs(fd - gD[i, j]) <= 1e-4 * abs(fd), (i, j, fd, gD[i, j])
    v = rng.standard_normal(size=xi0.shape)
    v -= v.mean(axis=0, keepdims=True)
    v /= np.linalg.norm(v)
    fd = (loss(D, xi0 + h * v) - loss(D, xi0 - h * v)) / (2 * h)
    ad = float((gx * v[: N - 1]).sum())
    assert abs(fd - ad) <= 1e-4 * abs(fd), (fd, ad)


def test_autograd_function():
    from paper_1808_06787_amd.adjoint import MSDiffusion

    rng = np.random.default_rng(70)
    N, shape = 3, (12, 8)
    D = rand_D(rng, N)
    xi0 = smooth_field(rng, N, shape[::-1], 0.1)
    target = smooth_field(rng, N, shape[::-1], 0.1)
    x = torch.tensor(xi0, device="cuda", requires_grad=True)
    Dt = torch.tensor(D, requires_grad=True)
    spec = dict(lattice="D2Q5", shape=shape, precision="f64", steps=10, every=3)
    xi = MSDiffusion.apply(x, Dt, spec)
    L = ((xi - torch.tensor(target, device="cuda")) ** 2).sum()
    L.backward()
    p = oracle_problem("D2Q5", D, shape)
    L0, gD0, gx0 = twin.misfit_gradients(p, xi0, target, 10)
    assert abs(L.item() - L0) <= 1e-12 * L0
    np.testing.assert_allclose(Dt.grad.numpy() + Dt.grad.numpy().T, gD0, rtol=1e-10, atol=1e-14)
    np.testing.assert_allclose(x.grad.cpu().numpy()[: N - 1], gx0, rtol=1e-10, atol=1e-14 * np.abs(gx0).max())
    assert np.all(x.grad.cpu().numpy()[N - 1] == 0)


BLOCKED_CASES = [
    ((300, 11), (("periodic", "periodic"), ("periodic", "periodic"))),
    ((260, 9), (("dirichlet", "zero_flux"), ("zero_flux", "dirichlet"))),
    ((7, 40), (("zero_flux", "zero_flux"), ("periodic", "periodic"))),
]


def _blocked_problem(case, N, seed):
    rng = np.random.default_rng(seed)
    shape, bc = BLOCKED_CASES[case]
    D = rand_D(rng, N)
    walls = {}
    for a, (lo, hi) in enumerate(bc):
        for side, kind in enumerate((lo, hi)):
            if kind == "dirichlet":
                walls[(a, side)] = rand_field(rng, N, ())
    xi0 = smooth_field(rng, N, shape[::-1], 0.1)
    target = smooth_field(rng, N, shape[::-1], 0.1)
    return shape, bc, walls, D, xi0, target


@pytest.mark.parametrize("case", range(len(BLOCKED_CASES)))
@pytest.mark.parametrize("tb", [2, 3, 4])
def test_blocked_adjoint_and_recording_fp64(case, tb):
    """Binary mixture in FP64: recomputation by blocked passes that store every
    step, and blocked adjoint passes (2 or 3 steps), across column tiles and
    4-row segments, every face kind, segments of 8 steps with remainders."""
    N = 2
    shape, bc, walls, D, xi0, target = _blocked_problem(case, N, 400 + case)
    steps, every = 23, 8
    p = oracle_problem("D2Q5", D, shape, bc=bc, xi_wall=walls)
    ref = twin.misfit_gradients(p, xi0, target, steps)
    got = _gpu_grads("D2Q5", D, shape, "f64", xi0, target, steps, every,
                     launch=dict(temporal=tb, seg_rows=4), bc=bc, xi_wall=walls)
    _compare(ref, got, 1e-10, f"blocked tb={tb} case {case}")


@pytest.mark.parametrize("case", range(len(BLOCKED_CASES)))
@pytest.mark.parametrize("tb", [2, 3])
def test_blocked_adjoint_fp32_ternary(case, tb):
    """Ternary FP32 with blocked passes against the FP64 result of one step per
    pass (the FP32 tolerance of the adjoint)."""
    N = 3
    shape, bc, walls, D, xi0, target = _blocked_problem(case, N, 410 + case)
    steps, every = 30, 13
    ref = _gpu_grads("D2Q5", D, shape, "f64", xi0, target, steps, every, launch=dict(temporal=0),
                     bc=bc, xi_wall=walls)
    got = _gpu_grads("D2Q5", D, shape, "f32", xi0, target, steps, every, launch=dict(temporal=tb, seg_rows=4),
                     bc=bc, xi_wall=walls)
    _compare(ref, got, 2e-4, f"fp32 blocked tb={tb} case {case}")


# Widths at which the last column tile of the blocked adjoint pass needs exactly 64 or 65 lanes
# (output columns and TB halo columns on either side), with one tile and with two.
LAST_TILE_WIDTHS = {2: (60, 61, 312, 313), 3: (58, 59, 308, 309)}


@pytest.mark.parametrize("tb", [2, 3])
@pytest.mark.parametrize("k", range(4))
@pytest.mark.parametrize("xbc", [("periodic", "periodic"), ("dirichlet", "zero_flux")])
def test_blocked_adjoint_last_tile_wave_boundary(tb, k, xbc):
    """Blocked adjoint passes and recording where the last tile's live lanes end exactly at a
    wave boundary or one lane past it; FP64 binary against the oracle's autograd twin."""
    N = 2
    shape = (LAST_TILE_WIDTHS[tb][k], 9)
    rng = np.random.default_rng(2300 + 10 * tb + k)
    D = rand_D(rng, N)
    bc = (xbc, ("periodic", "periodic"))
    walls = {(0, 0): rand_field(rng, N, ())} if xbc[0] == "dirichlet" else {}
    xi0 = smooth_field(rng, N, shape[::-1], 0.1)
    target = smooth_field(rng, N, shape[::-1], 0.1)
    steps, every = 2 * tb + 3, tb + 2
    p = oracle_problem("D2Q5", D, shape, bc=bc, xi_wall=walls)
    ref = twin.misfit_gradients(p, xi0, target, steps)
    got = _gpu_grads("D2Q5", D, shape, "f64", xi0, target, steps, every,
                     launch=dict(temporal=tb, seg_rows=4), bc=bc, xi_wall=walls)
    _compare(ref, got, 1e-10, f"last tile tb={tb} {shape} {xbc}")


DILUTE_CASES = [
    ("D2Q5", (13, 9), (("dirichlet", "zero_flux"), ("periodic", "periodic")), None),
    ("D1Q3", (23,), (("zero_flux", "dirichlet"),), None),
    ("D3Q7", (6, 5, 4), (("zero_flux", "zero_flux"), ("periodic", "periodic"), ("dirichlet", "dirichlet")), None),
    ("D2Q9", (12, 9), (("dirichlet", "zero_flux"), ("zero_flux", "dirichlet")), None),
    ("D2Q5", (11, 10), (("periodic", "periodic"), ("zero_flux", "dirichlet")), "linearised"),
    # wide enough for blocked forward recomputation (the adjoint passes stay single steps)
    ("D2Q5", (300, 11), (("dirichlet", "zero_flux"), ("zero_flux", "dirichlet")), "blocked"),
]


@pytest.mark.parametrize("case", range(len(DILUTE_CASES)))
@pytest.mark.parametrize("relax", ["paper", "trt"])
def test_adjoint_dilute_mode_matches_autograd_twin_fp64(case, relax):
    """Remark III's diagonal B through the hand-written adjoint: loss, dL/dD and
    dL/dxi(0) against the autograd twin of the oracle."""
    lattice, shape, bc, extra = DILUTE_CASES[case]
    N = 3 if extra == "blocked" else 4     # FP64 blocks up to m = 2
    rng = np.random.default_rng(90 + case)
    D = rand_D(rng, N)
    walls = {}
    for a, (lo, hi) in enumerate(bc):
        for s, kind in enumerate((lo, hi)):
            if kind == "dirichlet":
                walls[(a, s)] = rand_field(rng, N, ())
    xref = rand_field(rng, N, ()) if extra == "linearised" else None
    xi0 = smooth_field(rng, N, shape[::-1], 0.15)
    target = smooth_field(rng, N, shape[::-1], 0.15)
    steps, every = 17, 5
    p = oracle_problem(lattice, D, shape, bc=bc, xi_wall=walls, relax=relax, trt_magic=0.35, xi_ref=xref,
                       dilute=True)
    ref = twin.misfit_gradients(p, xi0, target, steps)
    launch = dict(temporal=3, seg_rows=4) if extra == "blocked" else None
    got = _gpu_grads(lattice, D, shape, "f64", xi0, target, steps, every, launch=launch, bc=bc, xi_wall=walls,
                     relax=relax, trt_magic=0.35, xi_ref=xref, dilute=True)
    _compare(ref, got, 1e-10, f"{lattice} dilute {relax} {extra}")


def test_adjoint_with_wide_tile_recomputation_fp32():
    """A domain of 6144 columns or more: the forward recomputation of the adjoint
    takes 512-column blocked passes (recording every state of a pass); the
    gradients match the autograd twin of the oracle to the FP32 bound of the
    other FP32 adjoint tests, and equal those of a run whose passes stay on
    256-column tiles (five steps per pass) to FP32 rounding.  An explicit segment
    height keeps both runs blocked on this short domain."""
    from paper_1808_06787_amd.sim import Sim

    N = 3
    rng = np.random.default_rng(95)
    D = rand_D(rng, N)
    shape = (6200, 20)
    xi0 = smooth_field(rng, N, shape[::-1], 0.1)
    target = smooth_field(rng, N, shape[::-1], 0.1)
    steps, every = 26, 13
    wide_launch, narrow_launch = dict(seg_rows=8), dict(temporal=5, seg_rows=8)
    for launch, want in ((wide_launch, 6), (narrow_launch, 5)):
        probe = Sim("D2Q5", D, shape, "f32")
        probe.set_launch(**launch)
        assert probe.steps_per_pass() == want, launch
        probe.close()
    wide = _gpu_grads("D2Q5", D, shape, "f32", xi0, target, steps, every, launch=wide_launch)
    narrow = _gpu_grads("D2Q5", D, shape, "f32", xi0, target, steps, every, launch=narrow_launch)
    ref = twin.misfit_gradients(oracle_problem("D2Q5", D, shape), xi0, target, steps)
    _compare(ref, wide, 2e-4, "wide-tile recomputation vs twin")
    _compare(narrow, wide, 2e-5, "wide vs 256-column recomputation")


RECORD_CASES = [
    ((300, 24), (("periodic", "periodic"), ("periodic", "periodic"))),
    ((250, 21), (("dirichlet", "zero_flux"), ("periodic", "periodic"))),
]


@pytest.mark.parametrize("case", range(len(RECORD_CASES)))
@pytest.mark.parametrize("precision,N,tb", [("f32", 3, 6), ("f32", 3, 4), ("f64", 2, 3)])
def test_record_slots_match_oracle(case, precision, N, tb):
    """msd_record through blocked passes (full passes and a shorter remainder,
    8-row segments over two column tiles) stores the state after every step:
    each slot, restored into a second handle at its time, reads back the
    oracle's moments at that time; the recording handle ends on the last slot.
    Periodic domains take the recording instantiation, walled ones the general
    blocked kernel."""
    from paper_1808_06787_amd import _ffi as F
    from paper_1808_06787_amd.sim import Sim

    rng = np.random.default_rng(500 + 10 * case + tb)
    shape, bc = RECORD_CASES[case]
    D = rand_D(rng, N)
    walls = {(0, 0): rand_field(rng, N, ())} if bc[0][0] == "dirichlet" else {}
    xi0 = smooth_field(rng, N, shape[::-1], 0.1)
    launch = dict(temporal=tb, seg_rows=8, lds_resident=0)
    sim = Sim("D2Q5", D, shape, precision, bc=bc, xi_wall=walls)
    sim.set_launch(**launch)
    assert sim.steps_per_pass() == tb
    sim.init(torch.from_numpy(xi0))
    sim.step(1)
    n = 2 * tb + 2
    sb = sim.state_bytes()
    stack = torch.empty(n * sb, dtype=torch.uint8, device=sim.device)
    torch.cuda.synchronize()
    F.check(sim.lib.msd_record(sim._h, n, C.c_void_p(stack.data_ptr())), "msd_record")
    torch.cuda.synchronize()
    assert sim.time == 1 + n
    last = sim.read(torch.float64)
    other = Sim("D2Q5", D, shape, precision, bc=bc, xi_wall=walls)
    other.init(torch.from_numpy(xi0))
    p = oracle_problem("D2Q5", D, shape, bc=bc, xi_wall=walls)
    for j in range(n):
        other.restore(stack[j * sb:(j + 1) * sb], 2 + j)
        got = [a.cpu().numpy() for a in other.read(torch.float64)]
        assert_parity(got, oracle_run(p, xi0, 2 + j), precision, f"slot {j} ({precision}, tb {tb}, case {case})")
    got = [a.cpu().numpy() for a in other.read(torch.float64)]
    for a, b in zip(got, last):
        np.testing.assert_array_equal(a, b.cpu().numpy())
    other.close()
    sim.close()
