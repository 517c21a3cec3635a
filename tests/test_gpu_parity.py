"""Parity of the HIP sweep (through the C ABI) with the FP64 oracle.

Grids are ragged (no extent a multiple of the tile) and span several tiles;
every lattice, N from 2 to 8, both precisions, every face kind, both
relaxation rules and the linearised mode are covered.  Tolerances: FP64 1e-12
relative on mole fractions; FP32 1e-5 absolute (see gpu_cases.PREC_TOL).
"""
import numpy as np
import pytest

from gpu_cases import (assert_parity, gpu_run, oracle_problem, oracle_run, rand_D, rand_field,
                       smooth_field)

pytestmark = pytest.mark.gpu

SHAPES = {"D1Q3": (301,), "D2Q5": (97, 45), "D3Q7": (37, 19, 11),
          "D1Q2": (301,), "D2Q4": (97, 45), "D3Q6": (37, 19, 11),
          "D2Q9": (97, 45), "D3Q15": (37, 19, 11)}
WALLS = {"D1Q3": 1, "D2Q5": 2, "D3Q7": 3, "D1Q2": 1, "D2Q4": 2, "D3Q6": 3, "D2Q9": 2, "D3Q15": 3}
ALL = ["D1Q3", "D2Q5", "D3Q7", "D1Q2", "D2Q4", "D3Q6", "D2Q9", "D3Q15"]
DIAG = ["D2Q9", "D3Q15"]


def _bc(lattice, kinds):
    d = WALLS[lattice]
    return tuple(kinds[a % len(kinds)] for a in range(d))


@pytest.mark.parametrize("lattice", ALL)
@pytest.mark.parametrize("N", [2, 3, 4, 5])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_periodic_and_zero_flux(lattice, N, precision):
    rng = np.random.default_rng(1000 + 10 * N + len(lattice))
    D = rand_D(rng, N)
    shape = SHAPES[lattice]
    bc = _bc(lattice, [("zero_flux", "zero_flux"), ("periodic", "periodic")])
    xi0 = smooth_field(rng, N, shape[::-1], 0.15)
    steps = 60
    orc = oracle_run(oracle_problem(lattice, D, shape, bc=bc), xi0, steps)
    gpu = gpu_run(lattice, D, shape, precision, xi0, steps, bc=bc)
    err = assert_parity(gpu, orc, precision, f"{lattice} N={N} {precision}")
    print(f"{lattice} N={N} {precision}: max |dxi| = {err:.3e}")


@pytest.mark.parametrize("lattice", ALL)
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("relax", ["paper", "srt", "trt"])
def test_dirichlet_faces(lattice, precision, relax):
    rng = np.random.default_rng(77)
    N = 3
    D = rand_D(rng, N)
    shape = SHAPES[lattice]
    bc = _bc(lattice, [("dirichlet", "zero_flux"), ("periodic", "periodic"), ("dirichlet", "dirichlet")])
    walls = {}
    for a, (lo, hi) in enumerate(bc):
        for s, kind in enumerate((lo, hi)):
            if kind == "dirichlet":
                walls[(a, s)] = rand_field(rng, N, ())
    xi0 = rand_field(rng, N, shape[::-1])
    magic = 0.11     # TRT: a product parameter away from Eq. (3-16)'s 3/16
    orc = oracle_run(oracle_problem(lattice, D, shape, bc=bc, xi_wall=walls, relax=relax, trt_magic=magic), xi0, 40)
    gpu = gpu_run(lattice, D, shape, precision, xi0, 40, bc=bc, xi_wall=walls, relax=relax, trt_magic=magic)
    assert_parity(gpu, orc, precision, f"{lattice} dirichlet {precision} {relax}")


@pytest.mark.parametrize("N", [6, 7, 8])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_many_species(N, precision):
    rng = np.random.default_rng(500 + N)
    D = rand_D(rng, N, 0.05, 0.3)
    shape = (70, 33)
    xi0 = smooth_field(rng, N, shape[::-1], 0.05)
    orc = oracle_run(oracle_problem("D2Q5", D, shape), xi0, 30)
    gpu = gpu_run("D2Q5", D, shape, precision, xi0, 30)
    assert_parity(gpu, orc, precision, f"N={N} {precision}")


@pytest.mark.parametrize("lattice", ALL)
@pytest.mark.parametrize("relax", ["paper", "srt"])
def test_linearised_mode(lattice, relax):
    rng = np.random.default_rng(31)
    N = 4
    D = rand_D(rng, N)
    shape = SHAPES[lattice]
    xref = np.array([0.1, 0.2, 0.3, 0.4])
    xi0 = smooth_field(rng, N, shape[::-1], 0.05)
    orc = oracle_run(oracle_problem(lattice, D, shape, relax=relax, xi_ref=xref), xi0, 50)
    gpu = gpu_run(lattice, D, shape, "f64", xi0, 50, relax=relax, xi_ref=xref)
    assert_parity(gpu, orc, "f64", f"{lattice} linearised {relax}")


def test_c_t_scales_flux_only():
    rng = np.random.default_rng(3)
    D = rand_D(rng, 3)
    xi0 = smooth_field(rng, 3, (40, 64), 0.1)
    a = gpu_run("D2Q5", D, (64, 40), "f64", xi0, 20)
    b = gpu_run("D2Q5", D, (64, 40), "f64", xi0, 20, c_t=2.5)
    np.testing.assert_array_equal(a[0], b[0])
    np.testing.assert_allclose(b[1], 2.5 * a[1], rtol=1e-14, atol=1e-18)
    np.testing.assert_array_equal(a[2], b[2])


def test_launch_configurations_are_bitwise_identical():
    """Tiling, XCD remapping and store hints change scheduling only."""
    rng = np.random.default_rng(4)
    D = rand_D(rng, 4)
    shape = (203, 67)
    xi0 = smooth_field(rng, 4, shape[::-1], 0.1)
    ref = gpu_run("D2Q5", D, shape, "f32", xi0, 25, launch=dict(block_x=256, block_y=1, xcd_remap=0, temporal=0))
    for launch in (dict(block_x=64, block_y=4), dict(block_x=128, block_y=2, nontemporal=1),
                   dict(block_x=192, block_y=1, xcd_remap=1), dict(block_x=64, block_y=1, xcd_remap=1)):
        got = gpu_run("D2Q5", D, shape, "f32", xi0, 25, launch=dict(launch, temporal=0))
        for a, b in zip(ref, got):
            np.testing.assert_array_equal(a, b, err_msg=str(launch))


def test_split_step_calls_equal_one_call():
    rng = np.random.default_rng(5)
    D = rand_D(rng, 3)
    shape = (50, 31, 9)
    xi0 = smooth_field(rng, 3, shape[::-1], 0.1)
    a = gpu_run("D3Q7", D, shape, "f64", xi0, 30)
    b = gpu_run("D3Q7", D, shape, "f64", xi0, 30, split=[1, 0, 7, 22])
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_lds_resident_path_matches_global_path(precision):
    rng = np.random.default_rng(6)
    D = rand_D(rng, 3)
    xi0 = smooth_field(rng, 3, (256,), 0.2)
    lds = gpu_run("D1Q3", D, (256,), precision, xi0, 500, launch=dict(lds_resident=1))
    glob = gpu_run("D1Q3", D, (256,), precision, xi0, 500, launch=dict(lds_resident=0))
    orc = oracle_run(oracle_problem("D1Q3", D, (256,)), xi0, 500)
    assert_parity(lds, orc, precision, "lds")
    assert_parity(glob, orc, precision, "global")
    tol = 1e-13 if precision == "f64" else 1e-6
    np.testing.assert_allclose(lds[0], glob[0], rtol=0, atol=tol)


def test_ternary_1d_workload_full_length():
    """The 1D ternary step workload (D1Q3, 256 nodes, FP64, 10,000 steps) in full."""
    import workloads

    w = workloads.ternary_1d()
    orc = oracle_run(oracle_problem(w.lattice, w.D, w.shape, bc=w.bc), w.xi0, w.steps)
    gpu = gpu_run(w.lattice, w.D, w.shape, w.precision, w.xi0, w.steps, bc=w.bc)
    assert_parity(gpu, orc, "f64", w.name)


@pytest.mark.parametrize("rest", [True, False])
@pytest.mark.parametrize("shape", [(1,), (2,), (1, 1), (1, 5), (3, 1, 2)])
def test_degenerate_extents(shape, rest):
    lattice = ({1: "D1Q3", 2: "D2Q5", 3: "D3Q7"} if rest else {1: "D1Q2", 2: "D2Q4", 3: "D3Q6"})[len(shape)]
    rng = np.random.default_rng(8)
    D = rand_D(rng, 3)
    xi0 = rand_field(rng, 3, shape[::-1])
    orc = oracle_run(oracle_problem(lattice, D, shape), xi0, 9)
    for launch in (dict(lds_resident=1), dict(lds_resident=0)):
        gpu = gpu_run(lattice, D, shape, "f64", xi0, 9, launch=launch)
        assert_parity(gpu, orc, "f64", f"{shape} {launch}")


@pytest.mark.parametrize("lattice", DIAG)
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("faces", range(3))
def test_diagonal_lattices_walls_on_every_face(lattice, precision, faces):
    """Walls on every face, of both kinds, so that diagonal directions leave through
    edges and corners where two or three wall faces meet (the wall of the lowest
    axis decides), and mixed with periodic axes."""
    kinds = [
        (("dirichlet", "zero_flux"), ("zero_flux", "dirichlet"), ("dirichlet", "zero_flux")),
        (("zero_flux", "zero_flux"), ("dirichlet", "dirichlet"), ("zero_flux", "dirichlet")),
        (("periodic", "periodic"), ("dirichlet", "zero_flux"), ("periodic", "periodic")),
    ][faces]
    rng = np.random.default_rng(1300 + faces)
    N = 3
    D = rand_D(rng, N)
    shape = {"D2Q9": (71, 38), "D3Q15": (29, 17, 10)}[lattice]
    bc = kinds[: len(shape)]
    walls = {}
    for a, (lo, hi) in enumerate(bc):
        for side, kind in enumerate((lo, hi)):
            if kind == "dirichlet":
                walls[(a, side)] = rand_field(rng, N, ())
    xi0 = rand_field(rng, N, shape[::-1])
    orc = oracle_run(oracle_problem(lattice, D, shape, bc=bc, xi_wall=walls), xi0, 35)
    gpu = gpu_run(lattice, D, shape, precision, xi0, 35, bc=bc, xi_wall=walls)
    assert_parity(gpu, orc, precision, f"{lattice} faces {faces} {precision}")


@pytest.mark.parametrize("shape", [(1, 1), (1, 6), (5, 1), (13, 8), (1, 1, 1), (3, 1, 2), (9, 7, 5)])
def test_diagonal_lattices_small_and_degenerate(shape):
    """Extents of one node (every diagonal wraps onto its own row or column) and
    small grids, through the LDS-resident kernel and the global one."""
    lattice = {2: "D2Q9", 3: "D3Q15"}[len(shape)]
    rng = np.random.default_rng(1400 + len(shape))
    D = rand_D(rng, 3)
    xi0 = rand_field(rng, 3, shape[::-1])
    bc = tuple(("zero_flux", "dirichlet") if n > 2 else ("periodic", "periodic") for n in shape)
    walls = {(a, 1): rand_field(rng, 3, ()) for a, n in enumerate(shape) if n > 2}
    orc = oracle_run(oracle_problem(lattice, D, shape, bc=bc, xi_wall=walls), xi0, 11)
    for launch in (dict(lds_resident=1), dict(lds_resident=0)):
        gpu = gpu_run(lattice, D, shape, "f64", xi0, 11, bc=bc, xi_wall=walls, launch=launch)
        assert_parity(gpu, orc, "f64", f"{lattice} {shape} {launch}")


@pytest.mark.parametrize("lattice", ["D1Q3", "D2Q5", "D3Q7", "D2Q4", "D2Q9", "D3Q15"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("linearised", [False, True])
def test_dilute_species_mode(lattice, precision, linearised):
    """Remark III's diagonal B (Eqs. (2-16), (2-17)) with Dirichlet and zero-flux
    walls, TRT relaxation, four species, one step per pass (the vector width is a
    hint the mode ignores)."""
    rng = np.random.default_rng(1500 + len(lattice))
    N = 4
    D = rand_D(rng, N)
    shape = SHAPES[lattice]
    bc = _bc(lattice, [("dirichlet", "zero_flux"), ("periodic", "periodic"), ("zero_flux", "dirichlet")])
    walls = {}
    for a, (lo, hi) in enumerate(bc):
        for side, kind in enumerate((lo, hi)):
            if kind == "dirichlet":
                walls[(a, side)] = rand_field(rng, N, ())
    xref = rand_field(rng, N, ()) if linearised else None
    xi0 = rand_field(rng, N, shape[::-1])
    orc = oracle_run(oracle_problem(lattice, D, shape, bc=bc, xi_wall=walls, relax="trt", trt_magic=0.3,
                                    xi_ref=xref, dilute=True), xi0, 30)
    gpu = gpu_run(lattice, D, shape, precision, xi0, 30, bc=bc, xi_wall=walls, relax="trt", trt_magic=0.3,
                  xi_ref=xref, dilute=True, launch=dict(vec=4, lds_resident=0, temporal=0))
    assert_parity(gpu, orc, precision, f"{lattice} dilute {precision} lin={linearised}")


def test_dilute_species_mode_lds_resident_and_steps_per_pass():
    """Small grid through the LDS-resident kernel; on D2Q5 the same steps per pass
    as the full model."""
    from paper_1808_06787_amd.sim import Sim

    rng = np.random.default_rng(1550)
    D = rand_D(rng, 3)
    shape = (21, 13)
    xi0 = rand_field(rng, 3, shape[::-1])
    orc = oracle_run(oracle_problem("D2Q5", D, shape, dilute=True), xi0, 25)
    gpu = gpu_run("D2Q5", D, shape, "f64", xi0, 25, dilute=True, launch=dict(lds_resident=1))
    assert_parity(gpu, orc, "f64", "dilute lds")
    n = 2048     # large enough for the blocked sweep (smaller domains run one step per pass)
    full = Sim("D2Q5", D, (n, n), "f32")
    sim = Sim("D2Q5", D, (n, n), "f32", dilute=True)
    assert sim.steps_per_pass() == full.steps_per_pass() > 1
    full.close()
    sim.close()


def test_zero_steps_reads_initial_state():
    rng = np.random.default_rng(9)
    D = rand_D(rng, 4)
    xi0 = rand_field(rng, 4, (13, 17))
    orc = oracle_run(oracle_problem("D2Q5", D, (17, 13)), xi0, 0)
    gpu = gpu_run("D2Q5", D, (17, 13), "f64", xi0, 0)
    assert_parity(gpu, orc, "f64", "t=0")
    np.testing.assert_allclose(gpu[0], xi0, rtol=0, atol=1e-15)


VEC_SHAPES = {"D1Q3": (1028,), "D2Q5": (1028, 13), "D3Q7": (68, 9, 5),
              "D1Q2": (1028,), "D2Q4": (1028, 13), "D3Q6": (68, 9, 5),
              "D2Q9": (1028, 13), "D3Q15": (68, 9, 5)}     # diagonal lattices ignore the vector width


@pytest.mark.parametrize("lattice", ALL)
@pytest.mark.parametrize("vec", [0, 1, 2, 4])
@pytest.mark.parametrize("xface", ["periodic", "zero_flux", "dirichlet"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_vectorised_paths(lattice, vec, xface, precision):
    """Rows whose length is a multiple of 4 (several waves per row, a partial last
    tile) exercise the V-wide loads and the lane exchange of the +-x neighbours."""
    rng = np.random.default_rng(900 + vec)
    N = 3
    D = rand_D(rng, N)
    shape = VEC_SHAPES[lattice]
    d = len(shape)
    bc = ((xface, xface),) + (("zero_flux", "zero_flux"), ("periodic", "periodic"))[: d - 1]
    walls = {}
    if xface == "dirichlet":
        walls = {(0, 0): rand_field(rng, N, ()), (0, 1): rand_field(rng, N, ())}
    xi0 = smooth_field(rng, N, shape[::-1], 0.15)
    steps = 23
    orc = oracle_run(oracle_problem(lattice, D, shape, bc=bc, xi_wall=walls), xi0, steps)
    gpu = gpu_run(lattice, D, shape, precision, xi0, steps, bc=bc, xi_wall=walls,
                  launch=dict(vec=vec, lds_resident=0, temporal=0))
    assert_parity(gpu, orc, precision, f"{lattice} vec={vec} {xface} {precision}")


def test_vector_widths_agree_to_rounding():
    """The vectorised kernels run the same per-node arithmetic; the compiler may
    contract it into FMAs differently, so they agree with the general kernel to a
    few FP32 ulps (each is separately pinned to the oracle above)."""
    rng = np.random.default_rng(41)
    D = rand_D(rng, 4)
    shape = (512, 37)
    xi0 = smooth_field(rng, 4, shape[::-1], 0.1)
    ref = gpu_run("D2Q5", D, shape, "f32", xi0, 17, launch=dict(vec=0, temporal=0))
    for launch in (dict(vec=1), dict(vec=2, block_x=64, block_y=4), dict(vec=4, block_x=128, block_y=2),
                   dict(vec=4, block_x=64, block_y=1, xcd_remap=0, nontemporal=7)):
        got = gpu_run("D2Q5", D, shape, "f32", xi0, 17, launch=dict(launch, temporal=0))
        np.testing.assert_allclose(got[0], ref[0], rtol=0, atol=2e-6, err_msg=str(launch))


@pytest.mark.parametrize("vec", [0, 1, 4])
def test_streaming_hints_and_padding_do_not_change_results(vec):
    """Non-temporal hints and plane padding change only where bytes live in the
    caches and in memory: results are bitwise identical."""
    import torch

    from paper_1808_06787_amd.sim import Sim

    rng = np.random.default_rng(42)
    D = rand_D(rng, 3)
    shape = (256, 21, 6)
    xi0 = smooth_field(rng, 3, shape[::-1], 0.1)
    outs = []
    for nt, pad in ((0, 0), (7, 0), (2, 64), (5, 128)):
        sim = Sim("D3Q7", D, shape, "f32", plane_pad=pad)
        sim.set_launch(vec=vec, nontemporal=nt)
        sim.init(torch.from_numpy(xi0))
        sim.step(11)
        outs.append(sim.read()[0].cpu().numpy())
        sim.close()
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


BLOCKED_CASES = [
    ((301, 29), (("zero_flux", "zero_flux"), ("periodic", "periodic"))),
    ((257, 40), (("periodic", "periodic"), ("dirichlet", "zero_flux"))),
    ((70, 130), (("dirichlet", "dirichlet"), ("zero_flux", "dirichlet"))),
    ((3, 700), (("periodic", "periodic"), ("periodic", "periodic"))),
    ((2, 50), (("zero_flux", "zero_flux"), ("dirichlet", "zero_flux"))),
]


@pytest.mark.parametrize("case", range(len(BLOCKED_CASES)))
@pytest.mark.parametrize("tb", [2, 3, 4, 6])
@pytest.mark.parametrize("N", [2, 3, 5])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_temporally_blocked_sweep(case, tb, N, precision):
    """Several steps per pass over HBM (rows of each time level in LDS): ragged
    tiles and row segments, every face kind, odd step counts (remainder single
    steps) and the pre-collision first step."""
    shape, bc = BLOCKED_CASES[case]
    rng = np.random.default_rng(300 + 10 * case + N)
    D = rand_D(rng, N)
    walls = {}
    for a, (lo, hi) in enumerate(bc):
        for s, kind in enumerate((lo, hi)):
            if kind == "dirichlet":
                walls[(a, s)] = rand_field(rng, N, ())
    xi0 = smooth_field(rng, N, shape[::-1], 0.15)
    steps = 23
    orc = oracle_run(oracle_problem("D2Q5", D, shape, bc=bc, xi_wall=walls), xi0, steps)
    for seg in (5, 32):
        gpu = gpu_run("D2Q5", D, shape, precision, xi0, steps, bc=bc, xi_wall=walls,
                      launch=dict(temporal=tb, seg_rows=seg, lds_resident=0), split=[1, 6, 16])
        assert_parity(gpu, orc, precision, f"blocked tb={tb} seg={seg} {shape} N={N} {precision}")


@pytest.mark.parametrize("N", [2, 3, 4])
@pytest.mark.parametrize("faces", [(("periodic", "periodic"), ("periodic", "periodic")),
                                   (("dirichlet", "zero_flux"), ("zero_flux", "dirichlet"))])
def test_blocked_sweep_wide_tiles(N, faces):
    """Domains of 6144 columns or more take 512-column tiles for full passes (FP32:
    six steps for up to two evolved species, five for three when x and y are
    periodic); shorter passes use 256 columns.  An explicit segment height keeps
    the blocked plan on this short domain (automatic segments would leave too
    few workgroups and fall back to one step per pass).  Calls of 1, tb, tb, 4 and
    3 steps: a single step from the initial state, two full passes, then passes
    of 4 and 3 steps on 256-column tiles."""
    from paper_1808_06787_amd.sim import Sim

    shape = (6250, 23)
    tb = 6 if N <= 3 else 5
    rng = np.random.default_rng(1600 + N)
    D = rand_D(rng, N)
    walls = {}
    for a, (lo, hi) in enumerate(faces):
        for side, kind in enumerate((lo, hi)):
            if kind == "dirichlet":
                walls[(a, side)] = rand_field(rng, N, ())
    launch = dict(lds_resident=0, seg_rows=8)
    probe = Sim("D2Q5", D, shape, "f32", bc=faces, xi_wall=walls)
    probe.set_launch(**launch)
    assert probe.steps_per_pass() == tb
    probe.close()
    split = [1, tb, tb, 4, 3]
    steps = sum(split)
    xi0 = smooth_field(rng, N, shape[::-1], 0.15)
    orc = oracle_run(oracle_problem("D2Q5", D, shape, bc=faces, xi_wall=walls), xi0, steps)
    gpu = gpu_run("D2Q5", D, shape, "f32", xi0, steps, bc=faces, xi_wall=walls, launch=launch, split=split)
    assert_parity(gpu, orc, "f32", f"wide tiles N={N} {faces}")


@pytest.mark.parametrize("tb", [2, 3, 4, 5, 6])
@pytest.mark.parametrize("steps", [1, 2, 7, 13, 20, 25])
def test_blocked_runs_split_into_near_equal_passes(tb, steps):
    """A run of `steps` from the initial state: one single step, then
    ceil((steps - 1) / tb) passes of near-equal length (no short remainder pass);
    the field matches the oracle whatever the split."""
    shape, bc = BLOCKED_CASES[2]
    rng = np.random.default_rng(1700 + tb)
    N = 3
    D = rand_D(rng, N)
    walls = {}
    for a, (lo, hi) in enumerate(bc):
        for s, kind in enumerate((lo, hi)):
            if kind == "dirichlet":
                walls[(a, s)] = rand_field(rng, N, ())
    xi0 = smooth_field(rng, N, shape[::-1], 0.15)
    orc = oracle_run(oracle_problem("D2Q5", D, shape, bc=bc, xi_wall=walls), xi0, steps)
    gpu = gpu_run("D2Q5", D, shape, "f64" if tb <= 3 else "f32", xi0, steps, bc=bc, xi_wall=walls,
                  launch=dict(temporal=tb, seg_rows=6, lds_resident=0))
    assert_parity(gpu, orc, "f64" if tb <= 3 else "f32", f"split tb={tb} steps={steps}")


@pytest.mark.parametrize("case", range(len(BLOCKED_CASES)))
@pytest.mark.parametrize("tb", [2, 3, 5, 6])
@pytest.mark.parametrize("N", [2, 3, 5])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_temporally_blocked_sweep_dilute(case, tb, N, precision):
    """The dilute-species collision (Remark III) inside the blocked sweep, with
    the linearised theory on every other case."""
    shape, bc = BLOCKED_CASES[case]
    rng = np.random.default_rng(700 + 10 * case + N)
    D = rand_D(rng, N)
    walls = {}
    for a, (lo, hi) in enumerate(bc):
        for s, kind in enumerate((lo, hi)):
            if kind == "dirichlet":
                walls[(a, s)] = rand_field(rng, N, ())
    xref = rand_field(rng, N, ()) if case % 2 else None
    xi0 = smooth_field(rng, N, shape[::-1], 0.15)
    steps = 23
    orc = oracle_run(oracle_problem("D2Q5", D, shape, bc=bc, xi_wall=walls, xi_ref=xref, dilute=True), xi0, steps)
    gpu = gpu_run("D2Q5", D, shape, precision, xi0, steps, bc=bc, xi_wall=walls, xi_ref=xref, dilute=True,
                  launch=dict(temporal=tb, seg_rows=7, lds_resident=0), split=[1, 6, 16])
    assert_parity(gpu, orc, precision, f"blocked dilute tb={tb} {shape} N={N} {precision}")


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("magic", [0.05, 0.5, 2.0])
def test_temporally_blocked_sweep_trt(precision, magic):
    """The TRT rule through the blocked sweep (the collision coefficients carry the
    product parameter): walls, ragged tiles, 6 steps per pass."""
    shape, bc = BLOCKED_CASES[2]
    rng = np.random.default_rng(330)
    N = 3
    D = rand_D(rng, N)
    walls = {(a, s): rand_field(rng, N, ()) for a, (lo, hi) in enumerate(bc) for s, kind in enumerate((lo, hi))
             if kind == "dirichlet"}
    xi0 = smooth_field(rng, N, shape[::-1], 0.15)
    steps = 19
    orc = oracle_run(oracle_problem("D2Q5", D, shape, bc=bc, xi_wall=walls, relax="trt", trt_magic=magic), xi0, steps)
    gpu = gpu_run("D2Q5", D, shape, precision, xi0, steps, bc=bc, xi_wall=walls, relax="trt", trt_magic=magic,
                  launch=dict(temporal=6, seg_rows=16, lds_resident=0))
    assert_parity(gpu, orc, precision, f"blocked trt magic={magic} {precision}")


def test_blocked_sweep_matches_single_step_sweep():
    rng = np.random.default_rng(310)
    D = rand_D(rng, 3)
    shape = (500, 97)
    xi0 = smooth_field(rng, 3, shape[::-1], 0.1)
    ref = gpu_run("D2Q5", D, shape, "f32", xi0, 41, launch=dict(lds_resident=0, temporal=0))
    for tb in (2, 3, 4, 5, 6):
        got = gpu_run("D2Q5", D, shape, "f32", xi0, 41, launch=dict(temporal=tb, seg_rows=16, lds_resident=0))
        for a, b in zip(ref, got):
            np.testing.assert_allclose(a, b, rtol=0, atol=2e-6)


def test_steps_per_pass_plan():
    """The library takes the largest pass its on-chip window allows for the species
    count and precision, and one step per pass where it cannot fill the GPU."""
    import torch

    from paper_1808_06787_amd.sim import Sim

    rng = np.random.default_rng(320)
    cases = [  # (N, precision, shape, launch, expected steps per pass)
        (3, "f32", (4096, 512), {}, 6),
        (3, "f32", (4096, 4096), dict(temporal=4, seg_rows=0), 4),
        (2, "f64", (2048, 512), {}, 6),
        (4, "f32", (2048, 1024), {}, 6),
        (4, "f32", (2048, 1024), dict(bc=(("zero_flux", "zero_flux"), ("periodic", "periodic"))), 5),
        (5, "f32", (2048, 1024), {}, 5),
        (5, "f32", (2048, 1024), dict(bc=(("zero_flux", "zero_flux"), ("periodic", "periodic"))), 3),
        (3, "f64", (2048, 1024), {}, 3),
        (4, "f64", (2048, 1024), {}, 1),
        (3, "f32", (2048, 1024), dict(temporal=3), 3),
        (3, "f32", (2048, 1024), dict(temporal=0), 1),
        (3, "f32", (200, 100), {}, 1),
        (3, "f32", (512, 512), {}, 1),
        (3, "f32", (1024, 1024), {}, 6),
        (3, "f32", (200, 100), dict(seg_rows=8), 6),
    ]
    for N, prec, shape, launch, want in cases:
        launch = dict(launch)
        bc = launch.pop("bc", None)
        sim = Sim("D2Q5", rand_D(rng, N), shape, prec, bc=bc)
        if launch:
            sim.set_launch(**launch)
        assert sim.steps_per_pass() == want, (N, prec, shape, launch)
        sim.close()
    sim = Sim("D3Q7", rand_D(rng, 3), (64, 64, 64), "f32")
    assert sim.steps_per_pass() == 1
    sim.close()


BLOCKED3D_CASES = [
    # shape, faces, (tile_x, tile_y), z-planes per workgroup
    ((70, 21, 13), (("zero_flux", "zero_flux"), ("periodic", "periodic"), ("periodic", "periodic")), (16, 5), 4),
    ((37, 19, 11), (("periodic", "periodic"), ("periodic", "periodic"), ("periodic", "periodic")), (64, 9), 8),
    ((23, 17, 9), (("dirichlet", "zero_flux"), ("zero_flux", "dirichlet"), ("dirichlet", "zero_flux")), (8, 6), 3),
    ((9, 30, 14), (("periodic", "periodic"), ("dirichlet", "dirichlet"), ("zero_flux", "zero_flux")), (5, 7), 5),
    ((1, 13, 6), (("periodic", "periodic"), ("zero_flux", "dirichlet"), ("periodic", "periodic")), (4, 4), 2),
    ((12, 1, 1), (("zero_flux", "dirichlet"), ("periodic", "periodic"), ("periodic", "periodic")), (7, 3), 1),
    ((5, 4, 3), (("periodic", "periodic"), ("periodic", "periodic"), ("zero_flux", "dirichlet")), (2, 2), 1),
]


@pytest.mark.parametrize("case", range(len(BLOCKED3D_CASES)))
@pytest.mark.parametrize("lattice", ["D3Q7", "D3Q6"])
@pytest.mark.parametrize("N", [2, 3, 4])
def test_temporally_blocked_sweep_3d(case, lattice, N):
    """Two steps per pass in 3D (an x-y tile plus a ring of one node marching along
    z, the first step's values on chip): ragged tiles and z-segments, every face
    kind on every axis, extents of one node, the pre-collision first step and
    passes of near-equal length (calls of 1, 6 and 16 steps), FP32 against the
    oracle."""
    from paper_1808_06787_amd.sim import Sim

    shape, bc, (tx, ty), zseg = BLOCKED3D_CASES[case]
    rng = np.random.default_rng(1800 + 10 * case + N)
    D = rand_D(rng, N)
    walls = {}
    for a, (lo, hi) in enumerate(bc):
        for s, kind in enumerate((lo, hi)):
            if kind == "dirichlet":
                walls[(a, s)] = rand_field(rng, N, ())
    xi0 = smooth_field(rng, N, shape[::-1], 0.15)
    launch = dict(temporal=2, seg_rows=zseg, tile_x=tx, tile_y=ty, lds_resident=0)
    probe = Sim(lattice, D, shape, "f32", bc=bc, xi_wall=walls)
    probe.set_launch(**launch)
    assert probe.steps_per_pass() == 2
    probe.close()
    steps = 23
    orc = oracle_run(oracle_problem(lattice, D, shape, bc=bc, xi_wall=walls), xi0, steps)
    gpu = gpu_run(lattice, D, shape, "f32", xi0, steps, bc=bc, xi_wall=walls, launch=launch, split=[1, 6, 16])
    assert_parity(gpu, orc, "f32", f"blocked 3D {lattice} {shape} N={N} tile {tx}x{ty} zseg {zseg}")


@pytest.mark.parametrize("xcd_remap", [0, 1])
def test_temporally_blocked_sweep_3d_default_tile(xcd_remap):
    """The automatic tile (64 x 9 for three evolved species) on a domain of several
    tiles and segments in each direction, zero-flux x walls as in the 512^3
    workload, with and without the XCD remapping of workgroups."""
    shape = (150, 40, 37)
    bc = (("zero_flux", "zero_flux"), ("periodic", "periodic"), ("periodic", "periodic"))
    rng = np.random.default_rng(1900 + xcd_remap)
    N = 4
    D = rand_D(rng, N, 0.02, 0.8)
    xi0 = smooth_field(rng, N, shape[::-1], 0.1)
    steps = 9
    orc = oracle_run(oracle_problem("D3Q7", D, shape, bc=bc), xi0, steps)
    gpu = gpu_run("D3Q7", D, shape, "f32", xi0, steps, bc=bc,
                  launch=dict(temporal=2, seg_rows=8, xcd_remap=xcd_remap, lds_resident=0))
    assert_parity(gpu, orc, "f32", f"blocked 3D default tile remap={xcd_remap}")


@pytest.mark.parametrize("case", range(len(BLOCKED_CASES)))
@pytest.mark.parametrize("tb", [2, 3, 5, 6])
@pytest.mark.parametrize("N", [2, 3, 5])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_temporally_blocked_sweep_d2q4(case, tb, N, precision):
    """The blocked sweep on D2Q4 (Eq. (3-6), no rest direction): the D2Q5 row march
    without the rest population, on the same ragged tiles and segments, every face
    kind and the pre-collision first step; steps per pass as the plan gives them."""
    from paper_1808_06787_amd.sim import Sim

    shape, bc = BLOCKED_CASES[case]
    rng = np.random.default_rng(1800 + 10 * case + N)
    D = rand_D(rng, N)
    walls = {}
    for a, (lo, hi) in enumerate(bc):
        for s, kind in enumerate((lo, hi)):
            if kind == "dirichlet":
                walls[(a, s)] = rand_field(rng, N, ())
    xi0 = smooth_field(rng, N, shape[::-1], 0.15)
    steps = 23
    orc = oracle_run(oracle_problem("D2Q4", D, shape, bc=bc, xi_wall=walls), xi0, steps)
    # FP32: m <= 2 up to six steps, m = 4 up to five with x and y periodic and three otherwise;
    # FP64: m = 1 up to six, m = 2 up to three, m = 4 one
    periodic = all(kind == "periodic" for pair in bc for kind in pair)
    want = {2: min(tb, 6), 3: min(tb, 6), 5: min(tb, 5 if periodic else 3)}[N] if precision == "f32" else \
        {2: min(tb, 6), 3: min(tb, 3), 5: 1}[N]
    for seg in (5, 32):
        launch = dict(temporal=tb, seg_rows=seg, lds_resident=0)
        probe = Sim("D2Q4", D, shape, precision, bc=bc, xi_wall=walls)
        probe.set_launch(**launch)
        assert probe.steps_per_pass() == want, (N, precision, tb)
        probe.close()
        gpu = gpu_run("D2Q4", D, shape, precision, xi0, steps, bc=bc, xi_wall=walls, launch=launch, split=[1, 6, 16])
        assert_parity(gpu, orc, precision, f"D2Q4 blocked tb={tb} seg={seg} {shape} N={N} {precision}")


# Widths at which the last tile of a row needs exactly 64 or 65 lanes (its output columns and TB
# halo columns on either side), with one column tile and with two: the boundary between the waves
# that run the row march and the waves past it, which only join the march's barriers.
LAST_TILE_WIDTHS = {6: (52, 53, 296, 297), 3: (58, 59, 308, 309)}


@pytest.mark.parametrize("tb", [3, 6])
@pytest.mark.parametrize("k", range(4))
@pytest.mark.parametrize("xbc", [("periodic", "periodic"), ("zero_flux", "dirichlet")])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_blocked_sweep_last_tile_wave_boundary(tb, k, xbc, precision):
    """The blocked sweep where the last tile's live lanes end exactly at a wave boundary or one
    lane past it, periodic and walled in x (the wall at the last column lies in that tile)."""
    from paper_1808_06787_amd.sim import Sim

    shape = (LAST_TILE_WIDTHS[tb][k], 14)
    N = 3 if precision == "f32" else 2          # six steps per pass: FP32 m <= 2, FP64 m = 1
    bc = (xbc, ("periodic", "periodic"))
    rng = np.random.default_rng(2200 + 10 * tb + k)
    D = rand_D(rng, N)
    walls = {(0, 1): rand_field(rng, N, ())} if xbc[1] == "dirichlet" else {}
    xi0 = smooth_field(rng, N, shape[::-1], 0.15)
    steps = 2 * tb + 2
    orc = oracle_run(oracle_problem("D2Q5", D, shape, bc=bc, xi_wall=walls), xi0, steps)
    launch = dict(temporal=tb, seg_rows=5, lds_resident=0)
    probe = Sim("D2Q5", D, shape, precision, bc=bc, xi_wall=walls)
    probe.set_launch(**launch)
    assert probe.steps_per_pass() == tb, (shape, tb, precision)
    probe.close()
    gpu = gpu_run("D2Q5", D, shape, precision, xi0, steps, bc=bc, xi_wall=walls, launch=launch)
    assert_parity(gpu, orc, precision, f"last tile tb={tb} {shape} {xbc} {precision}")


@pytest.mark.parametrize("lattice", ["D2Q5", "D2Q4"])
@pytest.mark.parametrize("shape", [(301, 29), (600, 41), (90, 130)])
@pytest.mark.parametrize("dilute", [False, True])
def test_blocked_sweep_quinary_periodic_passes(lattice, shape, dilute):
    """Five species in FP32 on a periodic domain: five steps per pass (three with walls), over
    several column tiles and ragged segments, calls of 1, 5, 4, 3 and 2 steps."""
    from paper_1808_06787_amd.sim import Sim

    N = 5
    rng = np.random.default_rng(2400 + shape[0])
    D = rand_D(rng, N)
    bc = (("periodic", "periodic"), ("periodic", "periodic"))
    xi0 = smooth_field(rng, N, shape[::-1], 0.15)
    split = [1, 5, 4, 3, 2]
    orc = oracle_run(oracle_problem(lattice, D, shape, bc=bc, dilute=dilute), xi0, sum(split))
    launch = dict(seg_rows=7, lds_resident=0)
    probe = Sim(lattice, D, shape, "f32", bc=bc, dilute=dilute)
    probe.set_launch(**launch)
    assert probe.steps_per_pass() == 5, (lattice, shape)
    probe.close()
    walled = Sim(lattice, D, shape, "f32", bc=(("zero_flux", "zero_flux"), ("periodic", "periodic")),
                 dilute=dilute)
    walled.set_launch(**launch)
    assert walled.steps_per_pass() == 3, (lattice, shape)
    walled.close()
    gpu = gpu_run(lattice, D, shape, "f32", xi0, sum(split), bc=bc, launch=launch, split=split, dilute=dilute)
    assert_parity(gpu, orc, "f32", f"quinary periodic passes {lattice} {shape} dilute={dilute}")


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("launch", [None, dict(temporal=6, seg_rows=8, lds_resident=0)])
def test_absent_species_reduces_to_the_binary_mixture(precision, launch):
    """A ternary mixture whose second species is absent everywhere (xi_2 = 0):
    the row of B for that species is diagonal (Eq. (2-10)), so it stays absent
    and the others evolve as the binary mixture with D = D_13.  The ternary run
    (m = 2 kernels) matches the oracle and the binary run (m = 1 kernels), one
    step per pass and through six-step blocked passes."""
    rng = np.random.default_rng(88)
    shape = (300, 24)
    bc = (("periodic", "periodic"), ("zero_flux", "zero_flux"))
    D3 = rand_D(rng, 3, 0.05, 0.5)
    D2 = np.array([[1.0, D3[0, 2]], [D3[0, 2], 1.0]])
    two = smooth_field(rng, 2, shape[::-1], 0.1)
    three = np.stack([two[0], np.zeros(shape[::-1]), two[1]])
    steps = 25
    got3 = gpu_run("D2Q5", D3, shape, precision, three, steps, bc=bc, launch=launch)
    got2 = gpu_run("D2Q5", D2, shape, precision, two, steps, bc=bc, launch=launch)
    assert_parity(got3, oracle_run(oracle_problem("D2Q5", D3, shape, bc=bc), three, steps), precision, "ternary")
    tol = 1e-13 if precision == "f64" else 2e-6
    assert np.abs(got3[0][1]).max() <= (1e-15 if precision == "f64" else 1e-7)
    assert np.abs(got3[1][1]).max() <= (1e-15 if precision == "f64" else 1e-7)
    np.testing.assert_allclose(got3[0][0], got2[0][0], rtol=0, atol=tol)
    np.testing.assert_allclose(got3[0][2], got2[0][1], rtol=0, atol=tol)
    np.testing.assert_allclose(got3[1][0], got2[1][0], rtol=0, atol=tol)


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("N", [4, 5, 8])
def test_equal_diffusivities_decouple_the_species(N, precision):
    """Remark II: with every D_ij equal, B = I/D (Eq. (2-15)), so the small
    inverse of the collision (cofactors for three and four evolved species,
    pivoted elimination for seven) is diagonal and each species evolves as the
    binary mixture (xi_i, 1 - xi_i) with the same D.  The N-species run matches
    the oracle and, species by species, the binary kernels."""
    rng = np.random.default_rng(90 + N)
    shape = (90, 40)
    d = 0.12
    xi0 = smooth_field(rng, N, shape[::-1], 0.1)
    steps = 30
    got = gpu_run("D2Q5", np.full((N, N), d), shape, precision, xi0, steps)
    assert_parity(got, oracle_run(oracle_problem("D2Q5", np.full((N, N), d), shape), xi0, steps), precision,
                  f"N={N}")
    tol = 1e-13 if precision == "f64" else 2e-6
    for i in range(N - 1):
        pair = np.stack([xi0[i], 1.0 - xi0[i]])
        bin_ = gpu_run("D2Q5", np.full((2, 2), d), shape, precision, pair, steps)
        np.testing.assert_allclose(got[0][i], bin_[0][0], rtol=0, atol=tol, err_msg=f"xi_{i}")
        np.testing.assert_allclose(got[1][i], bin_[1][0], rtol=0, atol=tol, err_msg=f"J_{i}")
