"""Batched sweep: every mixture of a heterogeneous batch matches the oracle, all
schedules give identical fields, the one-launch-per-mixture reference schedule
agrees, checkpoints and the autotuner leave the state intact, and the full
256-mixture workload matches the oracle on sampled nodes."""
import numpy as np
import pytest
import torch

from gpu_cases import assert_parity, oracle_problem, oracle_run, rand_D, rand_field, smooth_field

pytestmark = pytest.mark.gpu


def _specs(lattice, rng):
    if lattice in ("D2Q5", "D2Q4", "D2Q9"):
        shapes = [(64, 64), (97, 45), (128, 33), (65, 70), (1, 1), (130, 7)]
        Ns = [2, 3, 4, 5, 3, 6]
    else:
        shapes = [(16, 8, 8), (9, 13, 5), (32, 4, 3), (5, 5, 5)]
        Ns = [3, 4, 5, 2]
    d = len(shapes[0])
    specs = []
    for b, (shape, N) in enumerate(zip(shapes, Ns)):
        bc = None
        walls = None
        if b % 3 == 1:
            bc = (("zero_flux", "zero_flux"),) + (("periodic", "periodic"),) * (d - 1)
        elif b % 3 == 2:
            bc = (("dirichlet", "zero_flux"),) + (("periodic", "periodic"),) * (d - 1)
            walls = {(0, 0): rand_field(rng, N, ())}
        specs.append(dict(D=rand_D(rng, N), shape=shape, bc=bc, xi_wall=walls,
                          relax="srt" if b == 3 else ("trt" if b == 2 else "paper"), trt_magic=0.4))
    fields = [smooth_field(rng, sp["D"].shape[0], sp["shape"][::-1], 0.1) for sp in specs]
    return specs, fields


def _batch(lattice, precision, specs, fields):
    from paper_1808_06787_amd.batch import Batch

    b = Batch(specs, lattice, precision)
    for i, f in enumerate(fields):
        b.init(i, torch.from_numpy(f))
    return b


def _read_all(b):
    out = []
    for i in range(b.count):
        xi, J, g = b.read(i)
        out.append((xi.cpu().numpy(), J.cpu().numpy(), g.cpu().numpy()))
    return out


@pytest.mark.parametrize("lattice", ["D2Q5", "D3Q7", "D2Q4", "D3Q6", "D2Q9", "D3Q15"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_batch_matches_oracle_per_mixture(lattice, precision):
    rng = np.random.default_rng(70)
    specs, fields = _specs(lattice, rng)
    b = _batch(lattice, precision, specs, fields)
    b.step(25)
    got = _read_all(b)
    for i, (sp, f) in enumerate(zip(specs, fields)):
        p = oracle_problem(lattice, sp["D"], sp["shape"], bc=sp["bc"], xi_wall=sp["xi_wall"], relax=sp["relax"],
                           trt_magic=sp["trt_magic"])
        assert_parity(got[i], oracle_run(p, f, 25), precision, f"{lattice} mixture {i}")
    b.close()


@pytest.mark.parametrize("lattice", ["D2Q5", "D3Q7", "D2Q9"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("sched", [None, dict(temporal=0, mode="fused"), dict(temporal=3, seg_rows=8)])
def test_batch_with_dilute_species_mixtures(lattice, precision, sched):
    """Mixtures with the dilute-species collision (Remark III) next to full ones:
    they run in launches of their own (fused, per class, blocked), each against
    the oracle (blocked passes apply to D2Q5; the other lattices take single steps)."""
    rng = np.random.default_rng(75)
    specs, fields = _specs(lattice, rng)
    for i, sp in enumerate(specs):
        sp["dilute"] = i % 2 == 1
    b = _batch(lattice, precision, specs, fields)
    if sched:
        b.set_schedule(**sched)
    b.step(19)
    got = _read_all(b)
    for i, (sp, f) in enumerate(zip(specs, fields)):
        p = oracle_problem(lattice, sp["D"], sp["shape"], bc=sp["bc"], xi_wall=sp["xi_wall"], relax=sp["relax"],
                           trt_magic=sp["trt_magic"], dilute=sp["dilute"])
        assert_parity(got[i], oracle_run(p, f, 19), precision, f"{lattice} mixture {i} dilute={sp['dilute']}")
    b.close()


def test_schedules_are_bitwise_identical_and_match_reference_schedule():
    """One-step schedules move only the mapping of nodes to workgroups (bitwise
    identical fields); blocked passes run the same per-node arithmetic in another
    kernel (a few FP32 ulps); per-mixture launches agree as well."""
    rng = np.random.default_rng(71)
    specs, fields = _specs("D2Q5", rng)
    ref_b = _batch("D2Q5", "f32", specs, fields)
    ref_b.set_schedule(temporal=0)
    ref_b.step(13)
    ref = _read_all(ref_b)
    ref_b.close()
    for sched in (dict(block_x=256, block_y=1, mode="per_class", order="interleaved", xcd_remap=1),
                  dict(block_x=64, block_y=1, mode="fused", order="interleaved", xcd_remap=0, nontemporal=7),
                  dict(block_x=128, block_y=2, mode="per_class", order="instance", xcd_remap=1)):
        b = _batch("D2Q5", "f32", specs, fields)
        b.set_schedule(temporal=0, **sched)
        b.step(13)
        got = _read_all(b)
        for g, r in zip(got, ref):
            for x, y in zip(g, r):
                np.testing.assert_array_equal(x, y, err_msg=str(sched))
        b.close()
    for sched in (dict(temporal=4, seg_rows=16), dict(temporal=2, seg_rows=5, order="interleaved"),
                  dict(temporal=3, seg_rows=8, nontemporal=1)):
        b = _batch("D2Q5", "f32", specs, fields)
        b.set_schedule(**sched)
        b.step(5)
        b.step(8)
        got = _read_all(b)
        for g, r in zip(got, ref):
            for x, y in zip(g, r):
                np.testing.assert_allclose(x, y, rtol=0, atol=2e-6, err_msg=str(sched))
        b.close()
    e = _batch("D2Q5", "f32", specs, fields)
    e.step_each(13)
    got = _read_all(e)
    for g, r in zip(got, ref):
        np.testing.assert_allclose(g[0], r[0], rtol=0, atol=2e-6)
    e.close()


def test_blocked_batch_switches_schedules_midway():
    """Classes advance by passes of different lengths, so their buffer halves
    diverge; changing the schedule, stepping per mixture, saving and restoring in
    between must keep every mixture's state."""
    rng = np.random.default_rng(75)
    specs, fields = _specs("D2Q5", rng)
    ref_b = _batch("D2Q5", "f64", specs, fields)
    ref_b.set_schedule(temporal=0)
    ref_b.step(23)
    ref = _read_all(ref_b)
    ref_b.close()
    b = _batch("D2Q5", "f64", specs, fields)
    b.set_schedule(temporal=4, seg_rows=7)
    b.step(6)
    b.step_each(1)
    b.set_schedule(temporal=0, mode="fused")
    b.step(3)
    b.set_schedule(temporal=3, seg_rows=16)
    b.step(5)
    state, t = b.save()
    b.step(2)
    b.restore(state, t)
    b.step(8)
    assert b.time == 23
    for g, r in zip(_read_all(b), ref):
        for x, y in zip(g, r):
            np.testing.assert_allclose(x, y, rtol=0, atol=1e-13)
    b.close()


def test_batch_checkpoint_and_autotuner_keep_the_state(tmp_path):
    from paper_1808_06787_amd import autotune

    rng = np.random.default_rng(72)
    specs, fields = _specs("D2Q5", rng)
    a = _batch("D2Q5", "f64", specs, fields)
    a.step(20)
    ref = _read_all(a)
    a.close()
    b = _batch("D2Q5", "f64", specs, fields)
    b.step(8)
    res = autotune.tune_batch(b, cache_path=str(tmp_path / "tune.json"), steps=2, warmup=1)
    assert b.time == 8 and "best" in res and len(res["trials"]) > 10
    state, t = b.save()
    b.step(3)
    b.restore(state, t)
    b.step(12)
    # the tuned schedule may take passes of another length than the default: the
    # same arithmetic up to FMA contraction
    for g, r in zip(_read_all(b), ref):
        for x, y in zip(g, r):
            np.testing.assert_allclose(x, y, rtol=0, atol=1e-13)
    # cached result is applied without re-timing
    res2 = autotune.tune_batch(b, cache_path=str(tmp_path / "tune.json"))
    assert res2["best"] == res["best"] and b.get_schedule() == res["best"] and res2["trials"] == []
    # explicit candidates, cache ignored
    res3 = autotune.tune_batch(b, cache_path=str(tmp_path / "tune.json"), steps=2, force=True,
                               candidates=[dict(temporal=0, mode="fused"), dict(temporal=2, seg_rows=8)])
    assert len(res3["trials"]) == 2 and b.get_schedule() == res3["best"]
    b.close()


def test_batch_state_rules():
    from paper_1808_06787_amd._ffi import MsdError
    from paper_1808_06787_amd.batch import Batch

    rng = np.random.default_rng(73)
    specs, fields = _specs("D2Q5", rng)
    b = Batch(specs, "D2Q5", "f32")
    b.init(0, torch.from_numpy(fields[0]))
    with pytest.raises(MsdError) as e:
        b.step(1)                   # mixture 1 not initialised
    assert e.value.status == -9
    for i in range(1, b.count):
        b.init(i, torch.from_numpy(fields[i]))
    b.step(1)
    with pytest.raises(MsdError) as e:
        b.init(0, torch.from_numpy(fields[0]))
    assert e.value.status == -9
    b.close()


def test_batched_workload_sampled():
    """The 256-mixture workload (N in {3,4,5}, sides 64..1024) after 9 steps of the
    default schedule (blocked passes by class, as many steps per pass as each
    class's species count allows, with remainders): sampled nodes
    of several mixtures against the oracle on their light cones."""
    import workloads
    from paper_1808_06787_amd.batch import Batch

    ws = workloads.batched_2d()
    specs = [dict(D=w.D, shape=w.shape, bc=w.bc) for w in ws]
    b = Batch(specs, "D2Q5", "f32")
    for i, w in enumerate(ws):
        b.init(i, torch.from_numpy(w.xi0))
    b.release_inputs()
    steps = 9
    b.step(steps)
    rng = np.random.default_rng(74)
    from oracle import lbm

    for i in rng.choice(len(ws), 6, replace=False):
        w = ws[i]
        xi, J, _ = b.read(int(i), torch.float64, grad=False)
        for _ in range(4):
            x, y = (int(v) for v in rng.integers(0, w.shape[0], size=2))
            h = steps + 1
            idx = [np.arange(c - h, c + h + 1) % w.shape[0] for c in (x, y)]
            sub = np.take(np.take(w.xi0, idx[1], axis=1), idx[0], axis=2)
            p = lbm.Problem("D2Q5", w.D, (2 * h + 1, 2 * h + 1),
                            bc=((lbm.ZERO_FLUX, lbm.ZERO_FLUX), (lbm.ZERO_FLUX, lbm.ZERO_FLUX)))
            oxi, _, oJ = lbm.observables(p, lbm.run(p, sub, steps))
            assert np.abs(xi[:, y, x].cpu().numpy() - oxi[:, h, h]).max() <= 1e-5
            assert np.abs(J[:, :, y, x].cpu().numpy() - oJ[:, :, h, h]).max() <= 2e-6
    b.close()


def test_graph_replays_match_direct_launches():
    """msd_batch_step replays a captured graph of a span of full passes (twice the
    least common multiple of the classes' steps per pass) for as many whole spans
    as a call holds; the fields equal those of direct launches bit for bit after
    every call, with reads, diagnostics and direct steps of the other batch in
    between (graph replays are checked after the first one too)."""
    rng = np.random.default_rng(76)
    specs, fields = _specs("D2Q5", rng)
    g = _batch("D2Q5", "f32", specs, fields)
    d = _batch("D2Q5", "f32", specs, fields)
    g.set_schedule(temporal=4, seg_rows=8, graph=1)
    d.set_schedule(temporal=4, seg_rows=8, graph=0)
    span = 24      # classes at 4 and 3 steps per pass (and single steps)
    for n in (1, 3 * span + 5, 2 * span + 2, span, 7, span):
        g.step(n)
        d.step(n)
        assert g.time == d.time
        got, ref = _read_all(g), _read_all(d)
        for a, b_ in zip(got, ref):
            for x, y in zip(a, b_):
                np.testing.assert_array_equal(x, y, err_msg=f"after {g.time} steps")
        g.diagnostics(0)
    t = g.time
    for i, (sp, f) in enumerate(zip(specs, fields)):
        p = oracle_problem("D2Q5", sp["D"], sp["shape"], bc=sp["bc"], xi_wall=sp["xi_wall"], relax=sp["relax"],
                           trt_magic=sp["trt_magic"])
        if i in (0, 3):
            assert_parity(got[i], oracle_run(p, f, t), "f32", f"graph mixture {i}")
    g.close()
    d.close()


def test_separate_handles_reference_matches_oracle():
    """msd_batch_step_separate advances each mixture as its own handle with the
    default launch would: the tiny mixtures through the LDS-resident kernel, the
    1024^2 one through automatic blocked passes, the rest one step per pass; every
    mixture matches the oracle."""
    from paper_1808_06787_amd.sim import Sim

    rng = np.random.default_rng(77)
    specs, fields = _specs("D2Q5", rng)
    big = dict(D=rand_D(rng, 3), shape=(1024, 1024), bc=None, xi_wall=None, relax="paper", trt_magic=0.4)
    specs.append(big)
    fields.append(smooth_field(rng, 3, (1024, 1024), 0.1))
    probe = Sim("D2Q5", big["D"], big["shape"], "f32")
    assert probe.steps_per_pass() == 6
    probe.close()
    b = _batch("D2Q5", "f32", specs, fields)
    b.step_separate(1)
    b.step_separate(12)
    assert b.time == 13
    got = _read_all(b)
    for i, (sp, f) in enumerate(zip(specs, fields)):
        p = oracle_problem("D2Q5", sp["D"], sp["shape"], bc=sp["bc"], xi_wall=sp["xi_wall"], relax=sp["relax"],
                           trt_magic=sp["trt_magic"])
        assert_parity(got[i], oracle_run(p, f, 13), "f32", f"separate mixture {i}")
    b.close()


@pytest.mark.parametrize("steps", [9, 13, 20])
def test_remainder_passes_match_oracle(steps):
    """Calls whose length is not a multiple of a class's steps per pass: full
    blocked passes, then one shorter pass for a remainder of two or more steps
    (a remainder of one is a single step).  Six, six and five steps per pass
    for the classes of 2, 3 and 4 evolved species (walled members hold the
    class of 3 at five and of 4 at three); every mixture matches the oracle
    after each call."""
    rng = np.random.default_rng(78)
    specs, fields = _specs("D2Q5", rng)
    b = _batch("D2Q5", "f32", specs, fields)
    b.set_schedule(temporal=6, seg_rows=8, graph=0)
    b.step(1)            # the first step reads pre-collision values: a single step
    b.step(steps)
    b.step(steps)
    t = b.time
    assert t == 1 + 2 * steps
    got = _read_all(b)
    for i, (sp, f) in enumerate(zip(specs, fields)):
        p = oracle_problem("D2Q5", sp["D"], sp["shape"], bc=sp["bc"], xi_wall=sp["xi_wall"], relax=sp["relax"],
                           trt_magic=sp["trt_magic"])
        assert_parity(got[i], oracle_run(p, f, t), "f32", f"remainder {steps}: mixture {i}")
    b.close()


@pytest.mark.parametrize("walled", [False, True])
def test_quinary_class_steps_per_pass(walled):
    """A class of five-species mixtures over several column tiles: five steps per
    pass when every member is periodic, three when one has an x wall (the class
    then launches the walled kernel); ragged widths, remainder passes, graph
    replay, against the oracle."""
    rng = np.random.default_rng(79 + int(walled))
    shapes = [(300, 40), (261, 33), (90, 70)]
    specs = []
    for j, shape in enumerate(shapes):
        bc = (("zero_flux", "dirichlet"), ("periodic", "periodic")) if (walled and j == 1) else None
        walls = {(0, 1): rand_field(rng, 5, ())} if bc else None
        specs.append(dict(D=rand_D(rng, 5), shape=shape, bc=bc, xi_wall=walls))
    fields = [smooth_field(rng, 5, sp["shape"][::-1], 0.1) for sp in specs]
    b = _batch("D2Q5", "f32", specs, fields)
    b.set_schedule(temporal=6, seg_rows=8)
    for n in (1, 8, 7):
        b.step(n)
    got = _read_all(b)
    for i, (sp, f) in enumerate(zip(specs, fields)):
        p = oracle_problem("D2Q5", sp["D"], sp["shape"], bc=sp["bc"], xi_wall=sp["xi_wall"])
        assert_parity(got[i], oracle_run(p, f, 16), "f32", f"quinary class walled={walled}: mixture {i}")
    b.close()
