"""Benchmark of the fused Maxwell-Stefan lattice Boltzmann sweep on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload quaternary_3d|ternary_2d|ternary_1d]
                    [--no-cpu-baseline] [--no-extras]

Default workload: 3D quaternary mixture on a 512^3 D3Q7 lattice in FP32
(zero-flux x walls, periodic y and z, two slabs with 1 % noise, random D_ij),
K = 500 steps timed after W warm-up steps.  One step is one fused
collide-and-stream update of every node (propagation with face rules, moments,
the local Maxwell-Stefan solve, relaxation, store).  Prints one JSON line:

  value        MLUPS = nodes * (N - 1) * K / seconds / 1e6 (node-component updates)
  roofline     HBM roofline of the sweep kernel: algorithmic bytes per launch
               (2 q (N-1) bytes-per-value per node: every distribution read once
               and written once per pass over the state) over the average launch
               duration measured with HIP events on the sweep's stream; `traffic`
               is the HBM bytes per launch from rocprofv3 counters (FETCH_SIZE +
               WRITE_SIZE, calibrated on a copy kernel), when a summary taken on
               the current kernel sources is committed under profiles/
  cpu_baseline the FP64 numpy oracle on a bounded sample of the same workload
  extras       the 2D ternary workload (temporally blocked: several steps per
               launch, bound by VALU issue, so reported against the FP32 vector
               peak), the other lattices, the 1D workload, the 256-mixture batch
               and the gradient workload, timed the same way
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
Q = {"D1Q3": 3, "D2Q5": 5, "D3Q7": 7, "D1Q2": 2, "D2Q4": 4, "D3Q6": 6, "D2Q9": 9, "D3Q15": 15}
KERNEL_SOURCES = ["paper_1808_06787_amd/csrc/msd_device.h", "paper_1808_06787_amd/csrc/msd_kernels.h",
                  "paper_1808_06787_amd/csrc/msd_blocked3d.h"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_profile(kind: str, workload: str) -> dict:
    """Key/value lines of a committed rocprofv3 summary (profiles/<kind>_<workload>.txt),
    or {} if absent or taken on a different version of the kernel sources."""
    path = os.path.join(ROOT, "profiles", f"{kind}_{workload}.txt")
    if not os.path.exists(path):
        return {}
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_sources_sha256_16") != kernel_hash():
        return {}
    return vals


def load_traffic(workload: str):
    """Measured HBM bytes per launch of the sweep kernel (FETCH_SIZE + WRITE_SIZE, calibrated
    on a copy kernel), or None."""
    try:
        return float(load_profile("traffic", workload)["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def load_valu_time(workload: str):
    """VALU issue time per launch (seconds at 2.4 GHz) from the SQ_INSTS_VALU count, or None."""
    try:
        return float(load_profile("valu", workload)["valu_issue_time_us_at_2.4GHz"]) * 1e-6
    except (KeyError, ValueError):
        return None


def _on_lattice(w, lattice: str):
    """The same inputs on another lattice of equal dimension."""
    import dataclasses

    return dataclasses.replace(w, name=w.name.replace(w.lattice.lower(), lattice.lower()), lattice=lattice)


def make_workload(name: str):
    import workloads

    if name == "ternary_2d":
        return workloads.ternary_2d()
    if name == "quaternary_3d":
        return workloads.quaternary_3d()
    if name == "ternary_1d":
        return workloads.ternary_1d()
    raise SystemExit(f"unknown workload {name}")


def time_sweep(w, steps: int, warmup: int, launch=None):
    """Run warm-up then `steps` timed steps; returns (seconds, sim)."""
    import torch

    from paper_1808_06787_amd.sim import Sim

    sim = Sim(w.lattice, w.D, w.shape, w.precision, bc=w.bc, relax=w.relax)
    if launch:
        sim.set_launch(**launch)
    sim.init(torch.from_numpy(w.xi0))
    sim.step(warmup)
    stream = sim.stream
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    sim.step(steps)
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1e3, sim


def time_steps(sim, n: int) -> float:
    """Seconds for sim.step(n), HIP events on the sim's stream."""
    import torch

    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(sim.stream)
    sim.step(n)
    b.record(sim.stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / 1e3


def sweep_record(w, seconds, steps, steps_per_pass=1):
    """MLUPS of a timed run of `steps` steps from t > 0, and the launch count.

    A launch of the blocked sweep advances `steps_per_pass` steps (the host plan
    splits a run into passes of near-equal length, so `launches` is the number
    of passes of at most that length)."""
    m = w.N - 1
    nodes = w.nodes
    spp = max(1, int(steps_per_pass))
    launches = -(-steps // spp)
    return dict(mlups=nodes * m * steps / seconds / 1e6, per_step=seconds / steps, launches=launches,
                per_launch=seconds / launches, steps_per_pass=spp)


def pass_bytes(w) -> int:
    """Algorithmic bytes of one pass over the state: every distribution of the
    N - 1 evolved species read once and written once (2 q (N-1) value sizes per node)."""
    s = 4 if w.precision == "f32" else 8
    return w.nodes * (w.N - 1) * 2 * Q[w.lattice] * s


# FP32 vector issue without packed instructions: 256 CUs x 4 SIMDs x 16 lanes x
# 2 flops per FMA x 2.4 GHz (the packed-FP32 figure, 157.3 TFLOP/s, needs
# instructions this build does not emit)
ALU_PEAK_F32_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
ALU_PEAK_F64_TFLOPS = ALU_PEAK_F32_TFLOPS


def collision_flops(m: int, q: int) -> int:
    """Floating-point operations of one node update (FMA = 2), counted from the
    collision's algebra: species sums m (q-1); A = I + (a/2) B, 2 m (m-1) FMAs;
    the scaled small inverse (cofactors for m <= 4); the relaxation rule, 12 per
    species; the non-equilibrium parts, m (q-1) FMAs; the relaxation, (m+1) FMAs per
    species and moving direction; the rest closure, m (q-1)."""
    inv = {1: 2, 2: 9, 3: 43, 4: 145}.get(m, 2 * m ** 3)
    return m * (q - 1) * (4 + 2 * (m + 1)) + 4 * m * (m - 1) + inv + 12 * m


def measure(w, steps, warmup, launch=None):
    """Time `steps` steps after `warmup`; returns the record, the launch used and
    the sim (open).  With several steps per launch the dominant kernel's launch
    duration is measured again, live, over whole passes right after the timed
    region (HIP events on the sweep's stream)."""
    seconds, sim = time_sweep(w, steps, warmup, launch)
    rec = sweep_record(w, seconds, steps, sim.steps_per_pass())
    if rec["steps_per_pass"] > 1:
        passes = max(1, min(rec["launches"], 100))
        rec["per_launch"] = time_steps(sim, passes * rec["steps_per_pass"]) / passes
        rec["per_launch_over"] = f"{passes} whole passes after the timed region"
    else:
        rec["per_launch_over"] = "the timed region"
    used = sim.get_launch()
    used["steps_per_pass"] = rec["steps_per_pass"]
    rec["launch"] = used
    return rec, sim


def hbm_roofline(w, rec):
    """HBM roofline of the sweep kernel: algorithmic bytes per launch (the
    per-step model, 2 q (N-1) value sizes per node, times the steps one launch
    performs) over the measured launch duration, so that frac is the metric's
    "% of HBM peak" (MLUPS x bytes per node-component update / peak).  With two
    steps per launch the first step's values stay on chip, so the kernel moves
    fewer bytes than that: `traffic` (rocprofv3 FETCH_SIZE + WRITE_SIZE per
    launch, when a profile of the current kernel sources is committed) and its
    rate say how busy HBM actually is."""
    bpl = pass_bytes(w) * rec["steps_per_pass"]
    achieved = bpl / rec["per_launch"] / 1e9
    traffic = load_traffic(w.name)
    out = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "algorithmic_bytes_per_launch": bpl,
        "steps_per_launch": rec["steps_per_pass"],
        "launches_timed": rec["launches"],
        "ms_per_launch": round(rec["per_launch"] * 1e3, 5),
        "ms_per_launch_measured_over": rec["per_launch_over"],
        "traffic_over_algorithmic": round(traffic / bpl, 4) if traffic else None,
        "traffic_GBps": round(traffic / rec["per_launch"] / 1e9, 1) if traffic else None,
        "traffic_frac_of_hbm_peak": round(traffic / rec["per_launch"] / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
    }
    valu_time = load_valu_time(w.name)
    if valu_time:
        out["valu_busy_frac_at_2.4GHz"] = round(valu_time / rec["per_launch"], 4)
    return out


def sweep_roofline(w, rec):
    """The HBM roofline of the per-step bytes model while it bounds the kernel
    (frac <= 1); a kernel that performs enough steps per launch to run past it
    is reported against the ALU roofline instead."""
    roof = hbm_roofline(w, rec)
    return roof if roof["frac"] <= 1.0 else alu_roofline(w, rec)


def alu_roofline(w, rec):
    """ALU roofline of a temporally blocked sweep (several steps per launch, the
    intermediate levels kept on chip): algorithmic flops per launch (collision_flops
    per node and step) over the measured launch duration, against the FP32 (FP64)
    vector peak without packed instructions; the launch's HBM traffic and the
    measured VALU issue fraction come from committed counter profiles."""
    m, q = w.N - 1, Q[w.lattice]
    flops = collision_flops(m, q) * w.nodes * rec["steps_per_pass"]
    achieved = flops / rec["per_launch"] / 1e12
    peak = ALU_PEAK_F32_TFLOPS if w.precision == "f32" else ALU_PEAK_F64_TFLOPS
    traffic = load_traffic(w.name)
    valu_time = load_valu_time(w.name)
    try:
        valu_busy_clock = float(load_profile("valu", w.name)["valu_busy_frac_at_estimated_clock"])
        clock_ghz = float(load_profile("valu", w.name)["clock_estimate_GHz"])
    except (KeyError, ValueError):
        valu_busy_clock = clock_ghz = None
    return {
        "bound": "alu",
        "achieved": round(achieved, 2),
        "peak": round(peak, 2),
        "unit": "TFLOP/s",
        "frac": round(achieved / peak, 4),
        "traffic": traffic,
        "flops_per_node_update": collision_flops(m, q),
        "steps_per_launch": rec["steps_per_pass"],
        "ms_per_launch": round(rec["per_launch"] * 1e3, 5),
        "ms_per_launch_measured_over": rec["per_launch_over"],
        "traffic_GBps": round(traffic / rec["per_launch"] / 1e9, 1) if traffic else None,
        "traffic_frac_of_hbm_peak": round(traffic / rec["per_launch"] / 1e9 / HBM_PEAK_GBS, 4) if traffic else None,
        "valu_busy_frac_at_2.4GHz": round(valu_time / rec["per_launch"], 4) if valu_time else None,
        "valu_busy_frac_at_clock_under_load": valu_busy_clock,
        "clock_under_load_GHz": clock_ghz,
    }


def batched_extra(steps: int = 1000, warmup: int = 5):
    """256-mixture workload under the tuned batch schedule (graph replay of full
    passes) against two references on the same stream and device: each mixture
    as its own single-mixture handle with the default launch, and one launch of
    the single-step sweep per mixture and step."""
    import tempfile

    import torch

    import workloads
    from paper_1808_06787_amd import autotune
    from paper_1808_06787_amd.batch import Batch

    ws = workloads.batched_2d(steps=steps)
    specs = [dict(D=w.D, shape=w.shape, bc=w.bc) for w in ws]
    b = Batch(specs, "D2Q5", "f32")
    for i, w in enumerate(ws):
        b.init(i, torch.from_numpy(w.xi0))
    b.release_inputs()
    upd = sum(w.nodes * (w.N - 1) for w in ws)
    byt = sum(w.nodes * (w.N - 1) * 2 * 5 * 4 for w in ws)
    del ws
    cache = os.path.join(tempfile.gettempdir(), "msd_autotune.json")
    tune = autotune.tune_batch(b, cache_path=cache, steps=30, warmup=2)
    state, t0 = b.save()

    def timed(fn):
        fn(warmup)
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        start.record(b.stream)
        fn(steps)
        stop.record(b.stream)
        torch.cuda.synchronize()
        return start.elapsed_time(stop) / 1e3

    t_fused = timed(b.step)
    b.restore(state, t0)
    t_each = timed(b.step_each)
    b.restore(state, t0)
    t_sep = timed(b.step_separate)
    sched = b.get_schedule()
    b.close()
    return {
        "mixtures": 256, "steps": steps, "node_component_updates_per_step": upd,
        "MLUPS_batched": round(upd * steps / t_fused / 1e6, 1),
        "MLUPS_separate_handles": round(upd * steps / t_sep / 1e6, 1),
        "MLUPS_one_single_step_launch_per_mixture": round(upd * steps / t_each / 1e6, 1),
        "speedup_vs_separate_handles": round(t_sep / t_fused, 3),
        "speedup_vs_one_single_step_launch_per_mixture": round(t_each / t_fused, 3),
        "ms_per_step_batched": round(t_fused / steps * 1e3, 4),
        "ms_per_step_separate_handles": round(t_sep / steps * 1e3, 4),
        "ms_per_step_one_single_step_launch_per_mixture": round(t_each / steps * 1e3, 4),
        "GB_per_s_batched": round(byt * steps / t_fused / 1e9, 1),
        "schedule": sched,
        "baselines": "separate handles: each mixture stepped as its own single-mixture handle with the default "
                     "launch (its own plan: blocked passes where the plan takes them); one single-step launch per "
                     "mixture and step: the single-step sweep only",
    }


def adjoint_extra(precisions=("f32", "f64"), fd_check=True):
    """Gradient workload: 1024^2 ternary D2Q5, 2000 steps, checkpoints every 100.
    Per precision: time of the plain forward run (default launch, and one step per
    pass), of the checkpointed forward run and of the backward pass (recompute +
    adjoint).  FP64 (with fd_check): the adjoint gradients against central
    differences (h = 1e-4) for the three D_ij pairs and one direction of the
    initial field."""
    import torch

    import workloads
    from paper_1808_06787_amd import adjoint
    from paper_1808_06787_amd.sim import Sim

    w = workloads.adjoint_2d()
    every = w.meta["checkpoint_every"]
    N = w.N

    def run(D, prec, x0, steps):
        s = Sim(w.lattice, D, w.shape, prec, bc=w.bc)
        s.init(torch.from_numpy(x0))
        s.step(steps)
        return s

    ts = run(w.meta["D_target"], "f64", w.xi0, w.steps)
    target = ts.read(torch.float64, flux=False, grad=False)[0]
    ts.close()

    def events(fn):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        out = fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / 1e3, out

    res = {"extents": list(w.shape), "steps": w.steps, "checkpoint_every": every}
    for prec in precisions:
        s = Sim(w.lattice, w.D, w.shape, prec, bc=w.bc)
        s.init(torch.from_numpy(w.xi0))             # warm-up of every kernel used below
        ck = adjoint.forward_with_checkpoints(s, 5, 2)
        xi = s.read(torch.float64, flux=False, grad=False)[0]
        adjoint.gradients(s, ck, 5, 2.0 * (xi - target), 2)
        del ck
        s.init(torch.from_numpy(w.xi0))
        t_plain, _ = events(lambda: s.step(w.steps))
        launch = s.get_launch()
        s.set_launch(temporal=0)
        s.init(torch.from_numpy(w.xi0))
        t_plain1, _ = events(lambda: s.step(w.steps))
        s.set_launch(temporal=launch["temporal"])
        s.init(torch.from_numpy(w.xi0))
        t_fwd, ck = events(lambda: adjoint.forward_with_checkpoints(s, w.steps, every))
        xi = s.read(torch.float64, flux=False, grad=False)[0]
        L = float(((xi - target) ** 2).sum())
        t_bwd, (gx, gD) = events(lambda: adjoint.gradients(s, ck, w.steps, 2.0 * (xi - target), every))
        s.close()
        del ck
        res[prec] = {"loss": L, "forward_s": round(t_plain, 4), "forward_checkpointed_s": round(t_fwd, 4),
                     "backward_s": round(t_bwd, 4), "backward_over_forward": round(t_bwd / t_plain, 3),
                     "forward_one_step_per_pass_s": round(t_plain1, 4),
                     "backward_over_forward_one_step_per_pass": round(t_bwd / t_plain1, 3)}
        if prec == "f64" and fd_check:
            h = 1e-4

            def loss(D, x0):
                s2 = run(D, "f64", x0, w.steps)
                v = float(((s2.read(torch.float64, flux=False, grad=False)[0] - target) ** 2).sum())
                s2.close()
                return v

            worst = 0.0
            fd_pairs = {}
            for i in range(N):
                for j in range(i + 1, N):
                    Dp, Dm = w.D.copy(), w.D.copy()
                    Dp[i, j] = Dp[j, i] = w.D[i, j] + h
                    Dm[i, j] = Dm[j, i] = w.D[i, j] - h
                    fd = (loss(Dp, w.xi0) - loss(Dm, w.xi0)) / (2 * h)
                    fd_pairs[f"D{i + 1}{j + 1}"] = [fd, float(gD[i, j])]
                    worst = max(worst, abs(fd - gD[i, j]) / abs(fd))
            v = w.meta["direction"]
            fd = (loss(w.D, w.xi0 + h * v) - loss(w.D, w.xi0 - h * v)) / (2 * h)
            ad = float((gx.cpu().numpy() * v[: N - 1]).sum())
            worst = max(worst, abs(fd - ad) / abs(fd))
            res["fd_check_f64"] = {"h": h, "pairs_fd_vs_adjoint": fd_pairs, "direction_fd_vs_adjoint": [fd, ad],
                                   "max_relative_difference": worst}
    return res


def host_cpu_info() -> dict:
    """Logical CPUs of this host and their model name (from /proc/cpuinfo)."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        usable = os.cpu_count()
    return {"logical_cpus": os.cpu_count(), "usable_cpus": usable, "model": model}


def cpu_baseline(w, budget_s=15.0):
    """The FP64 oracle (unchanged) on a bounded sub-grid of the workload, single thread."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    from oracle import lbm

    d = len(w.shape)
    cap = {1: 1 << 30, 2: 512, 3: 96}[d]
    sub = tuple(min(cap, n) for n in w.shape)
    sl = tuple(slice(0, n) for n in sub[::-1])
    xi0 = w.xi0[(slice(None),) + sl]
    xi0 = xi0 / xi0.sum(axis=0, keepdims=True)
    p = lbm.Problem(w.lattice, w.D, sub, bc=w.bc)
    ctx = threadpool_limits(1) if threadpool_limits else None
    try:
        f = lbm.init(p, xi0)
        f = lbm.step(p, f)        # warm-up
        t0 = time.perf_counter()
        n = 0
        while time.perf_counter() - t0 < budget_s:
            f = lbm.step(p, f)
            n += 1
        dt = time.perf_counter() - t0
    finally:
        if ctx is not None:
            ctx.__exit__(None, None, None)
    nodes = int(np.prod(sub))
    return {
        "value": nodes * (w.N - 1) * n / dt / 1e6,
        "unit": "MLUPS",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{'x'.join(map(str, sub))} sub-grid of the same field, {n} steps, FP64 numpy, 1 thread",
        "host": host_cpu_info(),
    }


def lattice_extras(extras):
    """The lattices without a rest direction (Eqs. (3-6), (3-9)) and with diagonal
    directions (Eqs. (3-8), (3-11)) on the 2D and 3D inputs, each with its default
    launch (D2Q4: blocked passes of up to six steps; D3Q6: two steps per pass;
    D2Q9, D3Q15: one step per pass).  GB_per_s counts the per-step bytes model;
    with several steps per launch that exceeds the HBM traffic, and hbm_frac is
    then given as the model's fraction (model_bytes_frac) instead."""
    for name, base, lattice in (("ternary_2d_d2q4_4096^2_f32", "ternary_2d", "D2Q4"),
                                ("quaternary_3d_d3q6_512^3_f32", "quaternary_3d", "D3Q6"),
                                ("ternary_2d_d2q9_4096^2_f32", "ternary_2d", "D2Q9"),
                                ("quaternary_3d_d3q15_512^3_f32", "quaternary_3d", "D3Q15")):
        wr = _on_lattice(make_workload(base), lattice)
        n_steps = 500 if wr.lattice.startswith("D2") else 100
        rr, simr = measure(wr, n_steps, 5)
        simr.close()
        a = pass_bytes(wr) / rr["per_step"] / 1e9
        frac_key = "hbm_frac" if rr["steps_per_pass"] == 1 else "model_bytes_frac"
        extras[name] = {"MLUPS": round(rr["mlups"], 1), "ms_per_step": round(rr["per_step"] * 1e3, 4),
                        "steps": n_steps, "steps_per_launch": rr["steps_per_pass"], "GB_per_s": round(a, 1),
                        frac_key: round(a / HBM_PEAK_GBS, 4)}
        print(f"# {name}: {rr['mlups']:.0f} MLUPS, {a:.0f} GB/s of model bytes ({100 * a / HBM_PEAK_GBS:.1f}%; "
              f"{rr['steps_per_pass']} step(s) per launch)", file=sys.stderr, flush=True)
        del wr


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="quaternary_3d")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--block-x", type=int, default=0)
    ap.add_argument("--block-y", type=int, default=0)
    ap.add_argument("--nontemporal", type=int, default=0)
    ap.add_argument("--xcd-remap", type=int, default=None)
    ap.add_argument("--vec", type=int, default=0)
    ap.add_argument("--temporal", type=int, default=None,
                    help="steps per pass of the blocked sweep (0: one step per pass; default: library's)")
    ap.add_argument("--seg-rows", type=int, default=None,
                    help="rows (2D) or z-planes (3D) per workgroup of the blocked sweep (0: automatic)")
    ap.add_argument("--tile", type=int, nargs=2, default=None, metavar=("TX", "TY"),
                    help="output tile per workgroup of the 3D blocked sweep (0 0: automatic)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain copy kernel of this size first (calibrates HBM byte counters)")
    ap.add_argument("--only", choices=("adjoint", "batch"), default=None,
                    help="run only this extra (FP32 adjoint without the FD check, or the 256-mixture batch) "
                         "and print its JSON record; for profiling")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the sweep would shard by slabs with halo exchange; not implemented)", file=sys.stderr)
        raise SystemExit(2)
    import torch

    from paper_1808_06787_amd import lib

    lib()   # fail loudly if the HIP library is missing
    torch.cuda.set_device(0)
    if args.only:
        rec = adjoint_extra(precisions=("f32",), fd_check=False) if args.only == "adjoint" else batched_extra()
        print(json.dumps({"extra": args.only, **rec}), flush=True)
        return
    if args.copy_probe_mib:
        n = args.copy_probe_mib * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)          # reads and writes copy_probe_mib MiB once each
        torch.cuda.synchronize()
        print(f"# copy probe: {args.copy_probe_mib} MiB read + {args.copy_probe_mib} MiB written",
              file=sys.stderr, flush=True)
        del a, b
    w = make_workload(args.workload)
    steps = args.steps if args.steps is not None else w.steps
    launch = dict(block_x=args.block_x, block_y=args.block_y, xcd_remap=args.xcd_remap,
                  nontemporal=args.nontemporal, vec=args.vec, temporal=args.temporal, seg_rows=args.seg_rows,
                  tile_x=args.tile[0] if args.tile else None, tile_y=args.tile[1] if args.tile else None)
    print(f"# workload {w.name}: {w.lattice} N={w.N} shape={w.shape} {w.precision}; "
          f"warmup {args.warmup}, timing {steps} steps", file=sys.stderr, flush=True)
    rec, sim = measure(w, steps, args.warmup, launch)
    _, _, _, bad = sim.diagnostics(raise_on_diverged=False)
    sim.close()
    del sim
    roof = sweep_roofline(w, rec)
    out = {
        "metric": "MLUPS (node-component updates per second) of the fused collide-and-stream sweep",
        "value": round(rec["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(rec["per_step"] * 1e3, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.precision == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "lattice": w.lattice, "n_species": w.N, "extents": list(w.shape),
                   "faces": [list(b) for b in w.bc], "precision": w.precision, "launch": rec["launch"]},
        "roofline": roof,
        "nonfinite": bad,
    }
    print(f"# {w.name}: {rec['mlups']:.0f} MLUPS, {rec['per_step'] * 1e3:.4f} ms/step; roofline "
          f"{roof['bound']} {roof['achieved']} {roof['unit']} = {100 * roof['frac']:.1f}% of peak",
          file=sys.stderr, flush=True)
    extras = {}
    if not args.no_extras and args.workload == "quaternary_3d":
        w2 = make_workload("ternary_2d")
        r2, sim2 = measure(w2, w2.steps, 5)
        sim2.close()
        roof2 = sweep_roofline(w2, r2)
        extras["ternary_2d_d2q5_4096^2_f32"] = {
            "MLUPS": round(r2["mlups"], 1), "ms_per_step": round(r2["per_step"] * 1e3, 5), "steps": w2.steps,
            "launch": r2["launch"], "roofline": roof2}
        print(f"# {w2.name}: {r2['mlups']:.0f} MLUPS, {r2['per_step'] * 1e3:.4f} ms/step; roofline "
              f"{roof2['bound']} {roof2['achieved']} {roof2['unit']} = {100 * roof2['frac']:.1f}% of peak",
              file=sys.stderr, flush=True)
        del w2
        lattice_extras(extras)
        w1 = make_workload("ternary_1d")
        s1, sim1 = time_sweep(w1, w1.steps, 0)
        sim1.close()
        m1 = w1.nodes * (w1.N - 1) * w1.steps / s1 / 1e6
        extras["ternary_1d_d1q3_256_f64"] = {"MLUPS": round(m1, 2), "steps_per_s": round(w1.steps / s1, 1),
                                             "seconds": round(s1, 5)}
        print(f"# {w1.name}: {m1:.1f} MLUPS, {w1.steps / s1:.0f} steps/s", file=sys.stderr, flush=True)
        bx = batched_extra()
        extras["batched_256_mixtures_d2q5_f32"] = bx
        print(f"# batched: {bx['MLUPS_batched']:.0f} MLUPS vs {bx['MLUPS_separate_handles']:.0f} separate handles "
              f"({bx['speedup_vs_separate_handles']:.2f}x) and {bx['MLUPS_one_single_step_launch_per_mixture']:.0f} "
              f"single-step launches ({bx['speedup_vs_one_single_step_launch_per_mixture']:.2f}x)",
              file=sys.stderr, flush=True)
        ax = adjoint_extra()
        extras["adjoint_1024x1024_d2q5_ternary"] = ax
        print(f"# adjoint f32: backward/forward = {ax['f32']['backward_over_forward']:.2f}; FD check (f64) "
              f"max rel diff {ax['fd_check_f64']['max_relative_difference']:.2e}", file=sys.stderr, flush=True)
    if extras:
        out["extras"] = extras
    if not args.no_cpu_baseline:
        print("# timing the CPU oracle on a bounded sample ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
