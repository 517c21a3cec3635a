"""Autotuning of launch parameters by timing candidates on the real problem.

`tune_batch` picks the tile schedule of a Batch (tile shape, fused or per-N
launches, tile order, XCD remapping); `tune_sim` picks the launch of a single
Sim (tile shape, vector width, XCD remapping, streaming hints).  Each candidate
runs a few steps from a saved state, timed with HIP events on the handle's
stream; the state and the time are restored afterwards, so tuning does not
change the simulation.  Results are cached in a JSON file keyed by GPU
architecture, lattice, precision and problem sizes.
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
from typing import Optional

import torch

BATCH_BLOCKS = [(64, 4), (128, 2), (256, 1), (64, 2), (64, 1)]
SIM_BLOCKS = [(256, 1), (128, 2), (64, 4), (128, 1), (64, 1)]


def _arch() -> str:
    try:
        return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def _load(path):
    if path and os.path.exists(path):
        try:
            with open(path) as fh:
                return json.load(fh)
        except (OSError, ValueError):
            return {}
    return {}


def _store(path, cache):
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _time(stream, fn, steps):
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record(stream)
    fn(steps)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / 1e3 / steps


def batch_key(batch) -> str:
    sizes = sorted((n, s) for n, s in zip(batch.N, batch.shapes))
    h = hashlib.sha256(repr(sizes).encode()).hexdigest()[:16]
    return f"{_arch()}|batch|{batch.lattice}|{batch.precision}|{batch.count}|{h}"


def tune_batch(batch, cache_path: Optional[str] = None, steps: int = 8, warmup: int = 2, candidates=None,
               force: bool = False) -> dict:
    """Choose and apply the fastest schedule; returns {'best': schedule, 'seconds_per_step': t, 'trials': [...]}."""
    cache = _load(cache_path)
    key = batch_key(batch)
    if not force and key in cache:
        batch.set_schedule(**cache[key]["best"])
        return cache[key]
    if candidates is None:
        candidates = [dict(block_x=bx, block_y=by, mode=mode, order=order, xcd_remap=xcd, temporal=0)
                      for (bx, by), mode, order, xcd in itertools.product(
                          BATCH_BLOCKS, ("fused", "per_class"), ("instance", "interleaved"), (0, 1))]
        if batch.lattice == "D2Q5":
            candidates += [dict(block_x=64, block_y=4, mode="per_class", order=order, temporal=tb, seg_rows=seg)
                           for tb, seg, order in itertools.product((2, 3, 4), (8, 16, 32), ("instance", "interleaved"))]
    state, t0 = batch.save()
    trials = []
    for cand in candidates:
        batch.set_schedule(**cand)
        batch.step(warmup)
        sec = _time(batch.stream, batch.step, steps)
        batch.restore(state, t0)
        trials.append(dict(schedule=cand, seconds_per_step=sec))
    best = min(trials, key=lambda r: r["seconds_per_step"])
    batch.set_schedule(**best["schedule"])
    out = dict(best=best["schedule"], seconds_per_step=best["seconds_per_step"], trials=trials)
    cache[key] = out
    _store(cache_path, cache)
    del state
    return out


def sim_key(sim) -> str:
    return f"{_arch()}|sim|{sim.lattice}|{sim.precision}|N{sim.N}|{'x'.join(map(str, sim.shape))}"


def tune_sim(sim, cache_path: Optional[str] = None, steps: int = 10, warmup: int = 2, candidates=None,
             force: bool = False) -> dict:
    """Choose and apply the fastest launch of the single-mixture sweep."""
    cache = _load(cache_path)
    key = sim_key(sim)
    if not force and key in cache:
        sim.set_launch(**cache[key]["best"])
        return cache[key]
    if candidates is None:
        candidates = [dict(block_x=bx, block_y=by, vec=vec, xcd_remap=xcd, nontemporal=nt, temporal=0)
                      for (bx, by), vec, xcd, nt in itertools.product(SIM_BLOCKS, (0, 1, 4), (0, 1), (0, 7))]
        if sim.lattice == "D2Q5":
            candidates += [dict(temporal=tb, seg_rows=seg, nontemporal=nt)
                           for tb, seg, nt in itertools.product((2, 3, 4), (16, 32, 64), (0, 1))]
    state, t0 = sim.save()
    trials = []
    for cand in candidates:
        sim.set_launch(**cand)
        sim.step(warmup)
        sec = _time(sim.stream, sim.step, steps)
        sim.restore(state, t0)
        trials.append(dict(launch=cand, seconds_per_step=sec))
    best = min(trials, key=lambda r: r["seconds_per_step"])
    sim.set_launch(**best["launch"])
    out = dict(best=best["launch"], seconds_per_step=best["seconds_per_step"], trials=trials)
    cache[key] = out
    _store(cache_path, cache)
    del state
    return out
