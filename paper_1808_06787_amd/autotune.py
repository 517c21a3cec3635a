"""Autotuning by measurement: argument marshalling around msd_tune and
msd_batch_tune.

`tune_batch` picks the tile schedule of a Batch (tile shape, fused or per-N
launches, tile order, XCD remapping, steps per pass and segment height);
`tune_sim` picks the launch of a single Sim (tile shape, vector width, XCD
remapping, streaming hints, steps per pass and segment height).  The library
times each candidate (one warm-up step, then `steps` steps between HIP events)
from a saved state and restores state and time afterwards, so tuning does not
change the simulation.  Results are cached in a text file keyed by GPU
architecture, lattice, precision and problem sizes.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import torch

from . import _ffi as F
from .batch import MODES, ORDERS

LAUNCH_FIELDS = ("block_x", "block_y", "xcd_remap", "lds_resident", "nontemporal", "vec", "temporal", "seg_rows",
                 "tile_x", "tile_y")
MAX_LIBRARY_CANDIDATES = 256


def _schedule_struct(batch, cand: dict) -> F.MsdSchedule:
    cur = batch.get_schedule()
    cur.update(cand)
    s = F.MsdSchedule()
    s.block_x, s.block_y = int(cur["block_x"]), int(cur["block_y"])
    s.mode = MODES[cur["mode"]] if isinstance(cur["mode"], str) else int(cur["mode"])
    s.order = ORDERS[cur["order"]] if isinstance(cur["order"], str) else int(cur["order"])
    s.xcd_remap, s.nontemporal = int(cur["xcd_remap"]), int(cur["nontemporal"])
    s.temporal, s.seg_rows = int(cur["temporal"]), int(cur["seg_rows"])
    s.graph = int(cur["graph"])
    return s


def _schedule_dict(s: F.MsdSchedule) -> dict:
    inv_m = {v: k for k, v in MODES.items()}
    inv_o = {v: k for k, v in ORDERS.items()}
    return dict(block_x=s.block_x, block_y=s.block_y, mode=inv_m[s.mode], order=inv_o[s.order],
                xcd_remap=s.xcd_remap, nontemporal=s.nontemporal, temporal=s.temporal, seg_rows=s.seg_rows,
                graph=s.graph)


def _launch_struct(sim, cand: dict) -> F.MsdLaunch:
    cur = sim.get_launch()
    cur.update(cand)
    l = F.MsdLaunch()
    for k in LAUNCH_FIELDS:
        setattr(l, k, int(cur[k]))
    return l


def _launch_dict(l: F.MsdLaunch) -> dict:
    return {k: getattr(l, k) for k in LAUNCH_FIELDS}


def _run(fn, handle, struct_t, to_dict, cands, steps, budget_ms, cache_path, force, scratch, what):
    n = len(cands)
    arr = (struct_t * n)(*cands) if n else None
    times = (C.c_double * (n if n else MAX_LIBRARY_CANDIDATES))()
    for i in range(len(times)):
        times[i] = -1.0
    best = struct_t()
    ms = C.c_double(0.0)
    path = cache_path.encode() if cache_path else None
    F.check(fn(handle, arr, n, int(steps), float(budget_ms), path, F.TUNE_IGNORE_CACHE if force else 0,
               C.c_void_p(scratch.data_ptr()), C.c_size_t(scratch.numel()), C.byref(best), C.byref(ms), times), what)
    trials = []
    for i, t in enumerate(times):
        if t >= 0:
            trials.append(dict(candidate=to_dict(arr[i]) if n else i, seconds_per_step=t / 1e3))
    return dict(best=to_dict(best), seconds_per_step=ms.value / 1e3, trials=trials)


def tune_batch(batch, cache_path: Optional[str] = None, steps: int = 8, warmup: int = 1, candidates=None,
               force: bool = False, budget_ms: float = 0.0) -> dict:
    """Choose and apply the fastest schedule (candidates: partial schedule dicts, or
    None for the library's list).  Returns {'best': schedule, 'seconds_per_step': t,
    'trials': [...]} (no trials on a cache hit).  The library runs one warm-up step
    per candidate; `warmup` is accepted for compatibility."""
    cands = [_schedule_struct(batch, c) for c in candidates] if candidates else []
    scratch = torch.empty(max(batch.state_bytes(), 1), dtype=torch.uint8, device=batch.device)
    return _run(batch.lib.msd_batch_tune, batch._h, F.MsdSchedule, _schedule_dict, cands, steps, budget_ms,
                cache_path, force, scratch, "msd_batch_tune")


def tune_sim(sim, cache_path: Optional[str] = None, steps: int = 10, warmup: int = 1, candidates=None,
             force: bool = False, budget_ms: float = 0.0) -> dict:
    """Choose and apply the fastest launch of the single-mixture sweep (candidates:
    partial launch dicts, or None for the library's list)."""
    cands = [_launch_struct(sim, c) for c in candidates] if candidates else []
    scratch = torch.empty(max(sim.state_bytes(), 1), dtype=torch.uint8, device=sim.device)
    return _run(sim.lib.msd_tune, sim._h, F.MsdLaunch, _launch_dict, cands, steps, budget_ms, cache_path, force,
                scratch, "msd_tune")
