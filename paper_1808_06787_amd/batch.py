"""Python binding of a batch of independent mixtures (argument marshalling only).

All mixtures share lattice and precision; N, extents, D_ij, faces and
relaxation rule may differ.  `step` advances every mixture under the batch
schedule (a few launches per pass over all mixtures, replayed from a captured
HIP graph for long calls); the reference schedules run the mixtures one after
another: `step_each` with one launch of the single-step sweep per mixture and
step, `step_separate` exactly as separate single-mixture handles with their
default launches would.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _ffi as F
from .sim import DIMS, make_problem

MODES = {"fused": F.BATCH_FUSED, "per_class": F.BATCH_PER_CLASS}
ORDERS = {"instance": F.ORDER_INSTANCE, "interleaved": F.ORDER_INTERLEAVED}


class Batch:
    def __init__(self, specs, lattice: str = "D2Q5", precision: str = "f32", device=None, stream=None):
        """specs: list of dicts with keys D, shape and optionally bc, xi_wall, relax, c_t, xi_ref,
        trt_magic."""
        self.lib = F.lib()
        self.lattice = lattice
        self.precision = precision
        self.d = DIMS[lattice]
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.count = len(specs)
        arr = (F.MsdProblem * self.count)()
        self._keep = []
        self.shapes, self.N = [], []
        for i, sp in enumerate(specs):
            p, keep = make_problem(lattice, sp["D"], sp["shape"], precision, sp.get("bc"), sp.get("xi_wall"),
                                   sp.get("relax", "paper"), sp.get("c_t", 1.0), sp.get("xi_ref"),
                                   trt_magic=sp.get("trt_magic", F.MAGIC_PAPER), dilute=sp.get("dilute", False))
            arr[i] = p
            self._keep.append(keep)
            self.shapes.append(tuple(int(s) for s in sp["shape"]))
            self.N.append(p.n_species)
        self._problems = arr
        status = C.c_int32(0)
        nbytes = self.lib.msd_batch_workspace_bytes(arr, self.count, C.byref(status))
        F.check(status.value, "msd_batch_workspace_bytes")
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        F.check(self.lib.msd_batch_create(arr, self.count, C.c_void_p(self.workspace.data_ptr()), C.c_size_t(nbytes),
                                          C.c_void_p(self.stream.cuda_stream), C.byref(h)), "msd_batch_create")
        self._h = h
        self._xi0 = [None] * self.count

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.msd_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init(self, index: int, xi0):
        t = xi0 if isinstance(xi0, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(xi0))
        if t.dtype not in (torch.float32, torch.float64):
            t = t.to(torch.float64)
        t = t.to(self.device).contiguous()
        nodes = self.shapes[index][::-1]
        if tuple(t.shape[1:]) != nodes or t.shape[0] < self.N[index] - 1:
            raise ValueError(f"xi0 of mixture {index} has shape {tuple(t.shape)}, expected (N, {nodes})")
        prec = F.F64 if t.dtype == torch.float64 else F.F32
        self._xi0[index] = t
        F.check(self.lib.msd_batch_init(self._h, int(index), C.c_void_p(t.data_ptr()), prec), "msd_batch_init")

    def release_inputs(self):
        """Drop references to the initial fields (after the init kernels have run)."""
        torch.cuda.current_stream(self.device).synchronize()
        self._xi0 = [None] * self.count

    def step(self, n: int = 1):
        F.check(self.lib.msd_batch_step(self._h, int(n)), "msd_batch_step")

    def step_each(self, n: int = 1):
        F.check(self.lib.msd_batch_step_each(self._h, int(n)), "msd_batch_step_each")

    def step_separate(self, n: int = 1):
        F.check(self.lib.msd_batch_step_separate(self._h, int(n)), "msd_batch_step_separate")

    @property
    def time(self) -> int:
        return int(self.lib.msd_batch_time(self._h))

    @property
    def tiles(self) -> int:
        return int(self.lib.msd_batch_tiles(self._h))

    def read(self, index: int, dtype=torch.float64, flux=True, grad=True):
        N = self.N[index]
        nodes = self.shapes[index][::-1]
        prec = F.F64 if dtype == torch.float64 else F.F32
        xi = torch.empty((N,) + nodes, dtype=dtype, device=self.device)
        J = torch.empty((N - 1, self.d) + nodes, dtype=dtype, device=self.device) if flux else None
        g = torch.empty((N - 1, self.d) + nodes, dtype=dtype, device=self.device) if grad else None
        F.check(self.lib.msd_batch_read_moments(self._h, int(index), prec, C.c_void_p(xi.data_ptr()),
                                                C.c_void_p(J.data_ptr()) if J is not None else None,
                                                C.c_void_p(g.data_ptr()) if g is not None else None),
                "msd_batch_read_moments")
        return xi, J, g

    def diagnostics(self, index: int):
        N = self.N[index]
        mass, mn, mx = (C.c_double * N)(), (C.c_double * N)(), (C.c_double * N)()
        bad = C.c_int64(0)
        F.check(self.lib.msd_batch_diagnostics(self._h, int(index), mass, mn, mx, C.byref(bad)),
                "msd_batch_diagnostics")
        return np.array(mass[:]), np.array(mn[:]), np.array(mx[:]), int(bad.value)

    def set_schedule(self, **fields):
        """Change the named fields of the tile schedule (msd_schedule); the others
        keep their current values (the library defaults after creation)."""
        cur = self.get_schedule()
        unknown = set(fields) - set(cur)
        if unknown:
            raise TypeError(f"unknown schedule fields {sorted(unknown)}")
        cur.update({k: v for k, v in fields.items() if v is not None})
        s = F.MsdSchedule()
        s.block_x, s.block_y = int(cur["block_x"]), int(cur["block_y"])
        s.mode = MODES[cur["mode"]] if isinstance(cur["mode"], str) else int(cur["mode"])
        s.order = ORDERS[cur["order"]] if isinstance(cur["order"], str) else int(cur["order"])
        s.xcd_remap, s.nontemporal = int(cur["xcd_remap"]), int(cur["nontemporal"])
        s.temporal, s.seg_rows = int(cur["temporal"]), int(cur["seg_rows"])
        s.graph = int(cur["graph"])
        F.check(self.lib.msd_batch_set_schedule(self._h, C.byref(s)), "msd_batch_set_schedule")

    def get_schedule(self) -> dict:
        s = F.MsdSchedule()
        F.check(self.lib.msd_batch_get_schedule(self._h, C.byref(s)), "msd_batch_get_schedule")
        inv_m = {v: k for k, v in MODES.items()}
        inv_o = {v: k for k, v in ORDERS.items()}
        return dict(block_x=s.block_x, block_y=s.block_y, mode=inv_m[s.mode], order=inv_o[s.order],
                    xcd_remap=s.xcd_remap, nontemporal=s.nontemporal, temporal=s.temporal, seg_rows=s.seg_rows,
                    graph=s.graph)

    def state_bytes(self) -> int:
        return int(self.lib.msd_batch_state_bytes(self._h))

    def save(self, out=None):
        if out is None:
            out = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        step = C.c_int64(0)
        F.check(self.lib.msd_batch_save(self._h, C.c_void_p(out.data_ptr()), C.byref(step)), "msd_batch_save")
        return out, int(step.value)

    def restore(self, state, step: int):
        F.check(self.lib.msd_batch_restore(self._h, C.c_void_p(state.data_ptr()), int(step)), "msd_batch_restore")
