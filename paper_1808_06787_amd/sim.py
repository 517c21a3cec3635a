"""Python binding of one mixture: argument marshalling around the C ABI.

PyTorch provides the device workspace and the HIP stream; every step of the
method runs in the HIP library.  Arrays follow the library's conventions:
fields are (N, nz, ny, nx) / (N, ny, nx) / (N, nx) with x fastest, fluxes and
gradients (N-1, d, ...), all in lattice units.
"""
from __future__ import annotations

import ctypes as C
import warnings
from typing import Optional, Sequence

import numpy as np
import torch

from . import _ffi as F

LATTICES = {"D1Q3": F.D1Q3, "D2Q5": F.D2Q5, "D3Q7": F.D3Q7, "D1Q2": F.D1Q2, "D2Q4": F.D2Q4, "D3Q6": F.D3Q6,
            "D2Q9": F.D2Q9, "D3Q15": F.D3Q15}
DIMS = {"D1Q3": 1, "D2Q5": 2, "D3Q7": 3, "D1Q2": 1, "D2Q4": 2, "D3Q6": 3, "D2Q9": 2, "D3Q15": 3}
PRECISIONS = {"f32": F.F32, "f64": F.F64}
RELAX = {"paper": F.RELAX_PAPER, "srt": F.RELAX_SRT, "trt": F.RELAX_TRT}
BCS = {"periodic": F.BC_PERIODIC, "zero_flux": F.BC_ZERO_FLUX, "dirichlet": F.BC_DIRICHLET}
TORCH_DTYPES = {F.F32: torch.float32, F.F64: torch.float64}


def _dptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def make_problem(lattice: str, D, shape: Sequence[int], precision: str = "f32", bc=None, xi_wall=None,
                 relax: str = "paper", c_t: float = 1.0, xi_ref=None, plane_pad: int = 0,
                 trt_magic: float = F.MAGIC_PAPER, dilute: bool = False):
    """Build an msd_problem plus the host arrays it points to (kept alive by the caller).

    bc: per axis (low, high) names from BCS; xi_wall: {(axis, side): (N,) values};
    relax: "paper" (Eq. (3-16)), "srt" or "trt" (even parameter from the product
    rule with trt_magic; "paper" is the trt_magic = 3/16 case); dilute: B of the
    dilute-species approximation (Remark III) instead of Eq. (2-10).
    """
    d = DIMS[lattice]
    shape = tuple(int(s) for s in shape)
    if len(shape) != d:
        raise ValueError(f"{lattice} needs {d} extents, got {shape}")
    Dm = np.ascontiguousarray(np.asarray(D, dtype=np.float64))
    N = Dm.shape[0]
    p = F.MsdProblem()
    p.abi = F.ABI_VERSION
    p.lattice = LATTICES[lattice]
    p.n_species = N
    p.precision = PRECISIONS[precision]
    ext = list(shape) + [1] * (3 - d)
    p.nx, p.ny, p.nz = ext
    keep = [Dm]
    p.D = Dm.ctypes.data_as(C.POINTER(C.c_double))
    faces = [F.BC_PERIODIC] * 6
    if bc is not None:
        for a, (lo, hi) in enumerate(bc):
            faces[2 * a] = BCS[lo]
            faces[2 * a + 1] = BCS[hi]
    for f in range(6):
        p.bc[f] = faces[f]
    if xi_wall:
        W = np.zeros((6, N))
        for (a, s), v in xi_wall.items():
            W[2 * a + s] = np.asarray(v, dtype=np.float64)
        keep.append(W)
        p.xi_wall = W.ctypes.data_as(C.POINTER(C.c_double))
    if xi_ref is not None:
        R = np.ascontiguousarray(np.asarray(xi_ref, dtype=np.float64))
        keep.append(R)
        p.xi_ref = R.ctypes.data_as(C.POINTER(C.c_double))
        p.linearized = 1
    p.c_t = float(c_t)
    p.relax = RELAX[relax]
    p.trt_magic = float(trt_magic)
    p.plane_pad = int(plane_pad)
    p.dilute = 1 if dilute else 0
    return p, keep


def relaxation_radius(lattice: str, D, compositions, relax: str = "paper", trt_magic: float = F.MAGIC_PAPER,
                      dilute: bool = False, xi_ref=None):
    """Spectral radii of I - Lambda_1 and I - Lambda_2 (msd_relaxation_radius) at each of
    the given compositions (array (count, N)); host computation, no device.  Returns
    an array (count, 2)."""
    Dm = np.asarray(D, dtype=np.float64)
    N = Dm.shape[0]
    shape = (1,) * DIMS[lattice]
    p, keep = make_problem(lattice, Dm, shape, "f64", relax=relax, trt_magic=trt_magic, dilute=dilute,
                           xi_ref=xi_ref)
    xi = np.ascontiguousarray(np.asarray(compositions, dtype=np.float64).reshape(-1, N))
    out = np.zeros((xi.shape[0], 2))
    F.check(F.lib().msd_relaxation_radius(C.byref(p), xi.ctypes.data_as(C.POINTER(C.c_double)), xi.shape[0],
                                          out.ctypes.data_as(C.POINTER(C.c_double))), "msd_relaxation_radius")
    return out


class Sim:
    """One mixture on one lattice, evolved by the HIP sweep."""

    def __init__(self, lattice: str, D, shape, precision: str = "f32", bc=None, xi_wall=None,
                 relax: str = "paper", c_t: float = 1.0, xi_ref=None, device=None, stream=None,
                 plane_pad: int = 0, trt_magic: float = F.MAGIC_PAPER, dilute: bool = False):
        self.lib = F.lib()
        self.lattice = lattice
        self.shape = tuple(int(s) for s in shape)
        self.d = DIMS[lattice]
        self.precision = precision
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.problem, self._keep = make_problem(lattice, D, shape, precision, bc, xi_wall, relax, c_t, xi_ref,
                                                plane_pad, trt_magic, dilute)
        self.N = self.problem.n_species
        self.m = self.N - 1
        status = C.c_int32(0)
        nbytes = self.lib.msd_workspace_bytes(C.byref(self.problem), C.byref(status))
        F.check(status.value, "msd_workspace_bytes")
        self.workspace = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        F.check(self.lib.msd_create(C.byref(self.problem), C.c_void_p(_dptr(self.workspace)), C.c_size_t(nbytes),
                                    C.c_void_p(self.stream.cuda_stream), C.byref(h)), "msd_create")
        self._h = h
        r1, r2 = self.stability()
        if r1 >= 1.0 or r2 >= 1.0:
            warnings.warn(f"relaxation does not damp every mode at some checked composition (spectral radii of "
                          f"I - Lambda_1, I - Lambda_2: {r1:.6f}, {r2:.6f}); the run may diverge", RuntimeWarning,
                          stacklevel=2)

    # -- lifetime ---------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.msd_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def nodes_shape(self):
        return self.shape[::-1]

    @property
    def dtype(self):
        return TORCH_DTYPES[PRECISIONS[self.precision]]

    # -- calls --------------------------------------------------------------------
    def set_launch(self, **fields):
        """Change the named fields of the launch configuration (msd_launch); the
        others keep their current values (the library defaults after creation)."""
        cur = self.get_launch()
        unknown = set(fields) - set(cur)
        if unknown:
            raise TypeError(f"unknown launch fields {sorted(unknown)}")
        cur.update({k: int(v) for k, v in fields.items() if v is not None})
        l = F.MsdLaunch()
        for k, v in cur.items():
            setattr(l, k, v)
        F.check(self.lib.msd_set_launch(self._h, C.byref(l)), "msd_set_launch")

    def get_launch(self) -> dict:
        l = F.MsdLaunch()
        F.check(self.lib.msd_get_launch(self._h, C.byref(l)), "msd_get_launch")
        return {k: getattr(l, k) for k in ("block_x", "block_y", "xcd_remap", "lds_resident", "nontemporal", "vec",
                                          "temporal", "seg_rows", "tile_x", "tile_y")}

    def steps_per_pass(self) -> int:
        """Time steps per launch of the sweep under the current launch configuration."""
        n = int(self.lib.msd_steps_per_pass(self._h))
        if n < 1:
            F.check(n, "msd_steps_per_pass")
        return n

    def init(self, xi0):
        """xi0: (N or N-1, *nodes) array or tensor; float32/float64."""
        t = xi0 if isinstance(xi0, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(xi0))
        if t.dtype not in (torch.float32, torch.float64):
            t = t.to(torch.float64)
        t = t.to(self.device).contiguous()
        if tuple(t.shape[1:]) != self.nodes_shape or t.shape[0] < self.m:
            raise ValueError(f"xi0 has shape {tuple(t.shape)}, expected (N, {self.nodes_shape})")
        prec = F.F64 if t.dtype == torch.float64 else F.F32
        self._xi0 = t            # keep alive until the init kernel has read it
        with torch.cuda.stream(self.stream):
            F.check(self.lib.msd_init(self._h, C.c_void_p(_dptr(t)), prec), "msd_init")
        t.record_stream(self.stream)

    def release_inputs(self):
        """Drop the reference to the initial field (after the init kernel has run)."""
        self.stream.synchronize()
        self._xi0 = None

    def step(self, n: int = 1):
        F.check(self.lib.msd_step(self._h, int(n)), "msd_step")

    @property
    def time(self) -> int:
        return int(self.lib.msd_time(self._h))

    def read(self, dtype=torch.float64, flux: bool = True, grad: bool = True):
        """Returns (xi (N, *nodes), J (m, d, *nodes) or None, grad (m, d, *nodes) or None)."""
        prec = F.F64 if dtype == torch.float64 else F.F32
        xi = torch.empty((self.N,) + self.nodes_shape, dtype=dtype, device=self.device)
        J = torch.empty((self.m, self.d) + self.nodes_shape, dtype=dtype, device=self.device) if flux else None
        g = torch.empty((self.m, self.d) + self.nodes_shape, dtype=dtype, device=self.device) if grad else None
        F.check(self.lib.msd_read_moments(self._h, prec, C.c_void_p(_dptr(xi)),
                                          C.c_void_p(_dptr(J)) if J is not None else None,
                                          C.c_void_p(_dptr(g)) if g is not None else None), "msd_read_moments")
        return xi, J, g

    def diagnostics(self, raise_on_diverged: bool = True):
        """(mass (N,), min (N,), max (N,), nonfinite count); synchronises the stream."""
        mass = (C.c_double * self.N)()
        mn = (C.c_double * self.N)()
        mx = (C.c_double * self.N)()
        bad = C.c_int64(0)
        st = self.lib.msd_diagnostics(self._h, mass, mn, mx, C.byref(bad))
        if st != F.OK and (raise_on_diverged or st != -6):
            F.check(st, "msd_diagnostics")
        return np.array(mass[:]), np.array(mn[:]), np.array(mx[:]), int(bad.value)

    def set_health(self, neg_tol: Optional[float] = None, mass_rtol: Optional[float] = None):
        """Limits of the divergence checks of diagnostics() (negative: off)."""
        h = F.MsdHealth()
        F.check(self.lib.msd_get_health(self._h, C.byref(h)), "msd_get_health")
        if neg_tol is not None:
            h.neg_tol = float(neg_tol)
        if mass_rtol is not None:
            h.mass_rtol = float(mass_rtol)
        F.check(self.lib.msd_set_health(self._h, C.byref(h)), "msd_set_health")

    def stability(self):
        """(rho1, rho2): the largest spectral radii of I - Lambda_1 and I - Lambda_2 found
        at the compositions checked when the handle was created."""
        r1, r2 = C.c_double(0.0), C.c_double(0.0)
        F.check(self.lib.msd_stability(self._h, C.byref(r1), C.byref(r2)), "msd_stability")
        return float(r1.value), float(r2.value)

    def state_bytes(self) -> int:
        return int(self.lib.msd_state_bytes(self._h))

    def save(self, out: Optional[torch.Tensor] = None):
        """Copy the state into `out` (uint8 device tensor of state_bytes()); returns (out, time)."""
        if out is None:
            out = torch.empty(self.state_bytes(), dtype=torch.uint8, device=self.device)
        step = C.c_int64(0)
        F.check(self.lib.msd_save(self._h, C.c_void_p(_dptr(out)), C.byref(step)), "msd_save")
        return out, int(step.value)

    def restore(self, state: torch.Tensor, step: int):
        F.check(self.lib.msd_restore(self._h, C.c_void_p(_dptr(state)), int(step)), "msd_restore")
