"""ctypes declarations of the C ABI in include/msd.h.

Loading fails loudly if the HIP library has not been built: there is no
fallback implementation of the sweep in Python.
"""
from __future__ import annotations

import ctypes as C
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
# MSD_LIBRARY selects another build of the same library (e.g. the host
# AddressSanitizer build of build_asan.py for the CPU tests of the C ABI)
LIB_PATH = os.environ.get("MSD_LIBRARY") or os.path.join(_PKG, "libmsd.so")

ABI_VERSION = 4
STATIC_SCRATCH_BYTES = 64 << 20   # MSD_STATIC_SCRATCH_BYTES
MAX_SPECIES = 8

D1Q3, D2Q5, D3Q7, D1Q2, D2Q4, D3Q6, D2Q9, D3Q15 = 1, 2, 3, 4, 5, 6, 7, 8
F32, F64 = 4, 8
RELAX_PAPER, RELAX_SRT, RELAX_TRT = 0, 1, 2
MAGIC_PAPER = 3.0 / 16.0
BC_PERIODIC, BC_ZERO_FLUX, BC_DIRICHLET = 0, 1, 2

OK = 0
STATUS = {
    0: "MSD_OK", -1: "MSD_EINVAL", -2: "MSD_EDIFF", -3: "MSD_ECOMP", -4: "MSD_ERELAX",
    -5: "MSD_EHIP", -6: "MSD_EDIVERGED", -7: "MSD_ENOMEM", -8: "MSD_EABI", -9: "MSD_ESTATE",
}


class MsdProblem(C.Structure):
    _fields_ = [
        ("abi", C.c_int32),
        ("lattice", C.c_int32),
        ("n_species", C.c_int32),
        ("precision", C.c_int32),
        ("nx", C.c_int64),
        ("ny", C.c_int64),
        ("nz", C.c_int64),
        ("D", C.POINTER(C.c_double)),
        ("xi_wall", C.POINTER(C.c_double)),
        ("xi_ref", C.POINTER(C.c_double)),
        ("c_t", C.c_double),
        ("relax", C.c_int32),
        ("linearized", C.c_int32),
        ("bc", C.c_int32 * 6),
        ("plane_pad", C.c_int32),
        ("dilute", C.c_int32),
        ("trt_magic", C.c_double),
    ]


class MsdLaunch(C.Structure):
    _fields_ = [
        ("block_x", C.c_int32),
        ("block_y", C.c_int32),
        ("xcd_remap", C.c_int32),
        ("lds_resident", C.c_int32),
        ("nontemporal", C.c_int32),
        ("vec", C.c_int32),
        ("temporal", C.c_int32),
        ("seg_rows", C.c_int32),
        ("tile_x", C.c_int32),
        ("tile_y", C.c_int32),
    ]


class MsdSchedule(C.Structure):
    _fields_ = [
        ("block_x", C.c_int32),
        ("block_y", C.c_int32),
        ("mode", C.c_int32),
        ("order", C.c_int32),
        ("xcd_remap", C.c_int32),
        ("nontemporal", C.c_int32),
        ("temporal", C.c_int32),
        ("seg_rows", C.c_int32),
        ("graph", C.c_int32),
    ]


BATCH_FUSED, BATCH_PER_CLASS = 0, 1
TUNE_IGNORE_CACHE = 1
ORDER_INSTANCE, ORDER_INTERLEAVED = 0, 1


class MsdHealth(C.Structure):
    _fields_ = [
        ("neg_tol", C.c_double),
        ("mass_rtol", C.c_double),
    ]


class MsdError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        self.status = status
        super().__init__(f"{what}: {STATUS.get(status, status)} ({detail})")


_lib = None


def lib():
    """The loaded HIP library (raises if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"HIP library {LIB_PATH} is missing; build it with "
            "`python -m paper_1808_06787_amd.build` (no CPU fallback exists)"
        )
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
    P = C.POINTER
    sig = {
        "msd_abi_version": (C.c_int, []),
        "msd_last_error": (C.c_char_p, []),
        "msd_strerror": (C.c_char_p, [C.c_int]),
        "msd_workspace_bytes": (sz, [P(MsdProblem), P(i32)]),
        "msd_create": (C.c_int, [P(MsdProblem), vp, sz, vp, P(vp)]),
        "msd_set_stream": (C.c_int, [vp, vp]),
        "msd_set_launch": (C.c_int, [vp, P(MsdLaunch)]),
        "msd_get_launch": (C.c_int, [vp, P(MsdLaunch)]),
        "msd_steps_per_pass": (C.c_int, [vp]),
        "msd_init": (C.c_int, [vp, vp, i32]),
        "msd_step": (C.c_int, [vp, i64]),
        "msd_time": (i64, [vp]),
        "msd_read_moments": (C.c_int, [vp, i32, vp, vp, vp]),
        "msd_diagnostics": (C.c_int, [vp, P(C.c_double), P(C.c_double), P(C.c_double), P(i64)]),
        "msd_set_health": (C.c_int, [vp, P(MsdHealth)]),
        "msd_get_health": (C.c_int, [vp, P(MsdHealth)]),
        "msd_relaxation_radius": (C.c_int, [P(MsdProblem), P(C.c_double), i32, P(C.c_double)]),
        "msd_stability": (C.c_int, [vp, P(C.c_double), P(C.c_double)]),
        "msd_state_bytes": (sz, [vp]),
        "msd_save": (C.c_int, [vp, vp, P(i64)]),
        "msd_restore": (C.c_int, [vp, vp, i64]),
        "msd_destroy": (C.c_int, [vp]),
        "msd_record": (C.c_int, [vp, i64, vp]),
        "msd_adjoint_accum_bytes": (sz, [vp]),
        "msd_adjoint_begin": (C.c_int, [vp, vp]),
        "msd_adjoint_seed": (C.c_int, [vp, vp, vp]),
        "msd_adjoint_step": (C.c_int, [vp, i64, vp, vp, vp, vp]),
        "msd_adjoint_finish": (C.c_int, [vp, vp, vp, vp, P(C.c_double)]),
        "msd_adjoint_steps": (C.c_int, [vp, i64, i64, vp, vp, vp, vp, vp, P(i32)]),
        "msd_adjoint_scratch_bytes": (sz, [vp, i64]),
        "msd_forward_checkpointed": (C.c_int, [vp, i64, i64, vp]),
        "msd_adjoint": (C.c_int, [vp, i64, i64, vp, vp, vp, P(C.c_double), vp, sz]),
        "msd_adjoint_noalloc": (C.c_int, [vp, i64, i64, vp, vp, vp, P(C.c_double)]),
        "msd_batch_workspace_bytes": (sz, [P(MsdProblem), i32, P(i32)]),
        "msd_batch_create": (C.c_int, [P(MsdProblem), i32, vp, sz, vp, P(vp)]),
        "msd_batch_init": (C.c_int, [vp, i32, vp, i32]),
        "msd_batch_step": (C.c_int, [vp, i64]),
        "msd_batch_step_each": (C.c_int, [vp, i64]),
        "msd_batch_step_separate": (C.c_int, [vp, i64]),
        "msd_batch_time": (i64, [vp]),
        "msd_batch_read_moments": (C.c_int, [vp, i32, i32, vp, vp, vp]),
        "msd_batch_diagnostics": (C.c_int, [vp, i32, P(C.c_double), P(C.c_double), P(C.c_double), P(i64)]),
        "msd_batch_set_schedule": (C.c_int, [vp, P(MsdSchedule)]),
        "msd_batch_get_schedule": (C.c_int, [vp, P(MsdSchedule)]),
        "msd_batch_state_bytes": (sz, [vp]),
        "msd_batch_save": (C.c_int, [vp, vp, P(i64)]),
        "msd_batch_restore": (C.c_int, [vp, vp, i64]),
        "msd_batch_tiles": (i64, [vp]),
        "msd_batch_tune": (C.c_int, [vp, P(MsdSchedule), i32, i32, C.c_double, C.c_char_p, i32, vp, sz,
                                     P(MsdSchedule), P(C.c_double), P(C.c_double)]),
        "msd_tune": (C.c_int, [vp, P(MsdLaunch), i32, i32, C.c_double, C.c_char_p, i32, vp, sz, P(MsdLaunch),
                               P(C.c_double), P(C.c_double)]),
        "msd_batch_destroy": (C.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    if L.msd_abi_version() != ABI_VERSION:
        raise RuntimeError("libmsd ABI version mismatch; rebuild the library")
    _lib = L
    return L


def check(status: int, what: str) -> int:
    if status != OK:
        detail = lib().msd_last_error().decode(errors="replace")
        raise MsdError(status, what, detail)
    return status
