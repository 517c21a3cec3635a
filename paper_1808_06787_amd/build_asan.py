"""Host AddressSanitizer build of the library for the CPU tests of the C ABI.

    python -m paper_1808_06787_amd.build_asan
    MSD_LIBRARY=_build/asan/libmsd_asan.so \
    LD_PRELOAD=$(/opt/rocm/llvm/bin/clang -print-file-name=libclang_rt.asan-x86_64.so) \
    ASAN_OPTIONS=detect_leaks=0 python -m pytest tests/test_abi_cpu.py tests/test_stability_cpu.py

Only the host half of every translation unit is instrumented (each sanitizer
flag applies to the host compilation alone); the device code is built as
usual.  The result lives under _build/ and is never loaded by default.
"""
from __future__ import annotations

import os

from .build import ROOT, build

ASAN_DIR = os.path.join(ROOT, "_build", "asan")
ASAN_LIB = os.path.join(ASAN_DIR, "libmsd_asan.so")
HOST_ASAN = ("-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer")


def build_asan(verbose: bool = False) -> str:
    return build(verbose=verbose, build_dir=ASAN_DIR, lib=ASAN_LIB, extra=HOST_ASAN,
                 link_extra=("-Xarch_host", "-fsanitize=address"))


if __name__ == "__main__":
    build_asan(verbose=True)
