"""MI355X (gfx950) lattice Boltzmann solver for Maxwell-Stefan diffusion in
N-component mixtures (Chai, Guo, Wang & Shi, MRT lattice Boltzmann model).

The method runs in the HIP library ``libmsd.so`` behind the C ABI of
``include/msd.h``; this package is its Python binding (argument marshalling,
device memory and streams from PyTorch).  Importing it does not touch the GPU.
"""
from ._ffi import LIB_PATH, MsdError, lib  # noqa: F401

__all__ = ["LIB_PATH", "MsdError", "lib", "Sim"]


def __getattr__(name):
    if name == "Sim":
        from .sim import Sim

        return Sim
    raise AttributeError(name)
