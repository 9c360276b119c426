"""MI355X library for the coupled two-component Shan-Chen D3Q19 lattice Boltzmann /
Skalak capsule time step (Wouters, Aouane, Sega, Harting; arXiv:2007.15405).

The compute path is ``liblbm.so`` (HIP kernels for gfx950 behind the C ABI in
``include/lbm.h``); :class:`Sim` and :class:`Batch` are its ctypes binding.
"""
from . import lbm  # noqa: F401
from .lbm import Sim, Batch, Surrogate, LbmError, load_library, SIGNATURES, LIB_PATH, STORAGE  # noqa: F401
