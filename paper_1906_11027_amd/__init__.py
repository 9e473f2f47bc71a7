"""MI355X (gfx950) implementation of the Shan-Chen pseudo-potential lattice
Boltzmann hot path: psi(rho), the isotropic interaction force, Guo-forced
SRT/MRT collision and pull streaming on D2Q9 and D3Q19, with FP64 reductions.

The compute path is libsc_lbm.so (C ABI, include/sc_lbm.h); `sc_lbm` is its
ctypes binding.
"""
from . import sc_lbm  # noqa: F401
from .sc_lbm import Batch, Sim, batch_autotune  # noqa: F401
