"""Seeded synthetic inputs shared by the GPU library's callers and the oracle.

This package holds no arithmetic of the lattice Boltzmann method: only the
initial density fields of the test problems (a tanh droplet profile, a flat
slab, seeded jitter) and the parameter draws of the droplet sweeps.
"""
from .droplet import (  # noqa: F401
    splitmix64_uniform, droplet_rho, slab_rho, sweep_items,
)
