"""MI355X (gfx950) library for the D3Q19 non-orthogonal MRT lattice Boltzmann
step with the pseudopotential multiphase force (arXiv:1805.08643).

The compute path is the HIP library ``lib/libmrtlbm.so`` (C ABI in
``include/mrt_lbm.h``); ``binding`` is its ctypes binding.
"""
from .binding import Lattice, lib, make_params  # noqa: F401
