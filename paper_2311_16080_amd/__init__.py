"""MI355X-native lattice Boltzmann stream-collide hot path.

The compute path is the HIP library ``liblbm.so`` (C-ABI declared in
``include/lbm.h``); :mod:`paper_2311_16080_amd.lbm` is its Python binding.
Importing this package does no work and loads nothing.
"""
__all__ = ["lbm", "inputs"]
