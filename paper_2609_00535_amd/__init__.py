"""MI355X-native two-phase spectral-element lattice Boltzmann time step.

The compute path is ``libsemlbm.so`` (HIP kernels for gfx950 behind the C ABI of
``include/semlbm.h``); this package is its Python binding.
"""
from .binding import (SIGNATURES, Batch, Server, SLBMError, Solve, lib,  # noqa: F401
                      make_params, wall_geom)

__all__ = ["Solve", "Batch", "Server", "SLBMError", "lib", "SIGNATURES"]
