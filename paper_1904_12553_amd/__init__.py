"""MI355X (gfx950) implementation of the phase-field lattice Boltzmann model
for immiscible incompressible N-phase flows (Yuan, Liang, Chai & Shi,
arXiv:1904.12553).

The product is the C-ABI library ``libnplbm.so`` (include/nplbm.h) built from
``csrc/``; ``nplbm`` is its thin Python binding.
"""
from .nplbm import (Domain, Server, NplbmError, validate, accepts, footprint, device_copy,
                    make_params, lib, EXPORTS)

__all__ = ["Domain", "Server", "NplbmError", "validate", "accepts", "footprint",
           "device_copy", "make_params", "lib", "EXPORTS"]
