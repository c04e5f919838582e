"""MI355X-native relativistic lattice Boltzmann step (arXiv:1608.03004).

The product path is the HIP library ``librlb.so`` behind the C interface in
``include/rlb.h``; ``rlb`` is its Python binding.
"""
from .rlb import Box, BoxSpec, Lattice, Plane, PlaneSpec, Tube, RLBError, load_library  # noqa: F401
