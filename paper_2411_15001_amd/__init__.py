"""MI355X (gfx950) implementation of the positive- and bound-preserving
blended D2Q5 vectorial lattice Boltzmann scheme for the 2D Euler equations.

The numerical work runs in libvlbm.so (hand-written HIP kernels behind the C
ABI of include/vlbm.h); this package holds the ctypes binding, owning
wrappers, the autograd rollout and the seeded input generators.
"""
from . import binding, cases  # noqa: F401
from .binding import *  # noqa: F401,F403

__all__ = ["binding", "cases"]
