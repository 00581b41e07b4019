"""MI355X-native simulated bifurcation (bSB, dSB, GbSB, GdSB) for the Ising problem.

The compute path is libgsb.so (hand-written gfx950 HIP kernels behind the C ABI of
include/gsb.h); ``gsb`` is its ctypes binding and ``instances`` the seeded synthetic
instance generators.  Importing the package does not load the library; the first call
does, and fails loudly if it has not been built.
"""
from . import instances  # noqa: F401
from .gsb import *  # noqa: F401,F403
from .gsb import GSB, GsbError, load_library  # noqa: F401

__version__ = "0.1"
