"""MI355X-native ternary electrohydrodynamic lattice Boltzmann (HIP for gfx950).

The hot path lives in libehdlb.so (C ABI in include/ehdlb.h); this package only
marshals arguments to it.
"""
from . import _lib  # noqa: F401
from .sim import Context, Simulation  # noqa: F401
