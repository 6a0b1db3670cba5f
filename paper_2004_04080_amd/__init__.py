"""MI355X (gfx950) implementation of the LBsoft two-fluid + colloid
lattice-Boltzmann step (Bonaccorso et al., arXiv 2004.04080).

The computation lives in liblbhip.so (HIP kernels behind the C interface of
include/lbhip.h); this package is the thin Python front end.
"""
from .binding import LBError, lib  # noqa: F401
from .lattice import Lattice, Observables, Params, lattice, required_sizes  # noqa: F401

__all__ = ["Lattice", "Observables", "Params", "LBError", "lattice", "required_sizes", "lib"]
