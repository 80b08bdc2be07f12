"""libxfdtd for MI355X: the extended-Faraday-stencil Yee FDTD step
(Blinne et al., arXiv:1710.06829) as hand-written HIP kernels for gfx950,
behind the C interface of include/xfdtd.h.

The Python layer only marshals arguments; importing a GPU entry point without
the built library raises ImportError (there is no CPU fallback).
"""
from ._binding import XfdtdError, lib  # noqa: F401
from .solver import Solver, cfl_limit, consistent_alpha, dispersion  # noqa: F401
from .autograd import propagate  # noqa: F401
from .batch import Batch  # noqa: F401
from .norm import Family, dispersion_norm, optimize_stencil  # noqa: F401

__all__ = ["Batch", "Family", "Solver", "cfl_limit", "consistent_alpha", "dispersion", "dispersion_norm",
           "optimize_stencil", "propagate", "XfdtdError", "lib"]
