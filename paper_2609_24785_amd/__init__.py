"""MI355X library for one Runge-Kutta stage of the 2-D linearized Euler
equations with a normal-stencil ghost-point immersed boundary and a
mass-spring-damper ADE impedance wall.

The compute path is liblee.so (HIP kernels for gfx950 behind the C ABI of
include/lee.h); this package only marshals arguments.  Importing it loads the
library and fails loudly if it has not been built.
"""
from ._lib import LeeError, load as _load

_load()

from .lee import Batch, Instance  # noqa: E402

__all__ = ["Instance", "Batch", "LeeError"]
