"""MI355X library for one Runge-Kutta stage of the 2-D linearized Euler
equations with a normal-stencil ghost-point immersed boundary and a
mass-spring-damper ADE impedance wall.

The compute path is liblee.so (HIP kernels for gfx950 behind the C ABI of
include/lee.h); this package only marshals arguments.  The library is loaded
on first use (creating an Instance or Batch, or calling _lib.load()), which
fails loudly if it has not been built.  Importing the package does not load
it, so that the build module can run while an outdated library is present.
"""
from ._lib import LeeError
from .lee import Batch, Instance

__all__ = ["Instance", "Batch", "LeeError"]
